"""Span-1 (uncompressed) data on the GPU: ring-pair segments whose planes sit on every
other image plane (pitch 2), up to the mMR's 121 segments and 4084 planes.

* Projector parity (1e-5 relative, forward and backward, with and without mult) against
  the FP64 oracle on span-1 geometries that run the strip gather (nz >= 32), the column
  gather (nz < 32) and mixed pitches; the GPU adjoint identity.
* K epochs of SPDHG+ with TV on a span-1 slab of the mMR (8 rings: 344 x 344 x 15 image,
  15 segments, 64 planes, 252 angles) against the oracle: image within 1e-3, objective
  within 1e-4.
* Full mMR span-1 (344 x 344 x 127, 344 x 252 x 4084): sampled forward rays of a subset
  at every radial bin, and a single-angle backprojection, against the oracle."""
import numpy as np
import pytest

import synth
from oracle import projector as OP
from oracle import spdhg as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_1808_07150_amd as lib
    lib.load_library()
    return lib


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def close(gpu, ref, tol=1e-5):
    gpu = np.asarray(gpu, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    rel = np.linalg.norm(gpu - ref) / np.linalg.norm(ref)
    mx = np.max(np.abs(gpu - ref)) / np.max(np.abs(ref))
    assert rel <= tol and mx <= tol, (rel, mx)


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


GEOMS = {
    # nz = 33 >= 32: the strip gather's pitch-2 instance, 13 segments
    "span1_tall": synth.slab_span1(rings=17, max_ring_diff=6, nxy=21, v=4.0, n_ang=8),
    # nz = 9: the column gather, ragged in-plane size
    "span1_thin": synth.Geometry(nx=19, ny=23, nz=9, vx=3.0, vy=2.5, vz=2.0, n_rad=31,
                                 d_rad=2.2, n_ang=10,
                                 **dict(zip(("seg_planes", "seg_tan", "seg_pitch"),
                                            synth.span1_segments(5, 4, 2.0, 60.0)))),
    # mixed pitches (a pitch-1 segment next to pitch-2 ones): the column gather
    "mixed": synth.Geometry(nx=16, ny=16, nz=35, vx=3.0, vy=3.0, vz=3.0, n_rad=20, d_rad=3.0,
                            n_ang=8, seg_planes=(35, 18, 17, 17),
                            seg_tan=(0.0, 0.0, 0.2, -0.2), seg_pitch=(1, 2, 2, 2)),
}


def _inputs(g, seed):
    rng = np.random.default_rng(seed)
    return (rng.uniform(0, 2, g.image_shape).astype(np.float32),
            rng.uniform(0.5, 1.5, g.sino_shape).astype(np.float32),
            rng.normal(size=g.sino_shape).astype(np.float32))


@pytest.mark.parametrize("name", list(GEOMS))
@pytest.mark.parametrize("m,subset", [(1, -1), (4, 1)])
def test_span1_projector_parity(P, name, m, subset):
    g = GEOMS[name]
    print(f"[span1] {name}: {g.n_seg} segments, {g.n_planes} planes, m={m} subset={subset}",
          flush=True)
    x, mult, y = _inputs(g, 3)
    ang = list(range(g.n_ang)) if subset < 0 else g.subset_angles(m, subset)
    ref = mult[ang] * OP.forward(g, x.astype(np.float64), ang)
    out = torch.empty(len(ang) * g.n_planes * g.n_rad, dtype=torch.float32, device="cuda:0")
    P.spdhg_project(g, m, subset, dev(mult), dev(x), out)
    close(out.cpu().numpy(), ref)
    ysub = y[ang]
    ref = OP.backward(g, ysub.astype(np.float64), ang)
    xo = torch.empty(g.image_shape, dtype=torch.float32, device="cuda:0")
    P.spdhg_backproject(g, m, subset, None, dev(ysub), xo)
    close(xo.cpu().numpy(), ref)
    ref = OP.backward(g, (mult[ang] * ysub).astype(np.float64), ang)
    P.spdhg_backproject(g, m, subset, dev(mult), dev(ysub), xo)
    close(xo.cpu().numpy(), ref)


@pytest.mark.parametrize("name", list(GEOMS))
def test_span1_gpu_adjoint(P, name):
    g = GEOMS[name]
    x, mult, y = _inputs(g, 4)
    ax = torch.empty(g.n_bins, dtype=torch.float32, device="cuda:0")
    aty = torch.empty(g.image_shape, dtype=torch.float32, device="cuda:0")
    P.spdhg_project(g, 1, -1, dev(mult), dev(x), ax)
    P.spdhg_backproject(g, 1, -1, dev(mult), dev(y), aty)
    lhs = float(np.dot(ax.cpu().numpy().astype(np.float64), y.ravel()))
    rhs = float(np.dot(x.ravel().astype(np.float64), aty.cpu().numpy().ravel()))
    assert abs(lhs - rhs) <= 1e-6 * max(abs(lhs), abs(rhs))


SLAB_SEED, SLAB_COUNTS, SLAB_M, SLAB_EPOCHS = 18081400, 3e6, 21, 2
SLAB_ALPHA = 0.1 * (1e5 / SLAB_COUNTS) ** 0.5


def test_span1_slab_tv_parity(P):
    g = synth.slab_span1()
    print(f"[span1] slab {g.nx}x{g.ny}x{g.nz}, {g.n_seg} segments, {g.n_planes} planes: "
          f"oracle {SLAB_EPOCHS} epochs", flush=True)
    d = synth.brain_problem(g, SLAB_SEED, SLAB_COUNTS)
    prob = S.Problem(g, d["b"], d["r"], d["mult"], n_subsets=SLAB_M, prior="tv",
                     alpha=SLAB_ALPHA, sampling="balanced", precond=True)
    st = S.spdhg(prob, SLAB_EPOCHS * prob.iters_per_epoch(), seed=SLAB_SEED)
    X = prob.reported(st)
    psi_o = prob.objective(X)
    t = {k: dev(d[k]) for k in ("b", "r", "mult")}
    x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
    rec = P.Reconstruction(g, P.cparams(SLAB_M, "tv", "balanced", True, alpha=SLAB_ALPHA,
                                        seed=SLAB_SEED), t["b"], t["r"], t["mult"], x)
    try:
        rec.epoch(SLAB_EPOCHS)
        torch.cuda.synchronize()
        err = rel(x.cpu().numpy(), X[0])
        obj = float(rec.objective().cpu().numpy()[0])
        print(f"[span1] slab image rel err {err:.3e}, objective rel err "
              f"{abs(obj - psi_o) / abs(psi_o):.3e}", flush=True)
        assert err <= 1e-3
        assert abs(obj - psi_o) <= 1e-4 * abs(psi_o)
    finally:
        rec.close()


@pytest.fixture(scope="module")
def mmr1():
    g = synth.mmr_span1()
    rng = np.random.default_rng(12)
    return g, rng.uniform(0, 1, g.image_shape).astype(np.float32)


def test_mmr_span1_forward_sampled_rays(P, mmr1):
    g, x = mmr1
    print(f"[span1] mMR span 1: {g.n_seg} segments, {g.n_planes} planes, m=21 subset 2",
          flush=True)
    m, i = 21, 2
    ang = g.subset_angles(m, i)
    out = torch.empty(len(ang) * g.n_planes * g.n_rad, dtype=torch.float32, device="cuda:0")
    P.spdhg_project(g, m, i, None, dev(x), out)
    got = out.cpu().numpy().reshape(len(ang), g.n_planes, g.n_rad)
    rng = np.random.default_rng(13)
    xd = x.astype(np.float64)
    ref, val = [], []
    for k in range(0, g.n_rad, 2):
        ia, q = int(rng.integers(len(ang))), int(rng.integers(g.n_planes))
        ref.append(OP.ray(g, xd, ang[ia], q, k))
        val.append(got[ia, q, k])
    ref, val = np.array(ref), np.array(val)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(val - ref)) <= 1e-5 * scale
    assert np.linalg.norm(val - ref) <= 1e-5 * np.linalg.norm(ref)


def test_mmr_span1_backward_one_angle(P, mmr1):
    g, _ = mmr1
    print("[span1] mMR span 1: backprojection of one angle (m=252, subset 100)", flush=True)
    m, i = 252, 100
    ang = g.subset_angles(m, i)
    y = np.random.default_rng(14).uniform(0, 1, (len(ang), g.n_planes, g.n_rad)).astype(
        np.float32)
    ref = OP.backward(g, y.astype(np.float64), ang)
    out = torch.empty(g.image_shape, dtype=torch.float32, device="cuda:0")
    P.spdhg_backproject(g, m, i, None, dev(y), out)
    close(out.cpu().numpy(), ref)
