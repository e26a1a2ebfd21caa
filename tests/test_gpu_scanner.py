"""The closer scanner model on the GPU: non-arc-corrected radial bins, s-dependent slopes,
span-compressed data planes (sums of ring-pair rays) and detector gaps.

* Projector parity (1e-5 relative, forward and backward, with and without mult) against
  the FP64 oracle for each feature alone and all together, on geometries that run the
  column gather (nz < 32) and the strip gather's pitch-2 instance (nz >= 32); the GPU
  adjoint identity.
* K epochs of SPDHG+ with TV (and the objective) against the oracle with every feature and
  detector gaps on a 40 x 40 x 33 image (17 rings, span 3): image within 1e-3, objective
  within 1e-4.
* The mMR-sized model (344 x 344 x 127, span-11 data 344 x 252 x 837 from 4084 ring-pair
  planes): sampled data bins of a subset at every other radial bin, and a single-angle
  backprojection, against the oracle."""
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


def scanner(rings, max_rd, span, nxy, n_rad, n_ang, v, R, nonarc=True, oblique_s=True, nx=None):
    planes, tans, pitch = synth.span1_segments(rings, max_rd, v, R)
    return synth.Geometry(nx=nx or nxy, ny=nxy, nz=2 * rings - 1, vx=v, vy=v, vz=v,
                          n_rad=n_rad, d_rad=v, n_ang=n_ang, seg_planes=planes, seg_tan=tans,
                          seg_pitch=pitch, det_radius=R, nonarc=nonarc, oblique_s=oblique_s,
                          span=span)


GEOMS = {
    # every feature, nz = 15: the column gather
    "all_thin": synth.scanner_small(),
    # each feature alone (ragged in-plane sizes)
    "nonarc": scanner(6, 5, 0, 19, 25, 10, 4.0, 55.0, oblique_s=False, nx=17),
    "oblique": scanner(6, 5, 0, 19, 25, 10, 4.0, 55.0, nonarc=False, nx=17),
    "span5": scanner(6, 5, 5, 19, 25, 10, 4.0, 55.0, nonarc=False, oblique_s=False, nx=17),
    # every feature, nz = 33: the strip gather's pitch-2 instance on compressed data
    "all_tall": scanner(17, 7, 3, 21, 26, 8, 4.0, 60.0),
}


def _inputs(g, seed):
    rng = np.random.default_rng(seed)
    return (rng.uniform(0, 2, g.image_shape).astype(np.float32),
            rng.uniform(0.5, 1.5, g.sino_shape).astype(np.float32),
            rng.normal(size=g.sino_shape).astype(np.float32))


@pytest.mark.parametrize("name", list(GEOMS))
@pytest.mark.parametrize("m,subset", [(1, -1), (4, 1)])
def test_scanner_projector_parity(P, name, m, subset):
    g = GEOMS[name]
    print(f"[scanner] {name}: {g.n_seg} ray-pair segments, {g.n_planes} ray planes, "
          f"{g.n_data_planes} data planes, m={m} subset={subset}", flush=True)
    x, mult, y = _inputs(g, 3)
    ang = list(range(g.n_ang)) if subset < 0 else g.subset_angles(m, subset)
    ref = mult[ang] * OP.forward(g, x.astype(np.float64), ang)
    out = torch.empty(len(ang) * g.n_data_planes * g.n_rad, dtype=torch.float32,
                      device="cuda:0")
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
def test_scanner_gpu_adjoint(P, name):
    g = GEOMS[name]
    x, mult, y = _inputs(g, 4)
    ax = torch.empty(g.n_bins, dtype=torch.float32, device="cuda:0")
    aty = torch.empty(g.image_shape, dtype=torch.float32, device="cuda:0")
    P.spdhg_project(g, 1, -1, dev(mult), dev(x), ax)
    P.spdhg_backproject(g, 1, -1, dev(mult), dev(y), aty)
    lhs = float(np.dot(ax.cpu().numpy().astype(np.float64), y.ravel()))
    rhs = float(np.dot(x.ravel().astype(np.float64), aty.cpu().numpy().ravel()))
    assert abs(lhs - rhs) <= 1e-6 * max(abs(lhs), abs(rhs))


TV_SEED, TV_COUNTS, TV_M, TV_EPOCHS, TV_ALPHA = 18081500, 5e5, 6, 4, 0.05


@pytest.fixture(scope="module")
def scanner_problem():
    g = scanner(17, 7, 3, 40, 44, 24, 5.0, 150.0)
    return synth.brain_problem(g, TV_SEED, TV_COUNTS, gaps=True)


@pytest.mark.parametrize("sampling,precond", [("balanced", True), ("uniform", False)])
def test_scanner_tv_parity(P, scanner_problem, sampling, precond):
    d = scanner_problem
    g = d["geom"]
    assert float((d["mult"] == 0).mean()) > 0.1  # the gaps are there
    print(f"[scanner] TV {g.nx}x{g.ny}x{g.nz}, {g.n_data_planes} data planes from "
          f"{g.n_planes} ray planes, gaps, {sampling}: oracle {TV_EPOCHS} epochs", flush=True)
    prob = S.Problem(g, d["b"], d["r"], d["mult"], n_subsets=TV_M, prior="tv",
                     alpha=TV_ALPHA, sampling=sampling, precond=precond)
    st = S.spdhg(prob, TV_EPOCHS * prob.iters_per_epoch(), seed=TV_SEED)
    X = prob.reported(st)
    psi_o = prob.objective(X)
    t = {k: dev(d[k]) for k in ("b", "r", "mult")}
    x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
    rec = P.Reconstruction(g, P.cparams(TV_M, "tv", sampling, precond, alpha=TV_ALPHA,
                                        seed=TV_SEED), t["b"], t["r"], t["mult"], x)
    try:
        rec.epoch(TV_EPOCHS)
        torch.cuda.synchronize()
        err = rel(x.cpu().numpy(), X[0])
        obj = float(rec.objective().cpu().numpy()[0])
        print(f"[scanner] image rel err {err:.3e}, objective rel err "
              f"{abs(obj - psi_o) / abs(psi_o):.3e}", flush=True)
        assert err <= 1e-3
        assert abs(obj - psi_o) <= 1e-4 * abs(psi_o)
    finally:
        rec.close()


@pytest.fixture(scope="module")
def mmr_scanner():
    g = synth.mmr_scanner()
    rng = np.random.default_rng(22)
    return g, rng.uniform(0, 1, g.image_shape).astype(np.float32)


def test_mmr_scanner_forward_sampled_bins(P, mmr_scanner):
    g, x = mmr_scanner
    print(f"[scanner] mMR: {g.n_planes} ray planes -> {g.n_data_planes} data planes, m=21 "
          "subset 5", flush=True)
    m, i = 21, 5
    ang = g.subset_angles(m, i)
    out = torch.empty(len(ang) * g.n_data_planes * g.n_rad, dtype=torch.float32,
                      device="cuda:0")
    P.spdhg_project(g, m, i, None, dev(x), out)
    got = out.cpu().numpy().reshape(len(ang), g.n_data_planes, g.n_rad)
    rng = np.random.default_rng(23)
    xd = x.astype(np.float64)
    ref, val = [], []
    for k in range(0, g.n_rad, 2):
        ia, q = int(rng.integers(len(ang))), int(rng.integers(g.n_data_planes))
        ref.append(OP.ray(g, xd, ang[ia], q, k))
        val.append(got[ia, q, k])
    ref, val = np.array(ref), np.array(val)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(val - ref)) <= 1e-5 * scale
    assert np.linalg.norm(val - ref) <= 1e-5 * np.linalg.norm(ref)


def test_mmr_scanner_backward_one_angle(P, mmr_scanner):
    g, _ = mmr_scanner
    print("[scanner] mMR: backprojection of one angle (m=252, subset 40)", flush=True)
    m, i = 252, 40
    ang = g.subset_angles(m, i)
    y = np.random.default_rng(24).uniform(0, 1, (len(ang), g.n_data_planes, g.n_rad)).astype(
        np.float32)
    ref = OP.backward(g, y.astype(np.float64), ang)
    out = torch.empty(g.image_shape, dtype=torch.float32, device="cuda:0")
    P.spdhg_backproject(g, m, i, None, dev(y), out)
    close(out.cpu().numpy(), ref)
