"""Parity at the scale of an mMR slab and at the benchmark's launch configuration.

* K epochs of SPDHG+ with TV on a 344 x 344 x 16 slab of the mMR (segments 0, +-1: 16 + 4
  + 4 planes, 252 angles x 344 radial bins, 21 subsets) against the FP64 oracle's own
  Algorithm 2 loop on the same data and block sequence, with the ray-bundle split chosen
  from the launch size and fixed at 4 (the benchmark's fwd_wave<., F_DUAL, 4> instance).
  Bar: image within 1e-3 (relative L2), objective within 1e-4.
* The duality gap (box [0, U]) of a state that both sides hold exactly: the oracle's
  state after K epochs, rounded to FP32, is loaded into the library as a checkpoint, so
  the library's gap and the oracle's are evaluated on the same iterate.  Bar: relative to
  the gap itself.
"""
import numpy as np
import pytest

import synth
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


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


SLAB_M, SLAB_EPOCHS, SLAB_SEED, SLAB_COUNTS = 21, 3, 18081000, 3e6
SLAB_ALPHA = 0.1 * (1e5 / SLAB_COUNTS) ** 0.5  # beta = 0.1 sqrt(1e5 / counts)


@pytest.fixture(scope="module")
def slab_case():
    g = synth.slab(16)
    d = synth.brain_problem(g, SLAB_SEED, SLAB_COUNTS)
    print(f"[slab] oracle: {g.nx}x{g.ny}x{g.nz}, {g.n_ang} x {g.n_planes} x {g.n_rad}, "
          f"TV m={SLAB_M}, {SLAB_EPOCHS} epochs", flush=True)
    prob = S.Problem(g, d["b"], d["r"], d["mult"], n_subsets=SLAB_M, prior="tv",
                     alpha=SLAB_ALPHA, sampling="balanced", precond=True)
    st = S.spdhg(prob, SLAB_EPOCHS * prob.iters_per_epoch(), seed=SLAB_SEED)
    X = prob.reported(st)
    return g, d, prob, X, prob.objective(X)


@pytest.mark.parametrize("split", [0, 4])
def test_slab_tv_parity(P, slab_case, split):
    g, d, prob, X, psi_o = slab_case
    print(f"[slab] GPU split={split}", flush=True)
    t = {k: dev(d[k]) for k in ("b", "r", "mult")}
    x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
    rec = P.Reconstruction(g, P.cparams(SLAB_M, "tv", "balanced", True, alpha=SLAB_ALPHA,
                                        seed=SLAB_SEED), t["b"], t["r"], t["mult"], x)
    try:
        rec.set_tuning(split)
        assert rec.iters_per_epoch == prob.iters_per_epoch()
        rec.epoch(SLAB_EPOCHS)
        torch.cuda.synchronize()
        err = rel(x.cpu().numpy(), X[0])
        obj = float(rec.objective().cpu().numpy()[0])
        print(f"[slab] image rel err {err:.3e}, objective rel err "
              f"{abs(obj - psi_o) / abs(psi_o):.3e}", flush=True)
        assert err <= 1e-3
        assert abs(obj - psi_o) <= 1e-4 * abs(psi_o)
    finally:
        rec.close()


def state_buffer(rec, prob, st, X):
    """The oracle's state (reported image, z, data duals, prior dual) in the library's
    checkpoint format: each array FP32 in the internal layout (images z-fastest
    [y][x][z], sinograms [angle][radial][plane], fields component-major), padded to 256
    bytes, then the header [iteration, voxels, bins, tag]."""
    g = prob.geom
    parts = [X[0].transpose(1, 2, 0), st["z"][0].transpose(1, 2, 0)]
    y = np.zeros(g.sino_shape)
    for i, ang in enumerate(prob.angles):
        y[ang] = st["y"][i]
    parts.append(y.transpose(0, 2, 1))
    if prob.n_prior:
        parts.append(st["yp"][0].transpose(0, 2, 3, 1))
    blob = b""
    for a in parts:
        raw = np.ascontiguousarray(a, dtype=np.float32).tobytes()
        blob += raw + b"\0" * ((-len(raw)) % 256)
    blob += np.array([st["k"], g.n_vox, g.n_bins, 0x5350444847], dtype=np.int64).tobytes()
    n = rec.state_bytes()
    assert len(blob) <= n
    buf = np.zeros(n, dtype=np.uint8)
    buf[:len(blob)] = np.frombuffer(blob, dtype=np.uint8)
    return torch.from_numpy(buf).to("cuda:0")


@pytest.mark.parametrize("prior", ["tv", "atv", "none"])
def test_gap_on_a_shared_state(P, prior):
    """spdhg_gap against the oracle's duality gap on the very same FP32 state: within
    1e-3 of the gap itself (the gap is a small difference of the primal and dual sums)."""
    d = synth.slice64_problem()
    g = d["geom"]
    print(f"[gap] slice64 {prior}: oracle state after 20 epochs", flush=True)
    prob = S.Problem(g, d["b"], d["r"], d["mult"], n_subsets=10, prior=prior, alpha=0.1,
                     sampling="balanced")
    st = S.spdhg(prob, 20 * prob.iters_per_epoch(), seed=4)
    X = prob.reported(st)
    # the state both sides evaluate: FP32-rounded image, duals and z.  Rounding may push a
    # prior dual just outside its ball / box (f* = +inf there) or a data dual up to 1:
    # the prior duals are shrunk by 1e-6 first, the data duals kept below 1
    r32 = lambda a: np.asarray(a, np.float32).astype(np.float64)  # noqa: E731
    below1 = float(np.nextafter(np.float32(1.0), np.float32(0.0)))
    X = r32(X)
    st32 = dict(st, z=r32(st["z"]), y=[np.minimum(r32(v), below1) for v in st["y"]],
                yp=[r32(v * (1.0 - 1e-6)) for v in st["yp"]])
    U = 2.0 * float(X[0].max())
    ref = S.duality_gap(prob, X, st32, U)
    t = {k: dev(d[k]) for k in ("b", "r", "mult")}
    x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
    rec = P.Reconstruction(g, P.cparams(10, prior, "balanced", True, alpha=0.1, seed=4),
                           t["b"], t["r"], t["mult"], x)
    try:
        rec.load_state(state_buffer(rec, prob, st32, X))
        out = rec.gap(U).cpu().numpy()
    finally:
        rec.close()
    psi = prob.objective(X)
    print(f"[gap] {prior}: gap {out[0]:.6e} oracle {ref:.6e} (psi {psi:.6e}), "
          f"rel {abs(out[0] - ref) / ref:.3e}", flush=True)
    assert np.isfinite(ref) and ref > 0 and np.isfinite(out[0])
    assert abs(out[0] - ref) <= 1e-3 * ref
