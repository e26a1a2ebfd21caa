"""The compensated primal step (SPDHG_FLAG_COMPENSATED): the primal state x and z of
Algorithm 2 held as FP32 pairs (value + low part) and the primal step taken in FP64 on
their sums.

* Parity with the FP64 oracle to the bar of the plain path (image within 1e-3 relative
  L2, objective within 1e-4) for TV, dTV and no prior, SPDHG and PDHG (Algorithm 1), on
  geometries that run the strip gather, the column gather and both prior kernels; the
  image is the sum of the two parts.
* With one angle per subset (90 subsets of the 2-D slice) the compensated state is
  closer to the oracle than the plain FP32 state.
* Each pair is normalised: the value is the FP32 rounding of the sum and the low part
  is at most half an ulp of it.
* Epochs from the persistent graph are bitwise the eager ones; a checkpoint carries the
  low parts, so a restored run resumes bitwise.
* TGV with the flag is refused (SPDHG_E_NOTIMPL)."""
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


def pair_sum(rec, x):
    """The iterate of a compensated run: value + low part, in FP64 (caller layout)."""
    lo = rec.buffer("x_lo")
    return x.cpu().numpy().astype(np.float64) + lo.cpu().numpy().astype(np.float64)


def check_normalised(hi, lo):
    hi = np.asarray(hi, np.float32).ravel()
    lo = np.asarray(lo, np.float32).ravel()
    s = hi.astype(np.float64) + lo.astype(np.float64)
    np.testing.assert_array_equal(s.astype(np.float32), hi)
    assert np.all(np.abs(lo) <= 0.5 * np.spacing(np.abs(hi)))


CASES = {
    "slice64": lambda: synth.slice64_problem(),
    "tall3d": lambda: synth.brain_problem(
        synth.Geometry(nx=40, ny=40, nz=33, vx=5.0, vy=5.0, vz=5.0, n_rad=44, d_rad=5.0,
                       n_ang=24, seg_planes=(33, 29, 29), seg_tan=(0.0, 0.25, -0.25)),
        18081400, 5e5),
    "deep3d": lambda: synth.brain_problem(
        synth.Geometry(nx=21, ny=21, nz=70, vx=5.0, vy=5.0, vz=5.0, n_rad=26, d_rad=5.0,
                       n_ang=8, seg_planes=(70, 66, 66), seg_tan=(0.0, 0.25, -0.25)),
        18081401, 5e5, with_side=True),
}
_cache = {}


def case(name):
    if name not in _cache:
        _cache[name] = CASES[name]()
    return _cache[name]


def _rec(P, d, m, prior, sampling, alpha, seed, compensated, side=None):
    g = d["geom"]
    t = {k: dev(d[k]) for k in ("b", "r", "mult")}
    x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
    rec = P.Reconstruction(g, P.cparams(m, prior, sampling, True, alpha=alpha, seed=seed,
                                        compensated=compensated),
                           t["b"], t["r"], t["mult"], x,
                           side=dev(side) if side is not None else None)
    rec._keep = t
    return rec, x


@pytest.mark.parametrize("name,m,prior,sampling,alpha,epochs", [
    ("slice64", 10, "tv", "balanced", 0.1, 20),
    ("slice64", 10, "none", "uniform", 0.0, 10),
    ("tall3d", 8, "tv", "balanced", 0.05, 3),
    ("deep3d", 4, "dtv", "balanced", 0.05, 3)])
def test_compensated_spdhg_parity(P, name, m, prior, sampling, alpha, epochs):
    print(f"[compensated] SPDHG {name} {prior} m={m} {epochs} epochs", flush=True)
    d = case(name)
    side = d.get("side") if prior == "dtv" else None
    seed = 18081410
    prob = S.Problem(d["geom"], d["b"], d["r"], d["mult"], n_subsets=m, prior=prior,
                     alpha=alpha, sampling=sampling, side=side)
    st = S.spdhg(prob, epochs * prob.iters_per_epoch(), seed=seed)
    X = prob.reported(st)
    rec, x = _rec(P, d, m, prior, sampling, alpha, seed, True, side)
    try:
        rec.epoch(epochs)
        torch.cuda.synchronize()
        xs = pair_sum(rec, x)
        err = rel(xs, X[0])
        psi_o = prob.objective(X)
        obj = float(rec.objective().cpu().numpy()[0])
        print(f"[compensated] image rel err {err:.3e}, objective rel err "
              f"{abs(obj - psi_o) / abs(psi_o):.3e}", flush=True)
        assert err <= 1e-3
        assert abs(obj - psi_o) <= 1e-4 * abs(psi_o)
        check_normalised(x.cpu().numpy(), rec.buffer("x_lo").cpu().numpy())
        check_normalised(rec.buffer("z").cpu().numpy(), rec.buffer("z_lo").cpu().numpy())
    finally:
        rec.close()


@pytest.mark.parametrize("name,prior,alpha,iters", [
    ("slice64", "none", 0.0, 100), ("slice64", "tv", 0.1, 100), ("tall3d", "tv", 0.05, 30)])
def test_compensated_pdhg_parity(P, name, prior, alpha, iters):
    print(f"[compensated] PDHG {name} {prior} {iters} iterations", flush=True)
    d = case(name)
    sampling = "balanced" if prior != "none" else "uniform"
    prob = S.Problem(d["geom"], d["b"], d["r"], d["mult"], n_subsets=1, prior=prior,
                     alpha=alpha, sampling=sampling)
    pp = S.pdhg_problem(prob)
    st = S.pdhg(pp, iters)
    X = pp.reported(st)
    rec, x = _rec(P, d, 1, prior, sampling, alpha, 1, True)
    try:
        rec.pdhg_iterate(iters)
        torch.cuda.synchronize()
        err = rel(pair_sum(rec, x), X[0])
        psi_o = pp.objective(X)
        obj = float(rec.objective().cpu().numpy()[0])
        print(f"[compensated] image rel err {err:.3e}, objective rel err "
              f"{abs(obj - psi_o) / abs(psi_o):.3e}", flush=True)
        assert err <= 1e-3
        assert abs(obj - psi_o) <= 1e-4 * abs(psi_o)
    finally:
        rec.close()


def test_compensated_closer_with_single_angle_subsets(P):
    """90 single-angle subsets: each data iteration moves z by one angle's share, the
    regime where the plain FP32 state loses the most to rounding."""
    d = case("slice64")
    m, epochs, seed = 90, 15, 18081420
    print(f"[compensated] slice64 TV m={m}: oracle {epochs} epochs", flush=True)
    prob = S.Problem(d["geom"], d["b"], d["r"], d["mult"], n_subsets=m, prior="tv",
                     alpha=0.1, sampling="balanced")
    st = S.spdhg(prob, epochs * prob.iters_per_epoch(), seed=seed)
    X = prob.reported(st)[0]
    errs = {}
    for comp in (False, True):
        rec, x = _rec(P, d, m, "tv", "balanced", 0.1, seed, comp)
        try:
            rec.epoch(epochs)
            torch.cuda.synchronize()
            xs = pair_sum(rec, x) if comp else x.cpu().numpy()
            errs[comp] = rel(xs, X)
        finally:
            rec.close()
    print(f"[compensated] image rel err: plain {errs[False]:.3e}, compensated "
          f"{errs[True]:.3e}", flush=True)
    assert errs[True] <= 1e-3 and errs[False] <= 1e-3
    assert errs[True] < errs[False]


def test_compensated_graph_and_checkpoint_bitwise(P):
    d = case("tall3d")
    g = d["geom"]
    out = []
    for graph in (False, True):
        rec, x = _rec(P, d, 8, "tv", "balanced", 0.05, 31, True)
        try:
            for _ in range(2):
                if graph:
                    rec.epoch_graph(1)
                else:
                    rec.epoch(1)
                torch.cuda.synchronize()
                _ = rec.objective().cpu()  # eager work between the graphs
            out.append((x.cpu().numpy(), rec.buffer("x_lo").cpu().numpy(),
                        rec.buffer("z_lo").cpu().numpy()))
        finally:
            rec.close()
    for a, b in zip(out[0], out[1]):
        np.testing.assert_array_equal(a, b)
    # checkpoint after one epoch, continue one; restore, continue one again
    rec, x = _rec(P, d, 8, "tv", "balanced", 0.05, 31, True)
    try:
        rec.epoch(1)
        snap = rec.save_state()
        rec.epoch(1)
        torch.cuda.synchronize()
        a = (x.cpu().numpy(), rec.buffer("x_lo").cpu().numpy())
        np.testing.assert_array_equal(a[0], out[0][0])
        rec.iterate(5)
        rec.load_state(snap)
        rec.epoch(1)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(x.cpu().numpy(), a[0])
        np.testing.assert_array_equal(rec.buffer("x_lo").cpu().numpy(), a[1])
    finally:
        rec.close()
    assert g.nz == 33


def test_compensated_tgv_refused(P):
    from paper_1808_07150_amd.spdhg import SpdhgError
    d = case("tall3d")
    with pytest.raises(SpdhgError) as e:
        _rec(P, d, 8, "tgv", "balanced", 0.05, 1, True)
    assert e.value.code == -7
