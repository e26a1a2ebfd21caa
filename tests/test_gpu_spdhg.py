"""GPU SPDHG (Algorithm 2) through the C ABI against the FP64 oracle on the same seeded
inputs and the same SplitMix64 block sequence.

Bar: image after K epochs within 1e-3 (relative L2), objective within 1e-4 (relative);
step-size maps within 1e-5; reruns bitwise identical; a checkpointed run resumes bitwise."""
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


@pytest.fixture(scope="module")
def c1():
    return synth.slice64_problem()


@pytest.fixture(scope="module")
def small3d():
    g = synth.small_3d(nxy=40, nz=9, n_rad=44, n_ang=24, v=5.0, tan1=0.3)
    return synth.brain_problem(g, 18080300, 2e5, with_side=True)


@pytest.fixture(scope="module")
def tall3d():
    g = synth.Geometry(nx=40, ny=40, nz=33, vx=5.0, vy=5.0, vz=5.0, n_rad=44, d_rad=5.0,
                       n_ang=24, seg_planes=(33, 29, 29), seg_tan=(0.0, 0.25, -0.25))
    return synth.brain_problem(g, 18080400, 5e5)


@pytest.fixture(scope="module")
def deep3d():
    """nz = 70 (two 64-lane runs per column), odd and ragged in-plane sizes."""
    g = synth.Geometry(nx=21, ny=21, nz=70, vx=5.0, vy=5.0, vz=5.0, n_rad=26, d_rad=5.0,
                       n_ang=8, seg_planes=(70, 66, 66), seg_tan=(0.0, 0.25, -0.25))
    return synth.brain_problem(g, 18080600, 5e5, with_side=True)


@pytest.fixture(scope="module")
def maxnz3d():
    """nz = 128, the largest the library accepts: three overlapping 64-voxel runs per
    column in the wavefront prior kernels, and the per-column gather (the strip gather
    stops at 127 planes)."""
    g = synth.Geometry(nx=12, ny=13, nz=128, vx=5.0, vy=5.0, vz=5.0, n_rad=16, d_rad=5.0,
                       n_ang=6, seg_planes=(128, 126, 126), seg_tan=(0.0, 0.2, -0.2))
    return synth.brain_problem(g, 18080800, 5e5)


@pytest.fixture(scope="module")
def span11_3d():
    """The mMR's span-11 segment structure (11 segments, 837 planes) on a 13 x 13 x 127
    image: the 14-row forward instances of the iteration and the objective, and the strip
    gather with all 11 segment loads of a ray in one batch, at a size the oracle runs in a
    second."""
    g = synth.mmr(nxy=13, vxy=5.0, n_rad=16, n_ang=6)
    return synth.brain_problem(g, 18080900, 5e5)


def run_pair(P, d, n_subsets, prior, epochs, seed, sampling="uniform", precond=True,
             alpha=0.1, side=None, eta=1e-2, alpha1=0.0):
    g = d["geom"]
    prob = S.Problem(g, d["b"], d["r"], d["mult"], n_subsets=n_subsets, prior=prior,
                     alpha=alpha, sampling=sampling, precond=precond, side=side, eta=eta,
                     alpha1=alpha1)
    t = {k: dev(d[k]) for k in ("b", "r", "mult")}
    x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
    sd = dev(side) if side is not None else None
    rec = P.Reconstruction(g, P.cparams(n_subsets, prior, sampling, precond, alpha=alpha,
                                        eta=eta, seed=seed, alpha1=alpha1),
                           t["b"], t["r"], t["mult"], x, side=sd)
    assert rec.iters_per_epoch == prob.iters_per_epoch()
    st = S.spdhg(prob, epochs * prob.iters_per_epoch(), seed=seed)
    rec.epoch(epochs)
    torch.cuda.synchronize()
    return prob, st, rec, x


@pytest.mark.parametrize("sampling,precond,epochs", [("uniform", True, 50),
                                                     ("balanced", True, 30),
                                                     ("balanced", False, 20)])
def test_slice64_tv_parity(P, c1, sampling, precond, epochs):
    print(f"[spdhg] slice64 TV {sampling} precond={precond} epochs={epochs}", flush=True)
    prob, st, rec, x = run_pair(P, c1, 10, "tv", epochs, seed=1808, sampling=sampling,
                                precond=precond)
    xo = prob.reported(st)[0]
    xg = x.cpu().numpy()
    assert rel(xg, xo) <= 1e-3
    obj = rec.objective().cpu().numpy()
    psi_o = prob.objective(xo[None])
    assert abs(obj[0] - psi_o) <= 1e-4 * abs(psi_o)
    # the GPU objective of the oracle image matches the oracle objective closely
    obj2 = rec.objective(dev(xo)).cpu().numpy()
    assert abs(obj2[0] - psi_o) <= 1e-5 * abs(psi_o)


@pytest.mark.parametrize("prior", ["tv", "atv", "none"])
def test_slice64_duality_gap(P, c1, prior):
    """GPU duality gap (box U) against the oracle's on the same state after 20 epochs."""
    print(f"[spdhg] slice64 gap {prior}", flush=True)
    prob, st, rec, x = run_pair(P, c1, 10, prior, 20, seed=4, sampling="balanced")
    X = prob.reported(st)
    U = 2.0 * float(X[0].max())
    ref = S.duality_gap(prob, X, st, U)
    out = rec.gap(U).cpu().numpy()
    psi = prob.objective(X)
    assert np.isfinite(out[0]) and np.isfinite(ref)
    # pieces: primal (masked objective), dual sum, box term
    assert abs(out[0] - ref) <= 1e-4 * abs(psi)
    assert out[0] >= -1e-4 * abs(psi)


def test_slice64_step_sizes(P, c1):
    prob, _, rec, _ = run_pair(P, c1, 10, "tv", 0, seed=1, sampling="balanced")
    T = rec.buffer("T").cpu().numpy().reshape(c1["geom"].image_shape)
    assert rel(T, prob.T[0]) <= 1e-5
    sig = rec.buffer("sigma").cpu().numpy().reshape(c1["geom"].sino_shape)
    ref = np.zeros(c1["geom"].sino_shape)
    for i in range(prob.m):
        ref[prob.angles[i]] = prob.sigma[i]
    both = (sig > 0) & (ref > 0)
    assert np.sum((sig > 0) != (ref > 0)) <= 0.001 * sig.size
    assert rel(sig[both], ref[both]) <= 1e-5
    s, p, nrm = rec.block_info(10)
    assert p == prob.p[10] and s == pytest.approx(prob.prior_sigma[0], rel=1e-12)


@pytest.mark.parametrize("prior,sampling,epochs", [("tv", "balanced", 12), ("none", "uniform", 12),
                                                   ("dtv", "balanced", 12)])
def test_small3d_parity(P, small3d, prior, sampling, epochs):
    print(f"[spdhg] small3d {prior} {sampling} epochs={epochs}", flush=True)
    side = small3d["side"] if prior == "dtv" else None
    prob, st, rec, x = run_pair(P, small3d, 6, prior, epochs, seed=77, sampling=sampling,
                                alpha=0.05, side=side)
    xo = prob.reported(st)[0]
    xg = x.cpu().numpy()
    assert rel(xg, xo) <= 1e-3
    psi_o = prob.objective(xo[None])
    obj = rec.objective().cpu().numpy()
    assert abs(obj[0] - psi_o) <= 1e-4 * abs(psi_o)


@pytest.mark.parametrize("sampling,precond", [("balanced", True), ("uniform", False)])
def test_small3d_tgv_parity(P, small3d, sampling, precond):
    """TGV (two prior blocks, x = (u, w)): u, w and the objective after 12 epochs."""
    print(f"[spdhg] small3d TGV {sampling} precond={precond}", flush=True)
    prob, st, rec, x = run_pair(P, small3d, 6, "tgv", 12, seed=91, sampling=sampling,
                                precond=precond, alpha=0.05, alpha1=0.025)
    X = prob.reported(st)
    assert rel(x.cpu().numpy(), X[0]) <= 1e-3
    w = rec.buffer("w").cpu().numpy()
    print(f"[spdhg] TGV rel err u {rel(x.cpu().numpy(), X[0]):.3e} w {rel(w, X[1:4]):.3e}",
          flush=True)
    assert rel(w, X[1:4]) <= 1e-3
    psi_o = prob.objective(X)
    assert abs(rec.objective().cpu().numpy()[0] - psi_o) <= 1e-4 * abs(psi_o)
    # step scalars of both prior blocks (||(grad, -I)|| closed form, ||E|| by power iteration)
    for j in range(2):
        s, p, nrm = rec.block_info(6 + j)
        assert p == prob.p[6 + j]
        assert nrm == pytest.approx(prob.norms[6 + j], rel=1e-5)
        assert s == pytest.approx(prob.prior_sigma[j], rel=1e-5)


def test_small3d_atv_parity(P, small3d):
    print("[spdhg] small3d aTV uniform", flush=True)
    prob, st, rec, x = run_pair(P, small3d, 6, "atv", 12, seed=13, alpha=0.05)
    xo = prob.reported(st)[0]
    assert rel(x.cpu().numpy(), xo) <= 1e-3
    psi_o = prob.objective(xo[None])
    assert abs(rec.objective().cpu().numpy()[0] - psi_o) <= 1e-4 * abs(psi_o)


def test_tgv_checkpoint_bitwise(P, small3d):
    """Save after 3 epochs, run 2 more; restore and rerun: identical u and w."""
    g = small3d["geom"]
    t = {k: dev(small3d[k]) for k in ("b", "r", "mult")}
    prm = P.cparams(6, "tgv", "balanced", alpha=0.05, alpha1=0.025, seed=5)
    x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
    rec = P.Reconstruction(g, prm, t["b"], t["r"], t["mult"], x)
    rec.epoch(3)
    snap = rec.save_state()
    rec.epoch(2)
    torch.cuda.synchronize()
    a, wa = x.cpu().numpy(), rec.buffer("w").cpu().numpy()
    rec.load_state(snap)
    rec.epoch(2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(x.cpu().numpy(), a)
    np.testing.assert_array_equal(rec.buffer("w").cpu().numpy(), wa)


@pytest.mark.parametrize("sampling,precond,m", [("balanced", True, 8), ("uniform", False, 3)])
def test_tall3d_tv_parity(P, tall3d, sampling, precond, m):
    """nz = 33: the tiled gather backprojector inside the iteration."""
    print(f"[spdhg] tall3d TV {sampling} precond={precond} m={m}", flush=True)
    prob, st, rec, x = run_pair(P, tall3d, m, "tv", 10, seed=31, sampling=sampling,
                                precond=precond, alpha=0.05)
    xo = prob.reported(st)[0]
    assert rel(x.cpu().numpy(), xo) <= 1e-3
    psi_o = prob.objective(xo[None])
    assert abs(rec.objective().cpu().numpy()[0] - psi_o) <= 1e-4 * abs(psi_o)


@pytest.mark.parametrize("prior", ["tv", "dtv", "atv", "tgv"])
def test_deep3d_prior_parity(P, deep3d, prior):
    """nz = 70, ny = 21: the wavefront prior kernels with two overlapping runs per column
    (the upper run's first lane only passes its dual change on) and a ragged last row
    chunk."""
    print(f"[spdhg] deep3d {prior}", flush=True)
    side = deep3d["side"] if prior == "dtv" else None
    prob, st, rec, x = run_pair(P, deep3d, 4, prior, 10, seed=37, sampling="balanced",
                                alpha=0.05, side=side, alpha1=0.025 if prior == "tgv" else 0.0)
    X = prob.reported(st)
    assert rel(x.cpu().numpy(), X[0]) <= 1e-3
    if prior == "tgv":
        ew = rel(rec.buffer("w").cpu().numpy(), X[1:4])
        print(f"[spdhg] TGV rel err u {rel(x.cpu().numpy(), X[0]):.3e} w {ew:.3e}", flush=True)
        assert ew <= 1e-3
    psi_o = prob.objective(X)
    assert abs(rec.objective().cpu().numpy()[0] - psi_o) <= 1e-4 * abs(psi_o)


@pytest.mark.parametrize("prior", ["tv", "tgv"])
def test_maxnz_parity(P, maxnz3d, prior):
    print(f"[spdhg] maxnz (nz=128) {prior}", flush=True)
    prob, st, rec, x = run_pair(P, maxnz3d, 3, prior, 10, seed=41, sampling="balanced",
                                alpha=0.05, alpha1=0.025 if prior == "tgv" else 0.0)
    X = prob.reported(st)
    assert rel(x.cpu().numpy(), X[0]) <= 1e-3
    if prior == "tgv":
        ew = rel(rec.buffer("w").cpu().numpy(), X[1:4])
        print(f"[spdhg] TGV rel err u {rel(x.cpu().numpy(), X[0]):.3e} w {ew:.3e}", flush=True)
        assert ew <= 1e-3
    psi_o = prob.objective(X)
    assert abs(rec.objective().cpu().numpy()[0] - psi_o) <= 1e-4 * abs(psi_o)


@pytest.mark.parametrize("prior", ["tv", "tgv"])
def test_span11_parity(P, span11_3d, prior):
    print(f"[spdhg] span11 (837 planes) {prior}", flush=True)
    prob, st, rec, x = run_pair(P, span11_3d, 3, prior, 10, seed=43, sampling="balanced",
                                alpha=0.05, alpha1=0.025 if prior == "tgv" else 0.0)
    X = prob.reported(st)
    assert rel(x.cpu().numpy(), X[0]) <= 1e-3
    if prior == "tgv":
        ew = rel(rec.buffer("w").cpu().numpy(), X[1:4])
        print(f"[spdhg] TGV rel err u {rel(x.cpu().numpy(), X[0]):.3e} w {ew:.3e}", flush=True)
        assert ew <= 1e-3
    psi_o = prob.objective(X)
    assert abs(rec.objective().cpu().numpy()[0] - psi_o) <= 1e-4 * abs(psi_o)


def test_zero_counts(P, small3d):
    """No counts at all (b = 0): the minimiser is x = 0, which the oracle reaches exactly;
    the KL-dual prox degenerates to min(w, 1)."""
    print("[spdhg] small3d zero counts", flush=True)
    d = dict(small3d)
    d["b"] = np.zeros_like(small3d["b"])
    prob, st, rec, x = run_pair(P, d, 6, "tv", 10, seed=43, sampling="balanced", alpha=0.05)
    xo = prob.reported(st)[0]
    assert np.max(np.abs(xo)) == 0.0
    assert np.max(np.abs(x.cpu().numpy())) <= 1e-6 * np.max(np.abs(small3d["x_true"]))
    psi_o = prob.objective(xo[None])
    assert abs(rec.objective().cpu().numpy()[0] - psi_o) <= 1e-4 * abs(psi_o)


def test_scalar_steps_norms(P, small3d):
    prob, _, rec, _ = run_pair(P, small3d, 3, "tv", 0, seed=5, precond=False)
    for i in range(3):
        _, _, nrm = rec.block_info(i)
        assert nrm == pytest.approx(prob.norms[i], rel=1e-5)


def test_rerun_bitwise_and_checkpoint(P, c1):
    g = c1["geom"]
    t = {k: dev(c1[k]) for k in ("b", "r", "mult")}
    prm = P.cparams(10, "tv", "balanced", seed=99)
    xs = []
    for _ in range(2):
        x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
        rec = P.Reconstruction(g, prm, t["b"], t["r"], t["mult"], x)
        rec.epoch(5)
        torch.cuda.synchronize()
        xs.append(x.cpu().numpy())
    np.testing.assert_array_equal(xs[0], xs[1])
    # checkpoint after 2 epochs, continue 3; restore, continue 3 again
    x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
    rec = P.Reconstruction(g, prm, t["b"], t["r"], t["mult"], x)
    rec.epoch(2)
    snap = rec.save_state()
    rec.epoch(3)
    torch.cuda.synchronize()
    a = x.cpu().numpy()
    np.testing.assert_array_equal(a, xs[0])
    rec.iterate(7)  # move on, then restore
    rec.load_state(snap)
    rec.epoch(3)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(x.cpu().numpy(), a)


@pytest.mark.parametrize("prior", ["tv", "tgv"])
def test_graph_epochs_bitwise(P, small3d, prior):
    """Epochs recorded into HIP graphs give bitwise the eager result (three graphs in a
    row, with eager work and synchronisation between them)."""
    g = small3d["geom"]
    t = {k: dev(small3d[k]) for k in ("b", "r", "mult")}
    prm = P.cparams(6, prior, "balanced", alpha=0.05, alpha1=0.025, seed=21)
    xs = []
    for graph in (False, True):
        x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
        rec = P.Reconstruction(g, prm, t["b"], t["r"], t["mult"], x)
        for _ in range(3):
            if graph:
                rec.epoch_graph(1)
            else:
                rec.epoch(1)
            torch.cuda.synchronize()
            _ = rec.objective().cpu()  # eager work between the graphs
        xs.append(x.cpu().numpy())
    np.testing.assert_array_equal(xs[0], xs[1])


def test_domain_errors(P, c1):
    from paper_1808_07150_amd.spdhg import SpdhgError
    g = c1["geom"]
    b = c1["b"].copy()
    b[3, 0, 40] = -1.0
    x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
    with pytest.raises(SpdhgError) as e:
        P.Reconstruction(g, P.cparams(10, "tv"), dev(b), dev(c1["r"]), dev(c1["mult"]), x)
    assert e.value.code == -3
    # b > 0 with r = 0 on a bin no voxel reaches: objective infinite for every image
    r = c1["r"].copy()
    b = c1["b"].copy()
    r[0, 0, 0] = 0.0
    b[0, 0, 0] = 3.0
    with pytest.raises(SpdhgError) as e:
        P.Reconstruction(g, P.cparams(10, "tv"), dev(b), dev(r), dev(c1["mult"]), x)
    assert e.value.code == -3
    # mult < 0 is outside the model; mult = 0 (zero efficiency, e.g. a detector gap) is a
    # zero row of A: rejected only where b > 0 and r = 0 make the objective infinite
    mult = c1["mult"].copy()
    mult[2, 0, 30] = -0.5
    with pytest.raises(SpdhgError) as e:
        P.Reconstruction(g, P.cparams(10, "tv"), dev(c1["b"]), dev(c1["r"]), dev(mult), x)
    assert e.value.code == -3
    mult = c1["mult"].copy()
    b, r = c1["b"].copy(), c1["r"].copy()
    mult[2, 0, 30] = 0.0
    b[2, 0, 30], r[2, 0, 30] = 4.0, 0.0
    with pytest.raises(SpdhgError) as e:
        P.Reconstruction(g, P.cparams(10, "tv"), dev(b), dev(r), dev(mult), x)
    assert e.value.code == -3
    b[2, 0, 30] = 0.0
    P.Reconstruction(g, P.cparams(10, "tv"), dev(b), dev(r), dev(mult), x).close()


def _batch_problems():
    """A mixed batch: 2-D slices and thin 3-D slabs, different subset counts and priors."""
    specs = [(synth.slice_2d(48), 8, "tv", 1e5, 101), (synth.slice_2d(64), 12, "none", 3e5, 102),
             (synth.small_3d(nxy=40, nz=9, n_rad=44, n_ang=24, v=5.0, tan1=0.3), 6, "tv", 2e5, 103),
             (synth.Geometry(nx=40, ny=40, nz=33, vx=5.0, vy=5.0, vz=5.0, n_rad=44, d_rad=5.0,
                             n_ang=24, seg_planes=(33, 29, 29), seg_tan=(0.0, 0.25, -0.25)),
              8, "tv", 5e5, 104),
             (synth.slice_2d(48), 16, "tv", 1e6, 105)]
    out = []
    for g, m, prior, counts, seed in specs:
        d = synth.brain_problem(g, seed, counts)
        out.append((g, m, prior, d, seed))
    return out


@pytest.mark.parametrize("graph", [False, True])
def test_batch_bitwise_solo(P, graph):
    """Batched epochs (worker streams, optionally one HIP graph) equal solo runs bitwise."""
    probs = _batch_problems()

    def make(g, m, prior, d, seed):
        t = {k: dev(d[k]) for k in ("b", "r", "mult")}
        x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
        rec = P.Reconstruction(g, P.cparams(m, prior, "balanced", alpha=0.05, seed=seed),
                               t["b"], t["r"], t["mult"], x)
        return rec, x

    solo = []
    for pr in probs:
        rec, x = make(*pr)
        rec.epoch(3)
        torch.cuda.synchronize()
        solo.append(x.cpu().numpy())
    recs, xs = zip(*[make(*pr) for pr in probs])
    for _ in range(3):
        P.batch_epoch(list(recs), 1, n_streams=3, graph=graph)
        torch.cuda.synchronize()
    for a, x in zip(solo, xs):
        np.testing.assert_array_equal(x.cpu().numpy(), a)


def test_autotune_keeps_results(P, c1):
    """The autotuner only changes the ray-bundle split of the projection: iterates stay
    within FP32 summation-order differences of the untuned run."""
    g = c1["geom"]
    t = {k: dev(c1[k]) for k in ("b", "r", "mult")}
    prm = P.cparams(10, "tv", "balanced", seed=8)
    outs = []
    for tune in (False, True):
        x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
        rec = P.Reconstruction(g, prm, t["b"], t["r"], t["mult"], x)
        if tune:
            split, ms = rec.autotune()
            assert split in (1, 2, 4, 8, 20, 40) and ms > 0
        rec.epoch(5)
        torch.cuda.synchronize()
        outs.append(x.cpu().numpy())
    assert rel(outs[1], outs[0]) <= 1e-5


@pytest.mark.parametrize("split", [1, 2, 4, 8, 20, 40])
def test_forward_splits_parity(P, tall3d, split):
    """Every ray-bundle tiling of the subset projection (primary-step splits 1..8, plane
    splits 20/40) reproduces the oracle's iterates."""
    print(f"[spdhg] tall3d TV split={split}", flush=True)
    g = tall3d["geom"]
    prob = S.Problem(g, tall3d["b"], tall3d["r"], tall3d["mult"], n_subsets=4, prior="tv",
                     alpha=0.05, sampling="balanced", precond=True)
    t = {k: dev(tall3d[k]) for k in ("b", "r", "mult")}
    x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
    rec = P.Reconstruction(g, P.cparams(4, "tv", "balanced", True, alpha=0.05, seed=17),
                           t["b"], t["r"], t["mult"], x)
    rec.set_tuning(split)
    st = S.spdhg(prob, 6 * prob.iters_per_epoch(), seed=17)
    rec.epoch(6)
    torch.cuda.synchronize()
    xo = prob.reported(st)[0]
    assert rel(x.cpu().numpy(), xo) <= 1e-3


@pytest.mark.parametrize("prior,split_T", [("tv", False), ("tgv", False), ("tgv", True)])
def test_custom_sampling_parity(P, small3d, prior, split_T):
    """A constant tuned distribution (prior share 0.3; TGV block n 0.05 of it) and, for
    TGV, steps per variable (block n's scalar step caps w only): same block sequence, step
    maps and iterates as the oracle."""
    print(f"[spdhg] small3d custom sampling {prior} split_T={split_T}", flush=True)
    g = small3d["geom"]
    kw = dict(p_prior=0.3, p_tgv_n=0.05 if prior == "tgv" else 0.0, split_T=split_T)
    prob = S.Problem(g, small3d["b"], small3d["r"], small3d["mult"], n_subsets=6, prior=prior,
                     alpha=0.05, alpha1=0.025, sampling="custom", precond=True, **kw)
    t = {k: dev(small3d[k]) for k in ("b", "r", "mult")}
    x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
    rec = P.Reconstruction(g, P.cparams(6, prior, "custom", True, alpha=0.05, alpha1=0.025,
                                        seed=61, **kw), t["b"], t["r"], t["mult"], x)
    try:
        assert rec.iters_per_epoch == prob.iters_per_epoch()
        for i in range(prob.n):
            assert rec.block_info(i)[1] == prob.p[i]
        T = rec.buffer("T").cpu().numpy()
        assert rel(T, prob.T[0]) <= 1e-5
        st = S.spdhg(prob, 8 * prob.iters_per_epoch(), seed=61)
        rec.epoch(8)
        torch.cuda.synchronize()
        X = prob.reported(st)
        assert rel(x.cpu().numpy(), X[0]) <= 1e-3
        if prior == "tgv":
            assert rel(rec.buffer("w").cpu().numpy(), X[1:4]) <= 1e-3
        psi_o = prob.objective(X)
        assert abs(rec.objective().cpu().numpy()[0] - psi_o) <= 1e-4 * abs(psi_o)
    finally:
        rec.close()


def test_objective_failure_flag(P, c1):
    """The objective's failure flag counts non-finite voxels: 0 for a healthy iterate; a
    checkpoint whose image carries a NaN and an Inf, loaded back, raises it to 2 (and the
    objective itself is no longer finite)."""
    g = c1["geom"]
    t = {k: dev(c1[k]) for k in ("b", "r", "mult")}
    x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
    rec = P.Reconstruction(g, P.cparams(10, "tv", "balanced", seed=3), t["b"], t["r"],
                           t["mult"], x)
    try:
        rec.epoch(2)
        out = rec.objective().cpu().numpy()
        assert out[3] == 0.0 and np.isfinite(out[0])
        buf = rec.save_state()
        img = buf[:4 * g.n_vox].view(torch.float32)  # the image is the first array
        img[5] = float("nan")
        img[17] = float("inf")
        rec.load_state(buf)
        out = rec.objective().cpu().numpy()
        assert out[3] == 2.0 and not np.isfinite(out[0])
    finally:
        rec.close()


def test_persistent_graph_mixed_batch(P):
    """One persistent epoch graph (instantiated once) over problems of different shapes,
    subset counts and priors (TV, no prior, TGV): three graph epochs, with eager objective
    evaluations and synchronisations between them, equal solo epochs bitwise; a fourth
    epoch eager afterwards continues exactly."""
    probs = _batch_problems()[:4]
    specs = [(g, m, prior if j != 2 else "tgv", d, seed) for j, (g, m, prior, d, seed)
             in enumerate(probs)]

    def make(g, m, prior, d, seed):
        t = {k: dev(d[k]) for k in ("b", "r", "mult")}
        x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
        rec = P.Reconstruction(g, P.cparams(m, prior, "balanced", alpha=0.05, alpha1=0.025,
                                            seed=seed), t["b"], t["r"], t["mult"], x)
        return rec, x

    solo = []
    for sp in specs:
        rec, x = make(*sp)
        rec.epoch(4)
        torch.cuda.synchronize()
        solo.append(x.cpu().numpy())
        rec.close()
    made = [make(*sp) for sp in specs]
    graph = P.EpochGraph([r for r, _ in made])
    try:
        for _ in range(3):
            graph.epoch(1)
            torch.cuda.synchronize()
            for r, _ in made:
                _ = r.objective().cpu()
    finally:
        graph.close()
    for (r, x), a in zip(made, solo):
        r.epoch(1)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(x.cpu().numpy(), a)
        r.close()


@pytest.mark.parametrize("gather", [1, 2, 3])
def test_gather_tilings_parity(P, tall3d, gather):
    """Every tiling of the gather backprojection (strips of 10 columns, one or four
    primary indices per workgroup (13 rows: a ragged last group), whole columns)
    reproduces the oracle's iterates; the autotuner picks one of them."""
    print(f"[spdhg] tall3d TV gather={gather}", flush=True)
    g = tall3d["geom"]
    prob = S.Problem(g, tall3d["b"], tall3d["r"], tall3d["mult"], n_subsets=4, prior="tv",
                     alpha=0.05, sampling="balanced", precond=True)
    t = {k: dev(tall3d[k]) for k in ("b", "r", "mult")}
    x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
    rec = P.Reconstruction(g, P.cparams(4, "tv", "balanced", True, alpha=0.05, seed=19),
                           t["b"], t["r"], t["mult"], x)
    try:
        rec.set_gather(gather)
        assert rec.tuning()[1] == gather
        st = S.spdhg(prob, 6 * prob.iters_per_epoch(), seed=19)
        rec.epoch(6)
        torch.cuda.synchronize()
        assert rel(x.cpu().numpy(), prob.reported(st)[0]) <= 1e-3
        split, ms = rec.autotune()
        assert rec.tuning() in ((split, 1), (split, 2), (split, 3)) and ms > 0
    finally:
        rec.close()


def test_strip_workgroup_rows_bitwise(P, tall3d):
    """Strips grouped four primary indices to a workgroup compute exactly what one strip
    per workgroup computes (same arithmetic per strip): iterates bitwise equal."""
    g = tall3d["geom"]
    t = {k: dev(tall3d[k]) for k in ("b", "r", "mult")}
    out = []
    for gather in (1, 3):
        print(f"[spdhg] tall3d TV strips, gather={gather}", flush=True)
        x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
        rec = P.Reconstruction(g, P.cparams(4, "tv", "balanced", True, alpha=0.05, seed=5),
                               t["b"], t["r"], t["mult"], x)
        try:
            rec.set_gather(gather)
            rec.epoch(3)
            torch.cuda.synchronize()
            out.append(x.cpu().numpy())
        finally:
            rec.close()
    np.testing.assert_array_equal(out[0], out[1])


@pytest.mark.parametrize("name", ["span11_3d", "maxnz3d"])
def test_walk_runs_bitwise(P, name, request):
    """The forward walk's runs of consecutive planes per lane and its interleaved rays give
    bitwise the same iterates and objective (split 1 and 4: with and without the partial
    sums of several wavefronts)."""
    d = request.getfixturevalue(name)
    g = d["geom"]
    t = {k: dev(d[k]) for k in ("b", "r", "mult")}
    prm = P.cparams(4, "tv", "balanced", alpha=0.05, seed=41)
    for split in (1, 4):
        out = []
        for interleave in (False, True):
            x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
            rec = P.Reconstruction(g, prm, t["b"], t["r"], t["mult"], x)
            rec.set_tuning(split)
            rec.set_walk(interleave)
            rec.epoch(2)
            torch.cuda.synchronize()
            out.append((x.cpu().numpy(), rec.objective().cpu().numpy(),
                        rec.buffer("y").cpu().numpy()))
            rec.close()
        for a, b in zip(out[0], out[1]):
            np.testing.assert_array_equal(a, b)


def test_graph_epochs_async_then_eager(P, small3d):
    """Graph epochs return before the GPU has run them: three graph epochs launched back
    to back and an eager epoch right after, with no synchronisation in between, give the
    result of four eager epochs bitwise (the stream orders them; the graph's two copies
    alternate, each waiting for its own previous run)."""
    g = small3d["geom"]
    t = {k: dev(small3d[k]) for k in ("b", "r", "mult")}
    prm = P.cparams(6, "tv", "balanced", alpha=0.05, seed=23)
    xs = []
    for graph in (False, True):
        x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
        rec = P.Reconstruction(g, prm, t["b"], t["r"], t["mult"], x)
        if graph:
            for _ in range(3):
                rec.epoch_graph(1)
            rec.epoch(1)
        else:
            rec.epoch(4)
        torch.cuda.synchronize()
        xs.append((x.cpu().numpy(), rec.buffer("z").cpu().numpy()))
        rec.close()
    for a, b in zip(xs[0], xs[1]):
        np.testing.assert_array_equal(a, b)


def test_profiling_kinds(P, tall3d):
    """Per-kernel events limited to one kernel kind: the same seed gives the same image
    bitwise, the timed kind has the launch count of a run that times every kind, and the
    other kinds record nothing; a mask without a kind is refused."""
    from paper_1808_07150_amd.spdhg import SpdhgError
    g = tall3d["geom"]
    t = {k: dev(tall3d[k]) for k in ("b", "r", "mult")}
    prm = P.cparams(8, "tv", "balanced", alpha=0.05, seed=29)
    out = {}
    for kinds in (P.spdhg.PROF_KINDS, ("bwd",)):
        print(f"[spdhg] tall3d TV, events around {kinds}", flush=True)
        x = torch.zeros(g.image_shape, dtype=torch.float32, device="cuda:0")
        rec = P.Reconstruction(g, prm, t["b"], t["r"], t["mult"], x)
        try:
            rec.set_profiling(True, kinds=kinds)
            rec.epoch(2)
            prof = rec.profile()
            rec.set_profiling(False)
            torch.cuda.synchronize()
            out[len(kinds)] = (x.cpu().numpy(), prof)
            if len(kinds) == 1:
                with pytest.raises(SpdhgError):
                    rec.set_profiling(True, kinds=())
        finally:
            rec.close()
    (x_all, p_all), (x_one, p_one) = out[3], out[1]
    np.testing.assert_array_equal(x_all, x_one)
    assert p_all["fwd"][1] > 0 and p_all["prior"][1] > 0 and p_all["bwd"][1] > 0
    assert p_one["bwd"][1] == p_all["bwd"][1] and p_one["bwd"][0] > 0
    assert p_one["fwd"] == (0.0, 0) and p_one["prior"] == (0.0, 0)
