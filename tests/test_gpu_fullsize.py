"""Single iterations of Algorithm 2 at full mMR size (344 x 344 x 127, sinogram 344 x 252
x 837; the launch configuration of the benchmark) against the FP64 oracle applied to the
same state.

Data iteration: the oracle's own Algorithm 2 loop (oracle.spdhg.spdhg, one iteration of
the drawn subset: forward projection, KL-dual prox, backprojection, z and z-bar, then the
next iteration's primal step) from the library's state and step sizes.

Prior iterations: one TV and one TGV iteration (both blocks) against the oracle's
operators:

The state is taken from the library after k iterations (k = the first iteration whose
SplitMix64 draw is a prior block), the GPU runs iteration k, and the oracle recomputes
the dual step to the extrapolation of that iteration and the primal step of the next (which the library fuses into the
same launch) from the FP32 snapshot:

  TV (Section 4.3, eq. setting TV):  y' = P_alpha(y + sigma grad x),  dz = grad^T (y' - y)
  TGV block n-1:  q1' = P_alpha0(q1 + sigma (grad u - w)),  dz_u = grad^T dq1,  dz_w = -dq1
  TGV block n:    q2' = P_alpha1(q2 + sigma E w),           dz_u = 0,  dz_w = E^T dq2
  then z' = z + dz and x' = prox_g(x - T (z' + dz / p))  (for w: no prox, scalar T_w).

Bar: new duals within 1e-5 of their scale; the updates of z, x (and w, z_w) within 1e-3
of the update's scale plus two FP32 ulps of the result (FP32 against FP64)."""
import numpy as np
import pytest

import synth
from oracle import priors as PR
from oracle import prox as PX
from oracle import sampling as SA
from oracle import spdhg as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_1808_07150_amd as lib
    lib.load_library()
    return lib


@pytest.fixture(scope="module")
def mmr_inputs():
    g = synth.mmr()
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(18080700)
    shp = g.sino_shape
    mult = torch.rand(shp, device="cuda:0", generator=gen) * 0.4 + 0.8
    b = torch.floor(torch.rand(shp, device="cuda:0", generator=gen) * 4.0)
    r = torch.full(shp, 0.3, device="cuda:0")
    x0 = torch.rand(g.image_shape, device="cuda:0", generator=gen)
    return g, b, r, mult, x0


def close(got, ref, tol=1e-5):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.max(np.abs(ref))
    assert scale > 0
    err = np.max(np.abs(got - ref))
    assert err <= tol * scale, (err, scale)


def close_step(after, before, ref_after):
    """An FP32 update (after - before) against the FP64 one: within 1e-3 of the update's
    scale plus two FP32 ulps of the result's scale."""
    after, before, ref_after = (np.asarray(a, np.float64) for a in (after, before, ref_after))
    step = np.max(np.abs(ref_after - before))
    assert step > 0
    err = np.max(np.abs(after - ref_after))
    assert err <= 1e-3 * step + 2.0 ** -22 * np.max(np.abs(ref_after)), (err, step)


def snap(rec, names):
    torch.cuda.synchronize()
    return {n: rec.buffer(n).cpu().numpy().astype(np.float64) for n in names}


@pytest.mark.parametrize("prior,m,alpha,alpha1", [("tv", 21, 2e-3, 0.0),
                                                  ("tgv", 252, 2e-3, 1e-3)])
def test_mmr_prior_iteration(P, mmr_inputs, prior, m, alpha, alpha1):
    g, b, r, mult, x0 = mmr_inputs
    seed = 18080710
    n_prior = 2 if prior == "tgv" else 1
    p = SA.balanced(m, n_prior)
    blocks = SA.draw_blocks(seed, p, 400)
    # a prior iteration preceded by at least one data iteration (non-zero z)
    k = next(i for i in range(1, 400) if blocks[i] >= m and blocks[i - 1] < m)
    # TGV: test both blocks, the second at the next draw of the other block
    ks = [k]
    if prior == "tgv":
        k2 = next(i for i in range(k + 1, 400) if blocks[i] >= m and blocks[i] != blocks[k])
        ks.append(k2)
    print(f"[fullsize] {prior} m={m}: prior iterations {ks} (blocks "
          f"{[blocks[i] for i in ks]})", flush=True)
    x = x0.clone()
    prm = P.cparams(m, prior, "balanced", True, alpha=alpha, alpha1=alpha1, seed=seed)
    rec = P.Reconstruction(g, prm, b, r, mult, x)
    try:
        done = 0
        for kk in ks:
            rec.iterate(kk - done)
            done = kk
            assert rec.info()[1] == kk
            names = ["z", "T", "prior_dual"] + (["w", "q2", "zw"] if prior == "tgv" else [])
            s0 = snap(rec, names)
            x_before = x.cpu().numpy().astype(np.float64)
            blk = blocks[kk]
            sigma, pb, _ = rec.block_info(blk)
            rec.iterate(1)
            done += 1
            s1 = snap(rec, names)
            x_after = x.cpu().numpy().astype(np.float64)
            T = s0["T"]
            if prior == "tv":
                y = s0["prior_dual"]
                yn = PX.project_l2_ball(y + sigma * PR.grad(x_before), alpha)
                dz = PR.grad_adj(yn - y)
                zn = s0["z"] + dz
                close(s1["prior_dual"], yn)
                close_step(s1["z"], s0["z"], zn)
                close_step(x_after, x_before, PX.prox_nonneg(x_before - T * (zn + dz / pb)))
                continue
            # TGV: T_w is the smaller of the two prior blocks' scalar steps (rho = 0.99)
            tw = min(0.99 * rec.block_info(m + j)[1] / rec.block_info(m + j)[2]
                     for j in range(2))
            w = s0["w"]
            if blk == m:  # block n-1: A = (grad, -I)
                q = s0["prior_dual"]
                qn = PX.project_l2_ball(q + sigma * (PR.grad(x_before) - w), alpha)
                dq = qn - q
                dzu, dzw = PR.grad_adj(dq), -dq
                close(s1["prior_dual"], qn)
            else:  # block n: A = (0, E)
                q = s0["q2"]
                qn = PX.project_l2_ball(q + sigma * PR.sym_grad(w), alpha1)
                dq = qn - q
                dzu, dzw = np.zeros_like(x_before), PR.sym_grad_adj(dq)
                close(s1["q2"], qn)
            zun, zwn = s0["z"] + dzu, s0["zw"] + dzw
            if blk == m:
                close_step(s1["z"], s0["z"], zun)
            else:  # z_u is not touched by block n
                np.testing.assert_array_equal(s1["z"], s0["z"])
            close_step(s1["zw"], s0["zw"], zwn)
            close_step(x_after, x_before, PX.prox_nonneg(x_before - T * (zun + dzu / pb)))
            close_step(s1["w"], w, w - tw * (zwn + dzw / pb))
    finally:
        rec.close()


@pytest.mark.parametrize("split,gather", [(0, 0), (4, 3)])
def test_mmr_data_iteration(P, mmr_inputs, split, gather):
    """One data iteration (12 angles, nnz 3.3e9) of mMR with TV, SPDHG+: y of the subset,
    z and the next iterate against the oracle's Algorithm 2 loop; every other subset's y
    is left untouched.  Split 0 and gather 0 let the launch size choose the ray-bundle
    split and take one strip per workgroup; split 4 with gather tiling 3 (four strip rows
    per workgroup) is the benchmark's autotuned launch: fwd_wave<15, F_DUAL, 4, runs> and
    bwd_strip<B_PARTIAL / B_ITER, 1, 11> in 256-thread workgroups."""
    g, b, r, mult, x0 = mmr_inputs
    m, seed, alpha = 21, 18080720, 2e-3
    blocks = SA.draw_blocks(seed, SA.balanced(m, 1), 400)
    # a data iteration after at least one data and one prior iteration
    k = next(i for i in range(2, 400) if blocks[i] < m and any(v < m for v in blocks[:i])
             and any(v >= m for v in blocks[:i]))
    i = blocks[k]
    print(f"[fullsize] data iteration {k} (subset {i}), split {split}, gather {gather}",
          flush=True)
    x = x0.clone()
    rec = P.Reconstruction(g, P.cparams(m, "tv", "balanced", True, alpha=alpha, seed=seed),
                           b, r, mult, x)
    try:
        rec.set_tuning(split)
        rec.set_gather(gather)
        assert rec.tuning() == (split, 3 if gather == 3 else 1)
        rec.iterate(k)
        s0 = snap(rec, ["y", "z", "T", "sigma", "prior_dual"])
        x_before = x.cpu().numpy().astype(np.float64)
        prior_sigma = rec.block_info(m)[0]
        rec.iterate(1)
        s1 = snap(rec, ["y", "z"])
        x_after = x.cpu().numpy().astype(np.float64)
    finally:
        rec.close()

    class Given(S.Problem):  # the oracle's problem with the library's step sizes
        def _setup_steps(self):
            pass

    prob = Given(g, b.cpu().numpy(), r.cpu().numpy(), mult.cpu().numpy(), n_subsets=m,
                 prior="tv", alpha=alpha, sampling="balanced", precond=True)
    prob.sigma = [s0["sigma"][a] for a in prob.angles]
    prob.prior_sigma = [prior_sigma]
    prob.norms = [None] * prob.n
    prob.T = s0["T"][None]
    st = prob.new_state(x_before)  # z-bar = 0: the primal step returns x_before itself
    st["y"] = [s0["y"][a] for a in prob.angles]
    st["yp"] = [s0["prior_dual"]]
    st["z"] = s0["z"][None]
    S.spdhg(prob, 1, seed, state=st, blocks=[i])
    ang = prob.angles[i]
    # the KL-dual prox is non-expansive, so the new dual inherits the projection's error:
    # within 1e-5 of the largest sigma * (A_i x) (the projection bar) plus two FP32 ulps
    sax = prob.sigma[i] * prob.A_data(i, x_before[None])
    err = np.max(np.abs(s1["y"][ang] - st["y"][i]))
    assert err <= 1e-5 * np.max(np.abs(sax)) + 2.0 ** -22 * np.max(np.abs(st["y"][i])), err
    others = np.setdiff1d(np.arange(g.n_ang), ang)
    np.testing.assert_array_equal(s1["y"][others], s0["y"][others])
    close_step(s1["z"], s0["z"], st["z"][0])
    close_step(x_after, x_before, prob.reported(st)[0])
