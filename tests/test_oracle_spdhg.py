"""Pins of the oracle's algorithms against what the paper and convex analysis fix:

* SPDHG with one block and p = 1 is PDHG (remark after Theorem 2), bit for bit;
* PDHG reaches a relative duality gap below 1e-8 on tiny TV and ML problems;
* SPDHG converges to the PDHG minimiser from different seeds and starts (Theorem 1);
* both step rules satisfy ||S_i^1/2 A_i T^1/2||^2 < p_i (Theorem 1, Theorem 2);
* one voxel: the minimiser solves a scalar equation (bisection);
* the ML minimiser is a fixed point of MLEM (eq. MLEM);
* TGV: the primal-dual fixed-point residual vanishes at the PDHG limit.
"""
import math

import numpy as np
import pytest

from oracle import priors
from oracle import projector as proj
from oracle import spdhg as S
from synth import Geometry


def tiny_problem(seed=3, scale=10.0, nxy=8, n_ang=12, n_rad=12, nz=1, segs=None):
    if segs is None:
        g = Geometry(nx=nxy, ny=nxy, nz=nz, vx=4, vy=4, vz=4, n_rad=n_rad, d_rad=4,
                     n_ang=n_ang)
    else:
        g = Geometry(nx=nxy, ny=nxy, nz=nz, vx=4, vy=4, vz=4, n_rad=n_rad, d_rad=4,
                     n_ang=n_ang, seg_planes=segs[0], seg_tan=segs[1])
    rng = np.random.default_rng(seed)
    xt = rng.uniform(0.5, 2, g.image_shape)
    mult = scale * rng.uniform(0.8, 1.2, g.sino_shape)
    ax = mult * proj.forward(g, xt)
    r = np.full(g.sino_shape, 0.1 * ax.mean())
    b = rng.poisson(ax + r).astype(float)
    return g, b, r, mult


def test_spdhg_one_block_equals_pdhg_bitwise():
    g, b, r, mult = tiny_problem()
    prob = S.Problem(g, b, r, mult, n_subsets=1, prior="none")
    assert prob.p == [1.0]
    st1 = S.spdhg(prob, 30, seed=1)
    pp = S.pdhg_problem(prob, weights=[1.0])
    st2 = S.pdhg(pp, 30)
    np.testing.assert_array_equal(prob.reported(st1), pp.reported(st2))
    np.testing.assert_array_equal(st1["y"][0], st2["y"][0])


def _solve_pdhg(prob, tol=1e-9, max_iter=40000):
    pp = S.pdhg_problem(prob)
    st = pp.new_state()
    while st["k"] < max_iter:
        st = S.pdhg(pp, 500, state=st)
        xr = pp.reported(st)
        if S.duality_gap(pp, xr, st, 2 * xr.max() + 1) <= tol * abs(pp.objective(xr)):
            break
    return pp, st


def test_pdhg_gap_tv():
    g, b, r, mult = tiny_problem()
    prob = S.Problem(g, b, r, mult, n_subsets=4, prior="tv", alpha=0.5)
    pp, st = _solve_pdhg(prob, tol=1e-9)
    xr = pp.reported(st)
    gap = S.duality_gap(pp, xr, st, 2 * xr.max() + 1)
    assert gap <= 1e-8 * pp.objective(xr)


def test_pdhg_gap_atv():
    """aTV (alpha ||grad u||_{1,1}, Section 4.3): PDHG with the box projection as the dual
    prox closes the gap, whose dual part is the indicator of that same box and whose
    primal part charges alpha ||grad u||_1.  A dual prox onto any other box leaves a gap
    of (alpha - alpha') ||grad x*||_1 or an infeasible dual."""
    g, b, r, mult = tiny_problem()
    prob = S.Problem(g, b, r, mult, n_subsets=4, prior="atv", alpha=0.5)
    pp, st = _solve_pdhg(prob, tol=1e-9)
    xr = pp.reported(st)
    gap = S.duality_gap(pp, xr, st, 2 * xr.max() + 1)
    assert gap <= 1e-8 * pp.objective(xr)
    # the prior dual sits on the box's faces wherever the gradient is non-zero
    q = st["yp"][0]
    gr = priors.grad(xr[0])
    on = np.abs(gr) > 1e-6
    assert np.any(on)
    np.testing.assert_allclose(np.abs(q[on]), 0.5, rtol=1e-6)


def test_pdhg_gap_ml_interior():
    """High counts on a well-conditioned 4x4 problem (cond(A) ~ 26): the ML solution is
    interior and PDHG converges linearly."""
    g, b, r, mult = tiny_problem(scale=2000.0, nxy=4, n_ang=12, n_rad=8)
    prob = S.Problem(g, b, r, mult, n_subsets=4, prior="none")
    pp, st = _solve_pdhg(prob, tol=1e-9)
    xr = pp.reported(st)
    assert xr.min() > 0
    gap = S.duality_gap(pp, xr, st, 2 * xr.max() + 1)
    assert gap <= 1e-8 * pp.objective(xr)
    # the ML minimiser is an MLEM fixed point (eq. MLEM)
    u = xr[0]
    np.testing.assert_allclose(S.mlem_step(prob, u), u, rtol=1e-7)


@pytest.mark.parametrize("sampling,precond,epochs", [("uniform", True, 1000),
                                                     ("balanced", True, 1000),
                                                     ("balanced", False, 1600)])
def test_spdhg_converges_to_pdhg_minimiser(sampling, precond, epochs):
    g, b, r, mult = tiny_problem()
    prob = S.Problem(g, b, r, mult, n_subsets=4, prior="tv", alpha=0.5, sampling=sampling,
                     precond=precond)
    pp, st = _solve_pdhg(prob, tol=1e-10)
    xstar = pp.reported(st)[0]
    rng = np.random.default_rng(0)
    for seed, x0 in [(1, None), (2, rng.uniform(0, 3, (1,) + g.image_shape))]:
        s2 = S.spdhg(prob, epochs * prob.iters_per_epoch(), seed=seed, x0=x0)
        x = prob.reported(s2)[0]
        assert np.linalg.norm(x - xstar) / np.linalg.norm(xstar) < 1e-6


def _dense_op(apply, in_shape):
    n = int(np.prod(in_shape))
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(np.asarray(apply(e.reshape(in_shape))).ravel())
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("precond", [True, False])
@pytest.mark.parametrize("prior,sampling,split_T", [
    ("tv", "balanced", False), ("tgv", "balanced", False),
    # tuned constant sampling (prior share 0.3, TGV block n with 0.05 of it) and TGV steps
    # per variable: block n (0, E) caps only the step of w
    ("tv", "custom", False), ("tgv", "custom", False), ("tgv", "custom", True)])
def test_step_size_condition(precond, prior, sampling, split_T):
    # low sensitivities (mult scale 0.5) make the data steps larger than block n's, so that
    # the TGV split decides T_u
    g, b, r, mult = tiny_problem(nxy=5, n_ang=6, n_rad=8, scale=0.5 if split_T else 10.0)
    prob = S.Problem(g, b, r, mult, n_subsets=3, prior=prior, alpha=0.5, alpha1=0.25,
                     sampling=sampling, precond=precond, p_prior=0.3, p_tgv_n=0.05,
                     split_T=split_T)
    if split_T:
        # the split matters here: block n's scalar step is the smallest prior step and
        # caps w, while u may take the larger step of block n-1
        t_prev = 0.99 * prob.p[prob.m] / prob.norms[prob.m]
        t_n = 0.99 * prob.p[prob.m + 1] / prob.norms[prob.m + 1]
        assert t_n < t_prev
        assert np.max(prob.T[0]) > t_n and np.max(prob.T[1:4]) <= t_n
    ishape = prob.image_shape()
    Th = np.sqrt(prob.T.ravel())
    for i in range(prob.n):
        if i < prob.m:
            A = _dense_op(lambda X: prob.A_data(i, X), ishape)
            sig = np.broadcast_to(prob.sigma[i], prob.sub_b[i].shape).ravel()
        else:
            j = i - prob.m
            A = _dense_op(lambda X: prob.A_prior(j, X), ishape)
            sig = np.full(A.shape[0], prob.prior_sigma[j])
        M = np.sqrt(sig)[:, None] * A * Th[None, :]
        assert np.linalg.norm(M, 2) ** 2 < prob.p[i]


def test_single_voxel_closed_form():
    """One voxel: Psi(x) = sum_j phi_j(a_j x) and the minimiser solves
    sum_j a_j (1 - b_j / (a_j x + r_j)) = 0 (found by bisection)."""
    g = Geometry(nx=1, ny=1, nz=1, vx=4, vy=4, vz=4, n_rad=3, d_rad=2, n_ang=6)
    rng = np.random.default_rng(5)
    mult = rng.uniform(0.5, 1.5, g.sino_shape)
    r = np.full(g.sino_shape, 0.3)
    b = rng.integers(1, 9, g.sino_shape).astype(float)
    a = (mult * proj.forward(g, np.ones(g.image_shape))).ravel()
    bb, rr = b.ravel(), r.ravel()
    lo, hi = 0.0, 1e3
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.sum(a * (1 - bb / (a * mid + rr))) > 0:
            hi = mid
        else:
            lo = mid
    prob = S.Problem(g, b, r, mult, n_subsets=2, prior="none")
    pp, st = _solve_pdhg(prob, tol=1e-12)
    assert float(pp.reported(st).ravel()[0]) == pytest.approx(0.5 * (lo + hi), rel=1e-8)


def test_tgv_kkt_residual():
    g, b, r, mult = tiny_problem(nxy=6, n_ang=8, n_rad=10)
    prob = S.Problem(g, b, r, mult, n_subsets=2, prior="tgv", alpha=0.5, alpha1=0.25)
    pp = S.pdhg_problem(prob)
    st = S.pdhg(pp, 20000)
    xr = pp.reported(st)
    assert S.kkt_residual(pp, xr, st) < 1e-10


def test_dtv_with_flat_side_image_is_tv():
    """eta -> infinity gives D = I: the dTV iterates equal the TV iterates."""
    g, b, r, mult = tiny_problem()
    side = np.random.default_rng(9).random(g.image_shape)
    p1 = S.Problem(g, b, r, mult, n_subsets=4, prior="tv", alpha=0.5, sampling="balanced")
    p2 = S.Problem(g, b, r, mult, n_subsets=4, prior="dtv", alpha=0.5, side=side, eta=1e12,
                   sampling="balanced")
    p2.prior_sigma = list(p1.prior_sigma)
    p2.T = p1.T.copy()
    s1 = S.spdhg(p1, 50, seed=4)
    s2 = S.spdhg(p2, 50, seed=4)
    np.testing.assert_allclose(p2.reported(s2), p1.reported(s1), rtol=1e-10, atol=1e-12)


def test_objective_definitions():
    g, b, r, mult = tiny_problem()
    prob = S.Problem(g, b, r, mult, n_subsets=3, prior="tv", alpha=0.5)
    x = np.random.default_rng(1).uniform(0, 2, (1,) + g.image_shape)
    ax = mult * proj.forward(g, x[0])
    s = ax + r
    with np.errstate(divide="ignore", invalid="ignore"):
        data = np.sum(s - b + np.where(b > 0, b * np.log(b / s), 0.0))
    tv = 0.5 * np.sum(np.sqrt(np.sum(priors.grad(x[0]) ** 2, axis=0)))
    assert prob.objective(x) == pytest.approx(data + tv, rel=1e-12)
    assert math.isinf(prob.objective(-x))


def test_epoch_lengths():
    g, b, r, mult = tiny_problem()
    assert S.Problem(g, b, r, mult, n_subsets=4, prior="none").iters_per_epoch() == 4
    assert S.Problem(g, b, r, mult, n_subsets=4, prior="tv").iters_per_epoch() == 5
    assert S.Problem(g, b, r, mult, n_subsets=4, prior="tv",
                     sampling="balanced").iters_per_epoch() == 8


def test_osem_consistent_data_is_a_fixed_point():
    """With noise-free data b = P x + r every subset update leaves x unchanged (each ratio
    b / (P_i x + r) is 1, and P_i^T 1 / P_i^T 1 = 1 on the sensitivity's support), eq. OSEM;
    a wrong subset, factor or ordering breaks it."""
    g, _, r, mult = tiny_problem(seed=5, nz=3, segs=((3, 1, 1), (0.0, 0.3, -0.3)))
    rng = np.random.default_rng(9)
    xt = rng.uniform(0.5, 2.0, g.image_shape)
    b = mult * proj.forward(g, xt) + r
    prob = S.Problem(g, b, r, mult, n_subsets=4, prior="none")
    for i in range(4):
        np.testing.assert_allclose(S.osem_step(prob, xt, i), xt, rtol=1e-12)


def test_osem_subset_count_identity():
    """sum_v (P_i^T 1)_v x'_v = sum_{j in S_i} b_j (P_i x)_j / (P_i x + r)_j for the update x'
    of subset i (multiply eq. OSEM by P_i^T 1 and sum over voxels)."""
    g, b, r, mult = tiny_problem(seed=6)
    prob = S.Problem(g, b, r, mult, n_subsets=3, prior="none")
    rng = np.random.default_rng(10)
    x = rng.uniform(0.2, 3.0, g.image_shape)
    for i in range(3):
        ang = prob.angles[i]
        xn = S.osem_step(prob, x, i)
        sens = proj.backward(g, prob.sub_mult[i], ang)
        px = prob.sub_mult[i] * proj.forward(g, x, ang)
        lhs = float(np.sum(sens * xn))
        rhs = float(np.sum(prob.sub_b[i] * px / (px + prob.sub_r[i])))
        assert lhs == pytest.approx(rhs, rel=1e-12)


def test_mlem_is_osem_with_one_subset_and_increases_likelihood():
    """OSEM with one subset is MLEM (eq. MLEM); MLEM never decreases the Poisson
    likelihood (the EM property)."""
    g, b, r, mult = tiny_problem(seed=7)
    prob1 = S.Problem(g, b, r, mult, n_subsets=1, prior="none")
    u = np.ones(g.image_shape)
    ll = S.poisson_loglik(prob1, u)
    for _ in range(20):
        un = S.mlem_step(prob1, u)
        np.testing.assert_array_equal(S.osem_step(prob1, u, 0), un)
        ll_new = S.poisson_loglik(prob1, un)
        assert ll_new >= ll - 1e-9 * abs(ll)
        u, ll = un, ll_new


@pytest.mark.parametrize("precond", [True, False])
def test_zero_efficiency_bins_drop_out(precond):
    """A bin with mult = 0 (a detector gap) has a zero row of A: its term phi_j(0) is a
    constant, its dual never moves, and the iterates do not depend on its data.  Two
    problems that differ only in b, r on such bins (b = 0, r = 0 against b = 0, r = 5)
    give bitwise equal iterates; negative mult is rejected."""
    g, b, r, mult = tiny_problem(seed=9)
    gap = np.zeros(g.sino_shape, dtype=bool)
    gap[:, :, 2] = True
    gap[3::4, :, 7] = True
    mult = np.where(gap, 0.0, mult)
    b = np.where(gap, 0.0, b)
    out = []
    for rv in (0.0, 5.0):
        rr = np.where(gap, rv, r)
        prob = S.Problem(g, b, rr, mult, n_subsets=4, prior="tv", alpha=0.05,
                         sampling="balanced", precond=precond)
        st = S.spdhg(prob, 3 * prob.iters_per_epoch(), seed=4)
        x = prob.reported(st)[0]
        assert np.all(np.isfinite(x))
        out.append(x)
    np.testing.assert_array_equal(out[0], out[1])
    with pytest.raises(ValueError):
        S.Problem(g, b, r, np.where(gap, -1.0, mult), n_subsets=4, prior="tv", alpha=0.05)
