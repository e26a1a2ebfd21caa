"""FP64 oracle of the SPDHG reconstruction (Algorithms 1 and 2).  Test infrastructure only.

Problem (Section 2, Problem 1 and the generic Problem 2):
    min_x  Psi(x) = sum_i f_i(A_i x) + g(x)
with data blocks f_i = D_i, A_i = P_i = diag(mult) G restricted to the angles of subset i
(equidistantly divided angles, Section 4), g = non-negativity of the activity, and
optional prior blocks:
    'none'  (ML, n = m)
    'tv'    f_n = alpha ||.||_{2,1},  A_n = grad            (eq. setting TV)
    'atv'   f_n = alpha ||.||_{1,1},  A_n = grad            (Section 4.3, anisotropic TV)
    'dtv'   f_n = alpha ||.||_{2,1},  A_n = D grad          (Section 4.3, directional TV)
    'tgv'   x = (u, w); f_{n-1} = alpha0 ||.||_{2,1}, A_{n-1} = (grad, -I);
            f_n = alpha1 ||.||_{2,1}, A_n = (0, E)          (Section 4.3, TGV)

The primal variable is stored as X[c][z][y][x] with c = 1 (u) or c = 4 (u, w0, w1, w2).

Step sizes (Theorem 2): scalar S_i = gamma rho / ||A_i||, T_i = rho p_i / (gamma ||A_i||),
or, for the data blocks (A_i >= 0), preconditioned S_i = gamma rho / (A_i 1),
T_i = rho p_i / (gamma A_i^T 1).  Prior blocks always use the scalar rule (grad has
negative entries).  T = min_i T_i elementwise over all blocks (Theorem 1).

Readings where the paper is silent: rho = 0.99 (only rho < 1 is required); rows with
A_i 1 = 0 get sigma = 0 (their dual stays 0); voxels no block constrains get T = 0;
epoch = m / sum_{i<=m} p_i iterations (expected passes over the data).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from . import priors
from . import projector as proj
from . import prox as P
from .sampling import balanced, draw_blocks, prior_share, uniform


@dataclasses.dataclass
class Problem:
    geom: object
    b: np.ndarray
    r: np.ndarray
    mult: np.ndarray
    n_subsets: int
    prior: str = "tv"
    alpha: float = 0.1          # TV / aTV / dTV weight, TGV alpha0
    alpha1: float = 0.05        # TGV alpha1
    side: Optional[np.ndarray] = None
    eta: float = 1e-2
    gamma_d: float = 1.0
    sampling: str = "uniform"   # 'uniform' | 'balanced' | 'custom'
    precond: bool = True
    gamma: float = 1.0
    rho: float = 0.99
    p_prior: float = 0.5        # 'custom': total probability of the prior blocks
    p_tgv_n: float = 0.0        # 'custom', TGV: probability of block n (0: half of p_prior)
    split_T: bool = False       # TGV: each prior block's scalar T caps only its variables

    def __post_init__(self):
        g = self.geom
        self.b = np.asarray(self.b, dtype=np.float64).reshape(g.sino_shape)
        self.r = np.asarray(self.r, dtype=np.float64).reshape(g.sino_shape)
        self.mult = np.asarray(self.mult, dtype=np.float64).reshape(g.sino_shape)
        # mult = 0 (a bin of zero efficiency, e.g. a detector gap) gives the bin a zero
        # row of A, like a ray that misses the image
        if np.any(self.b < 0) or np.any(self.r < 0) or np.any(self.mult < 0):
            raise ValueError("domain: need b >= 0, r >= 0, mult >= 0")
        m = self.n_subsets
        self.m = m
        self.n_prior = {"none": 0, "tv": 1, "atv": 1, "dtv": 1, "tgv": 2}[self.prior]
        self.n = m + self.n_prior
        self.channels = 4 if self.prior == "tgv" else 1
        self.angles = [g.subset_angles(m, i) for i in range(m)]
        self.sub_b = [self.b[a] for a in self.angles]
        self.sub_r = [self.r[a] for a in self.angles]
        self.sub_mult = [self.mult[a] for a in self.angles]
        if self.sampling == "uniform":
            self.p = uniform(self.n)
        elif self.sampling == "balanced":
            self.p = balanced(m, self.n_prior)
        elif self.sampling == "custom":
            self.p = prior_share(m, self.n_prior, self.p_prior, self.p_tgv_n)
        else:
            raise ValueError(self.sampling)
        if self.prior == "dtv":
            if self.side is None:
                raise ValueError("dTV needs a side image")
            self.xi = priors.dtv_field(np.asarray(self.side, np.float64).reshape(g.image_shape),
                                       self.eta)
        self._setup_steps()

    # ------------------------------------------------------------ operators
    def image_shape(self):
        return (self.channels,) + tuple(self.geom.image_shape)

    def A_data(self, i, X):
        """A_i X = mult * G_{S_i} u (rows of subset i, packed)."""
        return self.sub_mult[i] * proj.forward(self.geom, X[0], self.angles[i])

    def AT_data(self, i, y):
        """A_i^T y = (G_{S_i}^T (mult * y), 0)."""
        out = np.zeros(self.image_shape())
        out[0] = proj.backward(self.geom, self.sub_mult[i] * y, self.angles[i])
        return out

    def A_prior(self, j, X):
        """Operator of prior block j (0-based among the prior blocks)."""
        if self.prior in ("tv", "atv"):
            return priors.grad(X[0])
        if self.prior == "dtv":
            return priors.dgrad(X[0], self.xi, self.gamma_d)
        if self.prior == "tgv":
            if j == 0:
                return priors.grad(X[0]) - X[1:4]
            return priors.sym_grad(X[1:4])
        raise ValueError(self.prior)

    def AT_prior(self, j, q):
        out = np.zeros(self.image_shape())
        if self.prior in ("tv", "atv"):
            out[0] = priors.grad_adj(q)
        elif self.prior == "dtv":
            out[0] = priors.dgrad_adj(q, self.xi, self.gamma_d)
        elif self.prior == "tgv":
            if j == 0:
                out[0] = priors.grad_adj(q)
                out[1:4] = -q
            else:
                out[1:4] = priors.sym_grad_adj(q)
        return out

    def prior_weight(self, j):
        if self.prior == "tgv":
            return self.alpha if j == 0 else self.alpha1
        return self.alpha

    def prior_dual_prox(self, j, v):
        if self.prior == "atv":
            return P.clip_linf_ball(v, self.alpha)
        return P.project_l2_ball(v, self.prior_weight(j), axis=0)

    def prior_norm(self, j) -> float:
        shape = self.geom.image_shape
        if self.prior in ("tv", "atv"):
            return priors.grad_norm_closed_form(shape)
        if self.prior == "tgv" and j == 0:
            return math.sqrt(priors.grad_norm_closed_form(shape) ** 2 + 1.0)
        if self.prior == "tgv":
            # block n = (0, E): the closed-form bound ||E|| <= ||grad|| (Frobenius: ||E w||^2
            # <= sum_k ||grad w_k||^2), so the step condition of Theorem 1 holds for sure; a
            # truncated power iteration approaches ||E|| from below
            return priors.grad_norm_closed_form(shape)
        if self.prior == "dtv":
            return priors.power_norm(lambda u: priors.dgrad(u, self.xi, self.gamma_d),
                                     lambda q: priors.dgrad_adj(q, self.xi, self.gamma_d),
                                     priors.checkerboard(tuple(shape)), iters=200)
        raise ValueError(self.prior)

    def data_norm(self, i) -> float:
        return priors.power_norm(lambda u: self.A_data(i, u[None])[...],
                                 lambda y: self.AT_data(i, y)[0],
                                 np.ones(self.geom.image_shape))

    # ------------------------------------------------------------ step sizes
    def _setup_steps(self):
        g, gam, rho = self.geom, self.gamma, self.rho
        ishape = self.image_shape()
        Tmin = np.full(ishape, np.inf)
        self.sigma = []
        self.norms = []
        for i in range(self.m):
            if self.precond:
                a1 = self.sub_mult[i] * proj.forward(g, np.ones(g.image_shape), self.angles[i])
                with np.errstate(divide="ignore"):
                    sig = np.where(a1 > 0, gam * rho / np.where(a1 > 0, a1, 1.0), 0.0)
                at1 = proj.backward(g, self.sub_mult[i], self.angles[i])
                with np.errstate(divide="ignore"):
                    Ti = np.where(at1 > 0, rho * self.p[i] / (gam * np.where(at1 > 0, at1, 1.0)),
                                  np.inf)
                self.sigma.append(sig)
                self.norms.append(None)
                Tmin[0] = np.minimum(Tmin[0], Ti)
            else:
                nrm = self.data_norm(i)
                self.norms.append(nrm)
                self.sigma.append(gam * rho / nrm)
                Tmin[0] = np.minimum(Tmin[0], rho * self.p[i] / (gam * nrm))
        self.prior_sigma = []
        for j in range(self.n_prior):
            nrm = self.prior_norm(j)
            self.norms.append(nrm)
            self.prior_sigma.append(gam * rho / nrm)
            tj = rho * self.p[self.m + j] / (gam * nrm)
            if self.prior == "tgv" and self.split_T and j == 1:
                # block n is (0, E): it constrains the step of w only (Theorem 1 bounds
                # ||S_n^1/2 A_n T^1/2||, in which T_u does not appear)
                Tmin[1:4] = np.minimum(Tmin[1:4], tj)
            else:
                Tmin = np.minimum(Tmin, tj)
        self.T = np.where(np.isfinite(Tmin), Tmin, 0.0)

    # ------------------------------------------------------------ objective
    def data_term(self, X) -> float:
        tot = 0.0
        for i in range(self.m):
            tot += float(np.sum(P.phi(self.A_data(i, X), self.sub_b[i], self.sub_r[i])))
        return tot

    def prior_term(self, X) -> float:
        if self.prior == "none":
            return 0.0
        if self.prior == "atv":
            return self.alpha * float(np.sum(np.abs(self.A_prior(0, X))))
        return sum(self.prior_weight(j) * priors.norm_l21(self.A_prior(j, X))
                   for j in range(self.n_prior))

    def objective(self, X) -> float:
        """Psi(X) = sum_i D_i(A_i X) + prior + nonnegativity indicator (eq. Problem 1)."""
        X = np.asarray(X, np.float64).reshape(self.image_shape())
        if np.any(X[0] < 0):
            return math.inf
        return self.data_term(X) + self.prior_term(X)

    # ------------------------------------------------------------ state
    def new_state(self, x0=None):
        ishape = self.image_shape()
        X = np.zeros(ishape)
        if x0 is not None:
            X[...] = np.asarray(x0, np.float64).reshape(ishape)
        y_data = [np.zeros_like(b) for b in self.sub_b]
        y_prior = [np.zeros_like(self.A_prior(j, X)) for j in range(self.n_prior)]
        return dict(x=X, y=y_data, yp=y_prior, z=np.zeros(ishape), zbar=np.zeros(ishape), k=0)

    def prox_g(self, X):
        out = X.copy()
        out[0] = P.prox_nonneg(X[0])
        return out

    def reported(self, st):
        """Iterate after K iterations: the primal step applied once more (x = prox_g(x - T zbar))."""
        return self.prox_g(st["x"] - self.T * st["zbar"])

    def iters_per_epoch(self) -> int:
        return int(round(self.m / sum(self.p[: self.m])))


def spdhg(prob: Problem, n_iter: int, seed: int, state=None, x0=None, blocks=None):
    """Algorithm 2 (SPDHG), n_iter iterations from `state` (or a fresh one).

    Block i is drawn from the SplitMix64 stream unless `blocks` gives the sequence."""
    st = prob.new_state(x0) if state is None else state
    seq = draw_blocks(seed, prob.p, n_iter, start=st["k"]) if blocks is None else list(blocks)
    x, z, zbar = st["x"], st["z"], st["zbar"]
    for i in seq:
        x = prob.prox_g(x - prob.T * zbar)                          # primal step
        if i < prob.m:                                              # sample block i
            yi = st["y"][i]
            v = yi + prob.sigma[i] * prob.A_data(i, x)
            y_plus = P.prox_kl_dual(v, prob.sigma[i], prob.sub_b[i], prob.sub_r[i])  # dual step
            dz = prob.AT_data(i, y_plus - yi)                       # backprojected dual change
            st["y"][i] = y_plus                                     # dual update
        else:
            j = i - prob.m
            yj = st["yp"][j]
            y_plus = prob.prior_dual_prox(j, yj + prob.prior_sigma[j] * prob.A_prior(j, x))
            dz = prob.AT_prior(j, y_plus - yj)
            st["yp"][j] = y_plus
        z = z + dz                                                  # z update
        zbar = z + dz / prob.p[i]                                   # extrapolation
        st["k"] += 1
    st["x"], st["z"], st["zbar"] = x, z, zbar
    return st


def pdhg_problem(prob: Problem, weights=None) -> Problem:
    """The same problem as one data block (all angles) plus the prior blocks, with PDHG
    step weights q (sum 1) in the role of p in Theorem 2: data 1/2 and prior 1/2 (TV,
    aTV, dTV), 1/2, 1/4, 1/4 (TGV), 1 (ML)."""
    q = weights
    if q is None:
        q = {0: [1.0], 1: [0.5, 0.5], 2: [0.5, 0.25, 0.25]}[prob.n_prior]
    pp = Problem(geom=prob.geom, b=prob.b, r=prob.r, mult=prob.mult, n_subsets=1,
                 prior=prob.prior, alpha=prob.alpha, alpha1=prob.alpha1, side=prob.side,
                 eta=prob.eta, gamma_d=prob.gamma_d, sampling="uniform",
                 precond=prob.precond, gamma=prob.gamma, rho=prob.rho)
    pp.p = list(q)
    pp._setup_steps()
    return pp


def pdhg(prob: Problem, n_iter: int, state=None, x0=None, tol_gap=None, U=None):
    """Algorithm 1 (PDHG): all dual blocks are updated in every iteration.

    `prob` is normally pdhg_problem(...).  If tol_gap is given, stop once the relative
    duality gap (box bound U) is below it."""
    st = prob.new_state(x0) if state is None else state
    x, z, zbar = st["x"], st["z"], st["zbar"]
    for _ in range(n_iter):
        x = prob.prox_g(x - prob.T * zbar)                          # primal step
        dz = np.zeros_like(x)
        new_y, new_yp = [], []
        for i in range(prob.m):                                     # dual step, every block
            yi = st["y"][i]
            v = yi + prob.sigma[i] * prob.A_data(i, x)
            new_y.append(P.prox_kl_dual(v, prob.sigma[i], prob.sub_b[i], prob.sub_r[i]))
        for j in range(prob.n_prior):
            yj = st["yp"][j]
            new_yp.append(prob.prior_dual_prox(j, yj + prob.prior_sigma[j] * prob.A_prior(j, x)))
        for i in range(prob.m):                                     # backprojected dual change
            dz = dz + prob.AT_data(i, new_y[i] - st["y"][i])
        for j in range(prob.n_prior):
            dz = dz + prob.AT_prior(j, new_yp[j] - st["yp"][j])
        z = z + dz                                                  # z update
        st["y"], st["yp"] = new_y, new_yp
        zbar = z + dz                                               # extrapolation
        st["k"] += 1
        st["x"], st["z"], st["zbar"] = x, z, zbar
        if tol_gap is not None and st["k"] % 50 == 0:
            xr = prob.reported(st)
            gp = duality_gap(prob, xr, st, U)
            if gp <= tol_gap * abs(prob.objective(xr)):
                break
    st["x"], st["z"], st["zbar"] = x, z, zbar
    return st


def data_mask(prob: Problem, i: int):
    return prob.sigma[i] > 0 if prob.precond else \
        (prob.sub_mult[i] * proj.forward(prob.geom, np.ones(prob.geom.image_shape),
                                          prob.angles[i]) > 0)


def duality_gap(prob: Problem, X, st, U: float) -> float:
    """Gap of the box-constrained problem g = indicator of [0, U] (U above max x*):
        Psi(X) + sum_i f_i*(y_i) + U sum_v max(0, -(A^T y)_v)
    over the bins with A_i 1 > 0 (rows with A_i 1 = 0 are constants of both problems).
    Not defined for TGV (its w-block makes g* infinite)."""
    if prob.prior == "tgv":
        raise ValueError("gap undefined for TGV; use kkt_residual")
    X = np.asarray(X, np.float64).reshape(prob.image_shape())
    primal = prob.prior_term(X)
    dual = 0.0
    ATy = np.zeros(prob.image_shape())
    for i in range(prob.m):
        mask = data_mask(prob, i)
        ax = prob.A_data(i, X)
        primal += float(np.sum(P.phi(ax, prob.sub_b[i], prob.sub_r[i])[mask]))
        dual += float(np.sum(P.phi_conj(st["y"][i], prob.sub_b[i], prob.sub_r[i])[mask]))
        ATy += prob.AT_data(i, st["y"][i])
    for j in range(prob.n_prior):
        q = st["yp"][j]
        if prob.prior == "atv":
            ok = np.all(np.abs(q) <= prob.alpha * (1 + 1e-12))
        else:
            ok = np.all(np.sqrt(np.sum(q * q, axis=0)) <= prob.prior_weight(j) * (1 + 1e-12))
        if not ok:
            return math.inf
        ATy += prob.AT_prior(j, q)
    box = U * float(np.sum(np.maximum(0.0, -ATy[0])))
    return primal + dual + box


def kkt_residual(prob: Problem, X, st) -> float:
    """Fixed-point residual of the primal-dual optimality conditions (max norm)."""
    res = 0.0
    ATy = np.zeros(prob.image_shape())
    for i in range(prob.m):
        yi = st["y"][i]
        yi_fix = P.prox_kl_dual(yi + prob.sigma[i] * prob.A_data(i, X), prob.sigma[i],
                                prob.sub_b[i], prob.sub_r[i])
        res = max(res, float(np.max(np.abs(yi_fix - yi))))
        ATy += prob.AT_data(i, yi)
    for j in range(prob.n_prior):
        q = st["yp"][j]
        q_fix = prob.prior_dual_prox(j, q + prob.prior_sigma[j] * prob.A_prior(j, X))
        res = max(res, float(np.max(np.abs(q_fix - q))))
        ATy += prob.AT_prior(j, q)
    x_fix = prob.prox_g(X - prob.T * ATy)
    res = max(res, float(np.max(np.abs(x_fix - X))))
    return res


def osem_step(prob: Problem, u, i: int):
    """One OSEM sub-iteration on subset i (eq. OSEM): u <- u / (P_i^T 1) * P_i^T(b_i /
    (P_i u + r_i)), with 0 where P_i^T 1 = 0 and b / (.) taken as 0 on bins with b = 0.
    The subsets are the problem's (equidistant angles); a full OSEM iteration visits
    i = 0, 1, ..., m - 1 in order."""
    g = prob.geom
    u = np.asarray(u, np.float64).reshape(g.image_shape)
    ang = prob.angles[i]
    sens = proj.backward(g, prob.sub_mult[i], ang)
    pu = prob.sub_mult[i] * proj.forward(g, u, ang)
    b, r = prob.sub_b[i], prob.sub_r[i]
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(b > 0, b / (pu + r), 0.0)
    back = proj.backward(g, prob.sub_mult[i] * ratio, ang)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(sens > 0, u / sens * back, 0.0)


def poisson_loglik(prob: Problem, u) -> float:
    """sum_j b_j log((P u + r)_j) - (P u + r)_j: the Poisson log-likelihood up to a constant
    (the negative of the data term of Problem 1 plus that constant)."""
    g = prob.geom
    ybar = prob.mult * proj.forward(g, np.asarray(u, np.float64).reshape(g.image_shape)) + prob.r
    with np.errstate(divide="ignore"):
        return float(np.sum(np.where(prob.b > 0, prob.b * np.log(ybar), 0.0) - ybar))


def mlem_step(prob: Problem, u):
    """One MLEM update u <- u / (P^T 1) * P^T(b / (P u + r)) (eq. MLEM)."""
    g = prob.geom
    sens = proj.backward(g, prob.mult, None)
    pu = prob.mult * proj.forward(g, u, None)
    ratio = np.where(prob.b > 0, prob.b / (pu + prob.r), 0.0)
    back = proj.backward(g, prob.mult * ratio, None)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(sens > 0, u / sens * back, 0.0)


def psnr_paper(xk, xstar) -> float:
    """PSNR(x^k, x*) = 20 log10(||x*||_inf / ||x^k - x*||_2) (Section 4)."""
    return 20.0 * math.log10(np.max(np.abs(xstar)) / np.linalg.norm((xk - xstar).ravel()))


def relative_objective(psi_k, psi_star, psi_0) -> float:
    """(Psi(x^k) - Psi(x*)) / (Psi(x^0) - Psi(x*)) (Section 4)."""
    return (psi_k - psi_star) / (psi_0 - psi_star)
