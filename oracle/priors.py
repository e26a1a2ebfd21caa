"""Linear operators of the priors, FP64.  Test infrastructure only.

* grad: forward differences with unit spacing and a zero difference at the last index
  (Neumann), as in the Chambolle-Pock discretisation the paper cites for TV
  (Section 2.1).  Components ordered (x, y, z), images [z][y][x].
* grad_adj: the exact adjoint grad^T (= -div with backward differences).
* dTV (Section 4.3): A_n = D grad with D_v = I - gamma_D xi_v xi_v^T,
  xi_v = grad(s)_v / sqrt(||grad(s)_v||^2 + eta^2) for a side image s.
* TGV (Section 4.3): A_{n-1} = (grad, -I), A_n = (0, E) with the symmetrised gradient
  E w = (J + J^T)/2, J_kl = forward difference of w_k along axis l (same rule as grad),
  stored as 6 components (d1w1, d2w2, d3w3, (d2w1+d1w2)/sqrt2, (d3w1+d1w3)/sqrt2,
  (d3w2+d2w3)/sqrt2) so that the plain Euclidean norm per voxel is the Frobenius norm.
"""
from __future__ import annotations

import math

import numpy as np

SQRT_HALF = math.sqrt(0.5)
# axis of component d in a [z][y][x] array
_AX = {0: 2, 1: 1, 2: 0}


def fdiff(u, d):
    """Forward difference of u along component d, zero at the last index."""
    ax = _AX[d]
    out = np.zeros_like(u, dtype=np.float64)
    n = u.shape[ax]
    if n > 1:
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        out[tuple(lo)] = u[tuple(hi)] - u[tuple(lo)]
    return out


def fdiff_adj(p, d):
    """Adjoint of fdiff along component d: (fdiff^T p)_i = p_{i-1} - p_i with
    p_{-1} = 0 and p_{n-1} treated as 0 (it multiplies a zero difference)."""
    ax = _AX[d]
    n = p.shape[ax]
    out = np.zeros_like(p, dtype=np.float64)
    if n > 1:
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        out[tuple(lo)] -= p[tuple(lo)]
        out[tuple(hi)] += p[tuple(lo)]
    return out


def grad(u):
    u = np.asarray(u, dtype=np.float64)
    return np.stack([fdiff(u, d) for d in range(3)])


def grad_adj(p):
    return sum(fdiff_adj(p[d], d) for d in range(3))


def grad_norm_closed_form(shape) -> float:
    """||grad|| = 2 sqrt(sum_k sin^2(pi (N_k - 1) / (2 N_k))): grad^T grad is the sum of
    path-graph Laplacians, whose largest eigenvalue is 4 sin^2(pi (N-1)/(2N))."""
    return 2.0 * math.sqrt(sum(math.sin(math.pi * (n - 1) / (2.0 * n)) ** 2 for n in shape))


# ---------------------------------------------------------------- directional TV
def dtv_field(side, eta: float):
    """xi = grad(s) / sqrt(|grad(s)|^2 + eta^2), per voxel."""
    gs = grad(side)
    nrm = np.sqrt(np.sum(gs * gs, axis=0) + eta * eta)
    return gs / nrm


def apply_D(p, xi, gamma_d: float = 1.0):
    """D_v p_v = p_v - gamma_D <xi_v, p_v> xi_v (symmetric)."""
    dot = np.sum(xi * p, axis=0, keepdims=True)
    return p - gamma_d * dot * xi


def dgrad(u, xi, gamma_d=1.0):
    return apply_D(grad(u), xi, gamma_d)


def dgrad_adj(p, xi, gamma_d=1.0):
    return grad_adj(apply_D(p, xi, gamma_d))


# ---------------------------------------------------------------- TGV
def sym_grad(w):
    """E w for a 3-component field w[3][z][y][x] -> 6 components."""
    J = [[fdiff(w[k], l) for l in range(3)] for k in range(3)]
    return np.stack([J[0][0], J[1][1], J[2][2],
                     SQRT_HALF * (J[0][1] + J[1][0]),
                     SQRT_HALF * (J[0][2] + J[2][0]),
                     SQRT_HALF * (J[1][2] + J[2][1])])


def sym_grad_adj(q):
    """E^T q for q[6][z][y][x] -> 3 components."""
    w = np.zeros((3,) + q.shape[1:], dtype=np.float64)
    w[0] += fdiff_adj(q[0], 0)
    w[1] += fdiff_adj(q[1], 1)
    w[2] += fdiff_adj(q[2], 2)
    # (d2 w1 + d1 w2)/sqrt2 -> q3
    w[0] += SQRT_HALF * fdiff_adj(q[3], 1)
    w[1] += SQRT_HALF * fdiff_adj(q[3], 0)
    # (d3 w1 + d1 w3)/sqrt2 -> q4
    w[0] += SQRT_HALF * fdiff_adj(q[4], 2)
    w[2] += SQRT_HALF * fdiff_adj(q[4], 0)
    # (d3 w2 + d2 w3)/sqrt2 -> q5
    w[1] += SQRT_HALF * fdiff_adj(q[5], 2)
    w[2] += SQRT_HALF * fdiff_adj(q[5], 1)
    return w


def norm_l21(p):
    """sum over voxels of the 2-norm of the component vector (axis 0)."""
    return float(np.sum(np.sqrt(np.sum(np.asarray(p, dtype=np.float64) ** 2, axis=0))))


def checkerboard(shape):
    """(-1)^(sum of indices): start vector for the norms of difference operators, whose
    top singular vectors oscillate at the grid frequency (constants are in their null
    spaces, so a constant start would be annihilated)."""
    idx = np.indices(shape).sum(axis=0)
    return np.where(idx % 2 == 0, 1.0, -1.0)


def power_norm(apply, apply_adj, x0, iters: int = 100, tol: float = 1e-10) -> float:
    """Operator norm by power iteration on A^T A, started from x0 (ones for A >= 0, a
    checkerboard for difference operators)."""
    v = np.array(x0, dtype=np.float64)
    v /= np.linalg.norm(v)
    est = 0.0
    for _ in range(iters):
        w = apply_adj(apply(v))
        nw = np.linalg.norm(w)
        if nw == 0:
            return 0.0
        new = math.sqrt(nw)
        v = w / nw
        if est > 0 and abs(new - est) <= tol * new:
            est = new
            break
        est = new
    return est
