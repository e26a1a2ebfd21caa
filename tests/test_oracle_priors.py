"""Pins of the prior operators: adjoint identities, exact stencil values on simple
fields, and operator norms against dense SVD of the explicitly built matrices."""
import math

import numpy as np
import pytest

from oracle import priors as R


def _dense(apply, in_shape):
    n = int(np.prod(in_shape))
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(np.asarray(apply(e.reshape(in_shape))).ravel())
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("shape", [(1, 6, 7), (4, 5, 6)])
def test_grad_adjoint(shape):
    rng = np.random.default_rng(0)
    u = rng.normal(size=shape)
    p = rng.normal(size=(3,) + shape)
    assert np.vdot(R.grad(u), p) == pytest.approx(np.vdot(u, R.grad_adj(p)), rel=1e-13)


def test_sym_grad_adjoint():
    rng = np.random.default_rng(1)
    w = rng.normal(size=(3, 4, 5, 6))
    q = rng.normal(size=(6, 4, 5, 6))
    assert np.vdot(R.sym_grad(w), q) == pytest.approx(np.vdot(w, R.sym_grad_adj(q)), rel=1e-13)


def test_dgrad_adjoint():
    rng = np.random.default_rng(2)
    side = rng.random((4, 5, 6))
    xi = R.dtv_field(side, 0.1)
    u = rng.normal(size=(4, 5, 6))
    p = rng.normal(size=(3, 4, 5, 6))
    assert np.vdot(R.dgrad(u, xi), p) == pytest.approx(np.vdot(u, R.dgrad_adj(p, xi)), rel=1e-13)


def test_grad_of_ramp_and_boundary():
    """u = 2 x + 3 y - z: forward differences are (2, 3, -1) except 0 at the last index."""
    z, y, x = np.meshgrid(np.arange(4), np.arange(5), np.arange(6), indexing="ij")
    u = 2.0 * x + 3.0 * y - 1.0 * z
    g = R.grad(u)
    assert np.all(g[0][:, :, :-1] == 2) and np.all(g[0][:, :, -1] == 0)
    assert np.all(g[1][:, :-1, :] == 3) and np.all(g[1][:, -1, :] == 0)
    assert np.all(g[2][:-1] == -1) and np.all(g[2][-1] == 0)


def test_sym_grad_of_shear():
    """w = (y, 0, 0): J_{xy} = d_y w_x = 1, so E w = (0,0,0, 1/sqrt2, 0, 0) inside."""
    z, y, x = np.meshgrid(np.arange(4), np.arange(5), np.arange(6), indexing="ij")
    w = np.stack([y.astype(float), np.zeros_like(x, float), np.zeros_like(x, float)])
    e = R.sym_grad(w)
    assert np.allclose(e[3][:, :-1, :], math.sqrt(0.5))
    for c in (0, 1, 2, 4, 5):
        assert np.all(e[c] == 0)


# Every entry J_kl = d_l w_k of the Jacobian, excited alone by the linear field w_k = l
# (component k of w equal to coordinate l, the other components zero).  E w = (J + J^T)/2
# stored as (J_xx, J_yy, J_zz, sqrt2 J_(xy), sqrt2 J_(xz), sqrt2 J_(yz)) (eq. setting TGV,
# with the Frobenius norm), so J_kl alone lands in exactly one component: 1 on the
# diagonal, 1/sqrt2 off it, on every voxel whose forward difference along l is interior.
_JAC_CASES = [  # (component k of w, coordinate l, component of E w that holds J_kl, value)
    (0, 0, 0, 1.0), (1, 1, 1, 1.0), (2, 2, 2, 1.0),
    (0, 1, 3, math.sqrt(0.5)), (1, 0, 3, math.sqrt(0.5)),
    (0, 2, 4, math.sqrt(0.5)), (2, 0, 4, math.sqrt(0.5)),
    (1, 2, 5, math.sqrt(0.5)), (2, 1, 5, math.sqrt(0.5)),
]


@pytest.mark.parametrize("k,l,comp,val", _JAC_CASES)
def test_sym_grad_every_jacobian_entry(k, l, comp, val):
    shape = (4, 5, 6)  # [z][y][x]
    coords = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), np.arange(shape[2]),
                         indexing="ij")
    coord = {0: coords[2], 1: coords[1], 2: coords[0]}[l].astype(float)  # x, y, z
    w = np.zeros((3,) + shape)
    w[k] = coord
    e = R.sym_grad(w)
    interior = [slice(None)] * 3
    interior[{0: 2, 1: 1, 2: 0}[l]] = slice(0, shape[{0: 2, 1: 1, 2: 0}[l]] - 1)
    expect = np.zeros(shape)
    expect[tuple(interior)] = val
    for c in range(6):
        np.testing.assert_array_equal(e[c], expect if c == comp else 0.0)
    # the adjoint moves a unit dual in component comp back onto w_k only through the
    # difference along l (and, off the diagonal, onto w_l through the difference along k)
    q = np.zeros((6,) + shape)
    q[comp] = 1.0
    back = R.sym_grad_adj(q)
    ref = np.zeros((3,) + shape)
    ref[k] = val * R.fdiff_adj(np.ones(shape), l)
    if k != l:
        ref[l] = val * R.fdiff_adj(np.ones(shape), k)
    np.testing.assert_allclose(back, ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("shape", [(1, 8, 8), (3, 4, 5), (2, 3, 7)])
def test_grad_norm_closed_form_vs_svd(shape):
    M = _dense(R.grad, shape)
    assert R.grad_norm_closed_form(shape) == pytest.approx(np.linalg.norm(M, 2), rel=1e-12)
    # TGV first block (grad, -I)
    n = int(np.prod(shape))
    M2 = np.concatenate([M, -np.eye(3 * n)], axis=1)
    assert math.sqrt(R.grad_norm_closed_form(shape) ** 2 + 1) == pytest.approx(
        np.linalg.norm(M2, 2), rel=1e-12)


def test_grad_norm_quoted_values():
    assert R.grad_norm_closed_form((1, 64, 64)) == pytest.approx(2.827575, abs=1e-6)
    assert R.grad_norm_closed_form((127, 344, 344)) == pytest.approx(3.463989, abs=1e-6)


@pytest.mark.parametrize("shape", [(1, 5, 5), (3, 4, 5), (2, 6, 3)])
def test_sym_grad_norm_below_grad_norm(shape):
    """||E|| <= ||grad|| (the TGV block-n step bound): dense SVD of E against the closed
    form, with ||E w||_F^2 <= sum_k ||grad w_k||^2 as the reason."""
    ME = _dense(R.sym_grad, (3,) + shape)
    assert np.linalg.norm(ME, 2) <= R.grad_norm_closed_form(shape) * (1 + 1e-12)


def test_power_iteration_vs_svd():
    shape = (3, 4, 5)
    ME = _dense(R.sym_grad, (3,) + shape)
    est = R.power_norm(R.sym_grad, R.sym_grad_adj, R.checkerboard((3,) + shape), iters=5000,
                       tol=1e-15)
    assert est == pytest.approx(np.linalg.norm(ME, 2), rel=1e-6)
    rng = np.random.default_rng(3)
    xi = R.dtv_field(rng.random(shape), 0.05)
    MD = _dense(lambda u: R.dgrad(u, xi), shape)
    assert np.linalg.norm(MD, 2) <= R.grad_norm_closed_form(shape) + 1e-12
    est = R.power_norm(lambda u: R.dgrad(u, xi), lambda p: R.dgrad_adj(p, xi),
                       R.checkerboard(shape), iters=5000, tol=1e-15)
    assert est == pytest.approx(np.linalg.norm(MD, 2), rel=1e-6)


def test_dtv_field_hand_values():
    """xi = grad s / sqrt(|grad s|^2 + eta^2) at eta = 1e-2 (Section 4.3, directional TV)
    on a side image that is a ramp of slope 0.01 along x plus a unit step along y between
    rows 1 and 2, values worked out by hand:
      ramp only          grad s = (0.01, 0, 0):  |.|^2 + eta^2 = 2e-4,
                         xi = (0.01 / sqrt(2e-4), 0, 0) = (1/sqrt2, 0, 0);
      ramp and step      grad s = (0.01, 1, 0):  |.|^2 + eta^2 = 1.0002,
                         xi = (0.01, 1, 0) / sqrt(1.0002);
      last column        grad s = (0, 0, 0) (Neumann), xi = 0;
      last column, step  grad s = (0, 1, 0):     xi = (0, 1 / sqrt(1.0001), 0)."""
    shape = (3, 4, 5)
    z, y, x = np.meshgrid(np.arange(3), np.arange(4), np.arange(5), indexing="ij")
    side = 0.01 * x + (y >= 2).astype(float)
    xi = R.dtv_field(side, 1e-2)
    np.testing.assert_allclose(xi[:, 0, 0, 0], [math.sqrt(0.5), 0.0, 0.0], rtol=1e-12)
    np.testing.assert_allclose(xi[:, 2, 3, 1], [math.sqrt(0.5), 0.0, 0.0], rtol=1e-12)
    np.testing.assert_allclose(xi[:, 1, 1, 2], np.array([0.01, 1.0, 0.0]) / math.sqrt(1.0002),
                               rtol=1e-12)
    np.testing.assert_array_equal(xi[:, 0, 0, 4], [0.0, 0.0, 0.0])
    np.testing.assert_allclose(xi[:, 0, 1, 4], [0.0, 1.0 / math.sqrt(1.0001), 0.0], rtol=1e-12)
    assert xi.shape == (3,) + shape


def test_dtv_operator_hand_values():
    """D grad u with D = I - gamma_D xi xi^T at one voxel: with xi = (1/sqrt2, 0, 0) and
    gamma_D = 1 the x-component of grad u is halved and the others pass unchanged."""
    shape = (3, 4, 5)
    z, y, x = np.meshgrid(np.arange(3), np.arange(4), np.arange(5), indexing="ij")
    xi = R.dtv_field(0.01 * x, 1e-2)
    u = 3.0 * x + 2.0 * y - 1.0 * z
    dg = R.dgrad(u, xi)
    np.testing.assert_allclose(dg[:, 1, 1, 1], [1.5, 2.0, -1.0], rtol=1e-12)
    assert xi.shape == (3,) + shape


def test_dtv_reduces_to_tv_for_large_eta():
    rng = np.random.default_rng(4)
    side = rng.random((3, 4, 5))
    xi = R.dtv_field(side, 1e12)
    u = rng.normal(size=(3, 4, 5))
    np.testing.assert_allclose(R.dgrad(u, xi), R.grad(u), atol=1e-11)
