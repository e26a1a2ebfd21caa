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


def test_dtv_reduces_to_tv_for_large_eta():
    rng = np.random.default_rng(4)
    side = rng.random((3, 4, 5))
    xi = R.dtv_field(side, 1e12)
    u = rng.normal(size=(3, 4, 5))
    np.testing.assert_allclose(R.dgrad(u, xi), R.grad(u), atol=1e-11)
