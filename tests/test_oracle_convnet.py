"""Pins of the warm-start network oracle (oracle/convnet.py) against library routines,
adjoint identities and closed forms (no GPU)."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import convnet as C


def rng(seed=0):
    return np.random.Generator(np.random.PCG64(seed))


def test_conv3d_matches_scipy_correlate():
    r = rng(1)
    x = r.standard_normal((5, 6, 7, 3))
    w = r.standard_normal((27, 4, 3))
    b = r.standard_normal(4)
    y = C.conv3d(x, w, b)
    for co in range(4):
        ref = np.full(x.shape[:3], b[co])
        for ci in range(3):
            k = w[:, co, ci].reshape(3, 3, 3)  # [dy+1][dx+1][dz+1]
            ref += ndimage.correlate(x[..., ci], k, mode="constant", cval=0.0)
        np.testing.assert_allclose(y[..., co], ref, rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(C.conv3d(x, w, b, relu=True), np.maximum(y, 0))


def test_conv3d_adjoint_and_weight_gradient():
    r = rng(2)
    x = r.standard_normal((4, 5, 6, 3))
    w = r.standard_normal((27, 2, 3))
    g = r.standard_normal((4, 5, 6, 2))
    lhs = np.sum(C.conv3d(x, w) * g)
    assert abs(lhs - np.sum(x * C.conv3d_input_grad(g, w))) <= 1e-11 * abs(lhs)
    dw, db = C.conv3d_weight_grad(x, g)
    assert abs(lhs - np.sum(w * dw)) <= 1e-11 * abs(lhs)
    # the bias enters every voxel once
    b = r.standard_normal(2)
    assert np.sum((C.conv3d(x, w, b) - C.conv3d(x, w)) * g) == pytest.approx(np.dot(b, db), rel=1e-12)
    # a single tap of a delta input reproduces the weight (no hidden flip)
    d = np.zeros((3, 3, 3, 1))
    d[1, 1, 1, 0] = 1.0
    wt = np.zeros((27, 1, 1))
    wt[C.TAPS.index((1, 0, -1)), 0, 0] = 2.5
    y = C.conv3d(d, wt)
    assert y[0, 1, 2, 0] == 2.5 and np.count_nonzero(y) == 1  # y[v] = w x[v + (1, 0, -1)]


def test_pool_and_upsample_adjoints():
    r = rng(3)
    x = r.standard_normal((4, 6, 8, 2))
    g = r.standard_normal((2, 3, 4, 2))
    assert np.sum(C.pool2(x) * g) == pytest.approx(np.sum(x * C.pool2_adjoint(g)), rel=1e-12)
    assert np.sum(C.up2(g) * x) == pytest.approx(np.sum(g * C.up2_adjoint(x)), rel=1e-12)
    np.testing.assert_allclose(C.pool2(C.up2(g)), g, rtol=1e-15)
    np.testing.assert_allclose(C.pool2(np.full((2, 2, 2, 1), 3.0)), 3.0)


def test_bf16_round_ties_to_even():
    e = 2.0 ** -8
    vals = np.array([1.0, 1 + e, 1 + 3 * e, 1 + 1.1 * e, -(1 + 3 * e), 3.0], np.float32)
    np.testing.assert_array_equal(C.bf16_round(vals),
                                  [1.0, 1.0, 1 + 4 * e, 1 + 2 * e, -(1 + 4 * e), 3.0])


def test_adam_first_step_closed_form():
    p, g = np.array([1.0, -2.0]), np.array([0.5, -3.0])
    pn, m, v = C.adam(p, np.zeros(2), np.zeros(2), g, 1, lr=0.1, eps=0.0)
    np.testing.assert_allclose(pn, p - 0.1 * np.sign(g), rtol=1e-14)


def test_network_gradient_by_finite_differences():
    """The oracle's backpropagation of the encoder-decoder against central differences of
    its loss (no rounding), on a few weights of every layer."""
    g = rng(4)
    shape = (4, 4, 8)
    img = np.abs(g.standard_normal(shape))
    tgt = 0.5 * img + 0.1
    w = {n: g.standard_normal((27, co, ci)) * np.sqrt(2.0 / (27 * ci)) for n, ci, co, _ in C.LAYERS}
    b = {n: 0.1 * g.standard_normal(co) for n, ci, co, _ in C.LAYERS}
    ident = lambda a: a  # noqa: E731
    _, grads = C.network_gradients(img, tgt, 1.0, w, b, rnd=ident)
    h = 1e-6
    for n, ci, co, _ in C.LAYERS:
        for idx in [(13, 0, 0), (4, co - 1, ci - 1)]:
            wp = {k: v.copy() for k, v in w.items()}
            wm = {k: v.copy() for k, v in w.items()}
            wp[n][idx] += h
            wm[n][idx] -= h
            fd = (C.network_gradients(img, tgt, 1.0, wp, b, ident)[0]
                  - C.network_gradients(img, tgt, 1.0, wm, b, ident)[0]) / (2 * h)
            assert fd == pytest.approx(grads[n + ".w"][idx], rel=1e-5, abs=1e-7), (n, idx)
