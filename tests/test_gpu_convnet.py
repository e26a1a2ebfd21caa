"""Warm-start network kernels (BF16 MFMA convolutions and their adjoints, pooling,
upsampling, Adam) against the FP64 oracle on BF16-rounded inputs."""
import numpy as np
import pytest

from oracle import convnet as C

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ULP = 2.0 ** -8  # one BF16 rounding of the result


@pytest.fixture(scope="module")
def W():
    from paper_1808_07150_amd import warmstart
    warmstart.lib()
    return warmstart


def r(seed):
    return np.random.Generator(np.random.PCG64(seed))


def to_dev(W, a):
    return W.from_float(torch.from_numpy(np.asarray(a, np.float32)).cuda()).contiguous()


def close_bf16(gpu, ref):
    gpu = np.asarray(gpu, np.float64)
    scale = np.abs(ref) + 1e-3 * np.max(np.abs(ref))
    err = np.max(np.abs(gpu - ref) / scale)
    assert err <= 1.01 * ULP, err


@pytest.mark.parametrize("ci,co", [(16, 16), (16, 32), (32, 64), (64, 32), (64, 64), (32, 16)])
@pytest.mark.parametrize("relu", [0, 1])
def test_conv_forward(W, ci, co, relu):
    print(f"[net] conv fwd {ci}->{co} relu={relu}", flush=True)
    g = r(ci * 100 + co + relu)
    shape = (5, 7, 21)  # ragged against the 4 x 16 output tiles
    x = C.bf16_round(g.standard_normal(shape + (ci,)))
    w = C.bf16_round(g.standard_normal((27, co, ci)) / np.sqrt(27 * ci))
    b = g.standard_normal(co).astype(np.float32)
    ref = C.conv3d(x, w, b, relu=bool(relu))
    w32 = torch.from_numpy(w.astype(np.float32)).cuda()
    out = W.conv_fwd(to_dev(W, x), W.pack(w32, ci, co), torch.from_numpy(b).cuda(), relu, co)
    close_bf16(W.as_float(out).cpu().numpy(), ref)


@pytest.mark.parametrize("ci,co", [(16, 32), (64, 64), (32, 16)])
def test_conv_input_gradient(W, ci, co):
    g = r(7 + ci + co)
    shape = (6, 5, 19)
    dy = C.bf16_round(g.standard_normal(shape + (co,)))
    w = C.bf16_round(g.standard_normal((27, co, ci)) / np.sqrt(27 * co))
    ref = C.conv3d_input_grad(dy, w)
    w16 = W.pack(torch.from_numpy(w.astype(np.float32)).cuda(), ci, co)
    dx = W.conv_fwd(to_dev(W, dy), W.adjoint_weights(w16, ci, co), None, False, ci)
    close_bf16(W.as_float(dx).cpu().numpy(), ref)


@pytest.mark.parametrize("ci,co,chunk", [(16, 16, 64), (32, 64, 256), (64, 32, 4096)])
def test_conv_weight_gradient(W, ci, co, chunk):
    g = r(11 + ci + co)
    shape = (6, 7, 13)
    x = C.bf16_round(g.standard_normal(shape + (ci,)))
    dy = C.bf16_round(g.standard_normal(shape + (co,)))
    dw_ref, db_ref = C.conv3d_weight_grad(x, dy)
    part = torch.empty(W.wgrad_part_floats(shape, ci, co, chunk), dtype=torch.float32, device="cuda")
    dw, db = W.conv_wgrad(to_dev(W, x), to_dev(W, dy), part, chunk=chunk)
    dw = dw.cpu().numpy()
    assert np.max(np.abs(dw - dw_ref)) <= 1e-5 * np.max(np.abs(dw_ref))
    assert np.max(np.abs(db.cpu().numpy() - db_ref)) <= 1e-5 * np.max(np.abs(db_ref))


def test_pool_upsample_and_adjoints(W):
    g = r(5)
    x = C.bf16_round(g.standard_normal((4, 6, 10, 32)))
    c = C.bf16_round(g.standard_normal((2, 3, 5, 32)))
    close_bf16(W.as_float(W.pool2(to_dev(W, x))).cpu().numpy(), C.pool2(x))
    close_bf16(W.as_float(W.pool2_adjoint(to_dev(W, c))).cpu().numpy(), C.pool2_adjoint(c))
    np.testing.assert_array_equal(W.as_float(W.up2(to_dev(W, c))).cpu().numpy(), C.up2(c))
    close_bf16(W.as_float(W.up2_adjoint(to_dev(W, x))).cpu().numpy(), C.up2_adjoint(x))


def test_adam_step(W):
    from paper_1808_07150_amd.warmstart import _chk, _p, _s, lib
    g = r(9)
    p, gr = g.standard_normal(1000), g.standard_normal(1000)
    m, v = np.zeros(1000), np.zeros(1000)
    tp = torch.from_numpy(p.astype(np.float32)).cuda()
    tm, tv = torch.zeros_like(tp), torch.zeros_like(tp)
    tg = torch.from_numpy(gr.astype(np.float32)).cuda()
    for step in (1, 2, 3):
        p, m, v = C.adam(p, m, v, gr, step, lr=1e-2)
        _chk(lib().spdhg_net_adam(1000, 1e-2, 0.9, 0.999, 1e-8, step, _p(tp), _p(tm), _p(tv),
                                  _p(tg), None, _s()))
    assert np.max(np.abs(tp.cpu().numpy() - p)) <= 1e-5


def test_network_gradients_match_oracle(W):
    """Loss and every layer's weight / bias gradient of the GPU network (BF16 activations
    and gradients, FP32 accumulation) against FP64 backpropagation through BF16-rounded
    activations, with trained-like random weights."""
    shape = (8, 8, 12)
    g = r(21)
    img_np = np.abs(g.standard_normal(shape)).astype(np.float32)
    tgt_np = (0.5 * img_np + 0.2).astype(np.float32)
    net = W.WarmStartNet(shape, "cuda", seed=2)
    # a non-zero last layer and biases, so every path carries gradient
    w, b = {}, {}
    for n, ci, co, relu in W.LAYERS:
        wn = g.standard_normal((27, co, ci)) * np.sqrt(2.0 / (27 * ci)) * (1.0 if relu else 0.3)
        w[n] = C.bf16_round(wn)
        b[n] = (0.05 * g.standard_normal(co)).astype(np.float32).astype(np.float64)
        net.w32[n].copy_(torch.from_numpy(w[n].astype(np.float32)))
        net.b32[n].copy_(torch.from_numpy(b[n].astype(np.float32)))
        W.pack(net.w32[n], ci, co, out=net.w16[n])
    img = torch.from_numpy(img_np).cuda()
    tgt = torch.from_numpy(tgt_np).cuda()
    loss, grads = net.gradients(img, tgt, 1.5)
    loss_ref, ref = C.network_gradients(img_np.astype(np.float64), tgt_np.astype(np.float64), 1.5, w, b)
    assert loss == pytest.approx(loss_ref, rel=2e-2)
    for n, *_ in W.LAYERS:
        for k in ("w", "b"):
            got = grads[f"{n}.{k}"].cpu().numpy().astype(np.float64)
            exp = ref[f"{n}.{k}"]
            err = np.linalg.norm(got - exp) / np.linalg.norm(exp)
            assert err <= 5e-2, (n, k, err)


def test_network_learns_a_fixed_pair(W):
    """A few Adam steps on one (input, target) pair lower the loss; the untrained network
    (zero last layer) returns its input."""
    shape = (8, 12, 16)
    g = r(3)
    img = torch.from_numpy(np.abs(g.standard_normal(shape)).astype(np.float32)).cuda()
    tgt = 0.5 * img + 0.2  # a map the network can represent
    net = W.WarmStartNet(shape, "cuda", seed=1)
    out = net.forward(img, 1.0)
    np.testing.assert_allclose(out.cpu().numpy(), img.cpu().numpy(), rtol=2 ** -8)
    losses = [net.train_step(img, tgt, 1.0, lr=3e-3) for _ in range(40)]
    assert losses[-1] < 0.7 * losses[0], losses


def _random_net(W, shape, seed):
    """A network with trained-like random weights and biases (BF16-representable)."""
    g = r(seed)
    net = W.WarmStartNet(shape, "cuda", seed=seed)
    w, b = {}, {}
    for n, ci, co, relu in W.LAYERS:
        wn = g.standard_normal((27, co, ci)) * np.sqrt(2.0 / (27 * ci)) * (1.0 if relu else 0.3)
        w[n] = C.bf16_round(wn)
        b[n] = (0.05 * g.standard_normal(co)).astype(np.float32).astype(np.float64)
        net.w32[n].copy_(torch.from_numpy(w[n].astype(np.float32)))
        net.b32[n].copy_(torch.from_numpy(b[n].astype(np.float32)))
    net.pack()
    return net, w, b


def test_network_inference_matches_oracle(W):
    """spdhg_ws_infer (the whole network in the library) against the FP64 forward through
    BF16-rounded activations."""
    shape = (8, 12, 8)
    img_np = np.abs(r(31).standard_normal(shape)).astype(np.float32)
    net, w, b = _random_net(W, shape, 32)
    out = net.forward(torch.from_numpy(img_np).cuda(), 1.5).cpu().numpy()
    ref = C.network_forward(img_np.astype(np.float64), 1.5, w, b)
    ref = ref[0] if isinstance(ref, tuple) else ref
    err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
    assert err <= 2e-2, err


def test_train_step_is_gradients_then_adam(W):
    """spdhg_ws_train_step = spdhg_ws_gradients, then one Adam step over the parameter blob
    and the packed copies: bitwise against the separate calls, over two steps."""
    shape = (8, 8, 12)
    g = r(41)
    img = torch.from_numpy(np.abs(g.standard_normal(shape)).astype(np.float32)).cuda()
    tgt = 0.5 * img + 0.2
    a, _, _ = _random_net(W, shape, 42)
    b, _, _ = _random_net(W, shape, 42)
    for step in (1, 2):
        la = a.train_step(img, tgt, 1.3, lr=2e-3)
        lb, grads = b.gradients(img, tgt, 1.3)
        flat = torch.empty_like(b.p32)
        for n, ci, co, _ in W.LAYERS:
            ow, ob, _ = W.param_layout()[2][n]
            flat[ow:ow + 27 * ci * co] = grads[f"{n}.w"].reshape(-1)
            flat[ob:ob + co] = grads[f"{n}.b"]
        W._chk(W.lib().spdhg_net_adam(b.p32.numel(), 2e-3, 0.9, 0.999, 1e-8, step, W._p(b.p32),
                                      W._p(b.m), W._p(b.v), W._p(flat), None, W._s()))
        b.pack()
        torch.cuda.synchronize()
        assert la == lb
        assert torch.equal(a.p32, b.p32) and torch.equal(a.w16blob, b.w16blob)
        assert torch.equal(a.m, b.m) and torch.equal(a.v, b.v)


def test_whole_network_argument_errors(W):
    import ctypes
    shape = (8, 8, 12)
    net = W.WarmStartNet(shape, "cuda", seed=0)
    img = torch.zeros(shape, device="cuda")
    out = torch.empty_like(img)
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    rc = W.lib().spdhg_ws_infer(net._dims(), W._p(net.p32), W._p(net.w16blob), 1.0, W._p(img),
                                W._p(out), ctypes.c_void_p(ws.data_ptr()), 1024, W._s())
    assert rc == -5  # workspace too small
    bad = (ctypes.c_int32 * 3)(8, 8, 10)
    nb = ctypes.c_size_t()
    assert W.lib().spdhg_ws_workspace_bytes(bad, 0, ctypes.byref(nb)) == -2
