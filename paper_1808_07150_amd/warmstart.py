"""Warm-start network for SPDHG (not part of the paper's method).

A 3-level 3-D convolutional encoder-decoder (channels 16/32/64, 3x3x3 kernels, BF16
weights and activations with FP32 accumulation on the MFMA units) maps the normalised
backprojection (A^T b) / (A^T 1) of the data to an initial image; SPDHG (Algorithm 2)
then runs from that image unchanged.  Every numerical step runs in libspdhg.so
(include/spdhg_net.h); this module holds the parameters in torch tensors (device memory
only) and sequences the calls.

Architecture (channel-last activations [y][x][z][C], sizes divisible by 4):
    e1 = relu(c2(relu(c1(in))))                  16 ch, full resolution
    e2 = relu(c4(relu(c3(pool(e1)))))            32 ch, 1/2
    b  = relu(c6(relu(c5(pool(e2)))))            64 ch, 1/4
    d2 = relu(c8(relu(c7(up(b))) + e2))          32 ch, 1/2
    d1 = relu(c10(relu(c9(up(d2))) + e1))        16 ch, full
    out = image_in + channel 0 of c11(d1)        (linear last layer, residual output)
"""
from __future__ import annotations

import ctypes
import math
from typing import Dict, List, Optional, Tuple

import torch

from .spdhg import load_library

NET_EXPORTED = ["spdhg_net_last_error", "spdhg_conv3d_fwd", "spdhg_conv3d_adjoint_weights",
                "spdhg_conv3d_wgrad", "spdhg_net_relu_bwd", "spdhg_net_add", "spdhg_net_pool2",
                "spdhg_net_up2", "spdhg_net_image_to_act", "spdhg_net_act_to_image",
                "spdhg_net_mse_grad", "spdhg_net_adam", "spdhg_net_pack_weights"]

# (name, cin, cout, relu)
LAYERS = [("c1", 16, 16, 1), ("c2", 16, 16, 1), ("c3", 16, 32, 1), ("c4", 32, 32, 1),
          ("c5", 32, 64, 1), ("c6", 64, 64, 1), ("c7", 64, 32, 1), ("c8", 32, 32, 1),
          ("c9", 32, 16, 1), ("c10", 16, 16, 1), ("c11", 16, 16, 0)]

_net = None


class NetError(RuntimeError):
    pass


def lib():
    """libspdhg.so with the network entry points typed."""
    global _net
    if _net is not None:
        return _net
    L = load_library()
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    f32 = ctypes.c_float
    dims = ctypes.POINTER(ctypes.c_int32)
    L.spdhg_net_last_error.restype = ctypes.c_char_p
    L.spdhg_conv3d_fwd.argtypes = [dims, i32, i32, vp, vp, vp, i32, vp, vp]
    L.spdhg_conv3d_adjoint_weights.argtypes = [i32, i32, vp, vp, vp]
    L.spdhg_conv3d_wgrad.argtypes = [dims, i32, i32, vp, vp, i32, vp, i64, vp, vp, vp]
    L.spdhg_net_relu_bwd.argtypes = [i64, vp, vp, vp]
    L.spdhg_net_add.argtypes = [i64, vp, vp, vp, vp]
    L.spdhg_net_pool2.argtypes = [dims, i32, i32, vp, vp, vp]
    L.spdhg_net_up2.argtypes = [dims, i32, i32, vp, vp, vp]
    L.spdhg_net_image_to_act.argtypes = [i64, f32, vp, vp, vp]
    L.spdhg_net_act_to_image.argtypes = [i64, f32, vp, i32, vp, vp, vp]
    L.spdhg_net_mse_grad.argtypes = [i64, i32, vp, vp, vp, f32, vp, vp, vp]
    L.spdhg_net_adam.argtypes = [i64, f32, f32, f32, f32, i64, vp, vp, vp, vp, vp, vp]
    L.spdhg_net_pack_weights.argtypes = [i32, i32, vp, vp, vp]
    for n in NET_EXPORTED[1:]:
        getattr(L, n).restype = ctypes.c_int
    _net = L
    return L


def _chk(rc):
    if rc != 0:
        raise NetError(f"{rc}: {lib().spdhg_net_last_error().decode()}")


def _p(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous()
    return ctypes.c_void_p(t.data_ptr())


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dims(shape) -> ctypes.Array:
    return (ctypes.c_int32 * 3)(*[int(v) for v in shape[:3]])


def bf16(shape, device, zero: bool = False) -> torch.Tensor:
    """A BF16 activation buffer (stored as int16 bit patterns); uninitialised unless
    `zero` (every kernel that fills one writes all of its elements)."""
    if zero:
        return torch.zeros(shape, dtype=torch.int16, device=device)
    return torch.empty(shape, dtype=torch.int16, device=device)


# ---------------------------------------------------------------- single kernels
def conv_fwd(x: torch.Tensor, w16: torch.Tensor, bias: Optional[torch.Tensor], relu: bool,
             cout: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    if out is None:
        out = bf16(tuple(x.shape[:3]) + (cout,), x.device)
    _chk(lib().spdhg_conv3d_fwd(_dims(x.shape), x.shape[3], cout, _p(x), _p(w16), _p(bias),
                                1 if relu else 0, _p(out), _s()))
    return out


def adjoint_weights(w16: torch.Tensor, cin: int, cout: int) -> torch.Tensor:
    wt = torch.empty_like(w16)
    _chk(lib().spdhg_conv3d_adjoint_weights(cin, cout, _p(w16), _p(wt), _s()))
    return wt


def conv_wgrad(x: torch.Tensor, dy: torch.Tensor, part: torch.Tensor, chunk: int = 4096,
               with_bias: bool = True) -> Tuple[torch.Tensor, Optional[torch.Tensor]]:
    cin, cout = x.shape[3], dy.shape[3]
    dw = torch.empty((27, cout, cin), dtype=torch.float32, device=x.device)
    db = torch.empty(cout, dtype=torch.float32, device=x.device) if with_bias else None
    _chk(lib().spdhg_conv3d_wgrad(_dims(x.shape), cin, cout, _p(x), _p(dy), chunk, _p(part),
                                  part.numel(), _p(dw), _p(db), _s()))
    return dw, db


def wgrad_part_floats(shape, cin: int, cout: int, chunk: int = 4096) -> int:
    nv = shape[0] * shape[1] * shape[2]
    return max(-(-nv // chunk) * 27 * cin * cout, -(-nv // 1024) * cout)


def relu_bwd(y: torch.Tensor, dy: torch.Tensor):
    _chk(lib().spdhg_net_relu_bwd(dy.numel(), _p(y), _p(dy), _s()))


def add(a: torch.Tensor, b: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    out = torch.empty_like(a) if out is None else out
    _chk(lib().spdhg_net_add(a.numel(), _p(a), _p(b), _p(out), _s()))
    return out


def pool2(x: torch.Tensor) -> torch.Tensor:
    ny, nx, nz, c = x.shape
    out = bf16((ny // 2, nx // 2, nz // 2, c), x.device)
    _chk(lib().spdhg_net_pool2(_dims(x.shape), c, 0, _p(x), _p(out), _s()))
    return out


def pool2_adjoint(g: torch.Tensor) -> torch.Tensor:
    ny, nx, nz, c = g.shape
    out = bf16((2 * ny, 2 * nx, 2 * nz, c), g.device)
    _chk(lib().spdhg_net_pool2(_dims(out.shape), c, 1, _p(g), _p(out), _s()))
    return out


def up2(x: torch.Tensor) -> torch.Tensor:
    ny, nx, nz, c = x.shape
    out = bf16((2 * ny, 2 * nx, 2 * nz, c), x.device)
    _chk(lib().spdhg_net_up2(_dims(out.shape), c, 0, _p(x), _p(out), _s()))
    return out


def up2_adjoint(g: torch.Tensor) -> torch.Tensor:
    ny, nx, nz, c = g.shape
    out = bf16((ny // 2, nx // 2, nz // 2, c), g.device)
    _chk(lib().spdhg_net_up2(_dims(g.shape), c, 1, _p(g), _p(out), _s()))
    return out


def pack(w32: torch.Tensor, cin: int, cout: int, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    out = torch.empty(27 * cin * cout, dtype=torch.int16, device=w32.device) if out is None else out
    _chk(lib().spdhg_net_pack_weights(cin, cout, _p(w32), _p(out), _s()))
    return out


def as_float(t: torch.Tensor) -> torch.Tensor:
    """BF16 bit patterns (int16) -> float32 (for inspection and tests)."""
    return (t.to(torch.int32) & 0xFFFF).mul(65536).view(torch.float32) if t.dtype == torch.int16 \
        else t.float()


def from_float(t: torch.Tensor) -> torch.Tensor:
    """float32 -> BF16 bit patterns (round to nearest even) as int16 (host-side setup)."""
    return t.to(torch.bfloat16).view(torch.int16)


# ---------------------------------------------------------------- the network
class WarmStartNet:
    """Parameters (FP32 masters, packed BF16 copies, Adam moments) and the forward /
    backward sequence of the encoder-decoder on one volume size."""

    def __init__(self, shape: Tuple[int, int, int], device, seed: int = 0):
        ny, nx, nz = shape
        if ny % 4 or nx % 4 or nz % 4:
            raise ValueError("volume sizes must be divisible by 4 (two poolings)")
        self.shape, self.device = tuple(shape), device
        g = torch.Generator(device="cpu")
        g.manual_seed(seed)
        self.w32: Dict[str, torch.Tensor] = {}
        self.b32: Dict[str, torch.Tensor] = {}
        for name, ci, co, relu in LAYERS:
            # He initialisation for ReLU layers; the last (linear) layer starts at zero so
            # the untrained network returns its input image
            std = math.sqrt(2.0 / (27 * ci)) if relu else 0.0
            self.w32[name] = (torch.randn((27, co, ci), generator=g) * std).to(device)
            self.b32[name] = torch.zeros(co, device=device)
        self.w16 = {n: pack(self.w32[n], ci, co) for n, ci, co, _ in LAYERS}
        self.m = {k: torch.zeros_like(v) for k, v in list(self._params().items())}
        self.v = {k: torch.zeros_like(v) for k, v in list(self._params().items())}
        self.step = 0
        self.lparts = torch.zeros(-(-ny * nx * nz // 256), dtype=torch.float64, device=device)

    def _params(self) -> Dict[str, torch.Tensor]:
        d = {f"{n}.w": self.w32[n] for n, *_ in LAYERS}
        d.update({f"{n}.b": self.b32[n] for n, *_ in LAYERS})
        return d

    def forward(self, img: torch.Tensor, scale: float, keep: bool = False):
        """Network output image from `img` ([ny][nx][nz] FP32, z fastest) scaled by
        `scale` into the network's range; with keep the activations are returned too."""
        nv = img.numel()
        spec = {n: (ci, co, relu) for n, ci, co, relu in LAYERS}
        a: Dict[str, torch.Tensor] = {}
        x = bf16(self.shape + (16,), self.device)
        _chk(lib().spdhg_net_image_to_act(nv, float(scale), _p(img), _p(x), _s()))
        a["in"] = x

        def conv(name, inp):
            ci, co, relu = spec[name]
            return conv_fwd(inp, self.w16[name], self.b32[name], bool(relu), co)

        a["c1"] = conv("c1", a["in"])
        a["e1"] = conv("c2", a["c1"])
        a["p1"] = pool2(a["e1"])
        a["c3"] = conv("c3", a["p1"])
        a["e2"] = conv("c4", a["c3"])
        a["p2"] = pool2(a["e2"])
        a["c5"] = conv("c5", a["p2"])
        a["b"] = conv("c6", a["c5"])
        a["u2"] = up2(a["b"])
        a["c7"] = conv("c7", a["u2"])
        a["s2"] = add(a["c7"], a["e2"])
        a["d2"] = conv("c8", a["s2"])
        a["u1"] = up2(a["d2"])
        a["c9"] = conv("c9", a["u1"])
        a["s1"] = add(a["c9"], a["e1"])
        a["d1"] = conv("c10", a["s1"])
        a["out"] = conv("c11", a["d1"])
        out = torch.empty_like(img)
        _chk(lib().spdhg_net_act_to_image(nv, float(scale), _p(a["out"]), 16, _p(img), _p(out), _s()))
        return (out, a) if keep else out

    def train_step(self, img: torch.Tensor, target: torch.Tensor, scale: float, lr: float = 1e-3,
                   part: Optional[torch.Tensor] = None) -> float:
        """One Adam step on 0.5 |net(img) - target|^2 (in the scaled range); returns the loss."""
        loss, grads = self.gradients(img, target, scale, part)
        self.step += 1
        for name, ci, co, _ in LAYERS:
            for kind in ("w", "b"):
                key = f"{name}.{kind}"
                p = self.w32[name] if kind == "w" else self.b32[name]
                _chk(lib().spdhg_net_adam(p.numel(), lr, 0.9, 0.999, 1e-8, self.step, _p(p),
                                          _p(self.m[key]), _p(self.v[key]), _p(grads[key]),
                                          None, _s()))
            pack(self.w32[name], ci, co, out=self.w16[name])
        return loss

    def gradients(self, img: torch.Tensor, target: torch.Tensor, scale: float,
                  part: Optional[torch.Tensor] = None):
        """Loss 0.5 |net(img) - target|^2 (scaled range) and its gradient with respect to
        every weight ([tap][co][ci], FP32) and bias (backpropagation through the layers in
        reverse order with the kernels' adjoints)."""
        nv = img.numel()
        _, a = self.forward(img, scale, keep=True)
        g_out = bf16(self.shape + (16,), self.device, zero=True)  # mse_grad writes channel 0
        _chk(lib().spdhg_net_mse_grad(nv, 16, _p(a["out"]), _p(img), _p(target), float(scale),
                                      _p(g_out), _p(self.lparts), _s()))
        if part is None:
            part = torch.empty(max(wgrad_part_floats(self.shape, ci, co) for _, ci, co, _ in LAYERS),
                               dtype=torch.float32, device=self.device)
        grads: Dict[str, torch.Tensor] = {}
        spec = {n: (ci, co, relu) for n, ci, co, relu in LAYERS}

        def back(name, inp, outp, gout, relu_applied):
            """Gradient through conv `name` (input inp, output outp): weights, bias, input."""
            ci, co, relu = spec[name]
            if relu:
                relu_bwd(outp, gout)
            dw, db = conv_wgrad(inp, gout, part)
            grads[f"{name}.w"], grads[f"{name}.b"] = dw, db
            wt = adjoint_weights(self.w16[name], ci, co)
            return conv_fwd(gout, wt, None, False, ci)

        g = back("c11", a["d1"], a["out"], g_out, False)
        g = back("c10", a["s1"], a["d1"], g, True)
        g_e1_skip = g  # d s1 / d e1 = identity
        g = back("c9", a["u1"], a["c9"], g.clone(), True)
        g = up2_adjoint(g)
        g = back("c8", a["s2"], a["d2"], g, True)
        g_e2_skip = g
        g = back("c7", a["u2"], a["c7"], g.clone(), True)
        g = up2_adjoint(g)
        g = back("c6", a["c5"], a["b"], g, True)
        g = back("c5", a["p2"], a["c5"], g, True)
        g = add(pool2_adjoint(g), g_e2_skip)
        g = back("c4", a["c3"], a["e2"], g, True)
        g = back("c3", a["p1"], a["c3"], g, True)
        g = add(pool2_adjoint(g), g_e1_skip)
        g = back("c2", a["c1"], a["e1"], g, True)
        back("c1", a["in"], a["c1"], g, True)
        return float(self.lparts.sum().item()), grads


# ---------------------------------------------------------------- data and experiment
def padded_shape(g) -> Tuple[int, int, int]:
    """Network volume for an image [nz][ny][nx]: [ny][nx][nz] with every size rounded up
    to a multiple of 4."""
    r4 = lambda n: (n + 3) // 4 * 4  # noqa: E731
    return r4(g.ny), r4(g.nx), r4(g.nz)


def to_net(img_zyx: torch.Tensor, shape) -> torch.Tensor:
    """Caller image [nz][ny][nx] -> zero-padded network volume [ny][nx][nz'] (FP32)."""
    nz, ny, nx = img_zyx.shape
    out = torch.zeros(shape, dtype=torch.float32, device=img_zyx.device)
    out[:ny, :nx, :nz] = img_zyx.permute(1, 2, 0)
    return out.contiguous()


def from_net(vol: torch.Tensor, g) -> torch.Tensor:
    return vol[:g.ny, :g.nx, :g.nz].permute(2, 0, 1).contiguous()


def normalised_backprojection(g, d, stats: Optional[torch.Tensor] = None) -> torch.Tensor:
    """(A^T b) / (A^T 1) on the voxels some ray reaches (0 elsewhere): the network input,
    computed by the library (spdhg_normalised_backprojection); `stats` (3 float64 on the
    device, optional) receives [sum, count, count / sum] over the positive voxels."""
    from .spdhg import normalised_backprojection as nbp
    out = torch.empty(g.image_shape, dtype=torch.float32, device=d["b"].device)
    if stats is None:
        stats = torch.empty(3, dtype=torch.float64, device=d["b"].device)
    return nbp(g, d["b"], d["mult"], out, stats)


def input_scale(nbp: torch.Tensor) -> float:
    """Scale that brings the network input to order one: 1 / mean over its support."""
    pos = nbp[nbp > 0]
    return 1.0 / float(pos.mean().item()) if pos.numel() else 1.0
