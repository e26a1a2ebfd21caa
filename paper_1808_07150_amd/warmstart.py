"""Warm-start network for SPDHG (not part of the paper's method).

A 3-level 3-D convolutional encoder-decoder (channels 16/32/64, 3x3x3 kernels, BF16
weights and activations with FP32 accumulation on the MFMA units) maps the normalised
backprojection (A^T b) / (A^T 1) of the data to an initial image; SPDHG (Algorithm 2)
then runs from that image unchanged.  The network runs in libspdhg.so (include/
spdhg_net.h: spdhg_ws_infer, spdhg_ws_gradients, spdhg_ws_train_step sequence its
layers, backpropagation and Adam); this module holds the parameter blobs and
workspaces in torch tensors (device memory only) and marshals the calls.

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
                "spdhg_net_mse_grad", "spdhg_net_adam", "spdhg_net_pack_weights",
                "spdhg_ws_param_count", "spdhg_ws_param_offsets", "spdhg_ws_pack",
                "spdhg_ws_workspace_bytes", "spdhg_ws_infer", "spdhg_ws_gradients",
                "spdhg_ws_train_step"]

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
    i64p = ctypes.POINTER(ctypes.c_int64)
    L.spdhg_ws_param_count.argtypes = [i64p, i64p]
    L.spdhg_ws_param_offsets.argtypes = [i32, i64p, i64p, i64p]
    L.spdhg_ws_pack.argtypes = [vp, vp, vp]
    L.spdhg_ws_workspace_bytes.argtypes = [dims, i32, ctypes.POINTER(ctypes.c_size_t)]
    L.spdhg_ws_infer.argtypes = [dims, vp, vp, f32, vp, vp, vp, ctypes.c_size_t, vp]
    L.spdhg_ws_gradients.argtypes = [dims, vp, vp, f32, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    L.spdhg_ws_train_step.argtypes = [dims, vp, vp, vp, vp, i64, f32, f32, vp, vp, vp, vp,
                                      ctypes.c_size_t, vp]
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
def param_layout():
    """(n32, n16, {layer: (w32 offset, b32 offset, w16 offset)}) of the parameter blobs."""
    n32, n16 = ctypes.c_int64(), ctypes.c_int64()
    _chk(lib().spdhg_ws_param_count(ctypes.byref(n32), ctypes.byref(n16)))
    offs = {}
    for l, (name, *_) in enumerate(LAYERS):
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _chk(lib().spdhg_ws_param_offsets(l, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        offs[name] = (a.value, b.value, c.value)
    return n32.value, n16.value, offs


class WarmStartNet:
    """Parameter blobs (FP32 masters with per-layer views, packed BF16 copies, Adam
    moments) and workspaces of the encoder-decoder on one volume size; the library runs
    the network (spdhg_ws_infer, spdhg_ws_gradients, spdhg_ws_train_step)."""

    def __init__(self, shape: Tuple[int, int, int], device, seed: int = 0):
        ny, nx, nz = shape
        if ny % 4 or nx % 4 or nz % 4:
            raise ValueError("volume sizes must be divisible by 4 (two poolings)")
        self.shape, self.device = tuple(shape), device
        n32, n16, offs = param_layout()
        self.p32 = torch.zeros(n32, dtype=torch.float32, device=device)
        self.w16blob = torch.zeros(n16, dtype=torch.int16, device=device)
        self.w32: Dict[str, torch.Tensor] = {}
        self.b32: Dict[str, torch.Tensor] = {}
        self.w16: Dict[str, torch.Tensor] = {}
        g = torch.Generator(device="cpu")
        g.manual_seed(seed)
        for name, ci, co, relu in LAYERS:
            ow, ob, o16 = offs[name]
            nw = 27 * ci * co
            self.w32[name] = self.p32[ow:ow + nw].view(27, co, ci)
            self.b32[name] = self.p32[ob:ob + co]
            self.w16[name] = self.w16blob[o16:o16 + nw]
            # He initialisation for ReLU layers; the last (linear) layer starts at zero so
            # the untrained network returns its input image
            std = math.sqrt(2.0 / (27 * ci)) if relu else 0.0
            self.w32[name].copy_(torch.randn((27, co, ci), generator=g) * std)
        self.pack()
        self.m = torch.zeros_like(self.p32)
        self.v = torch.zeros_like(self.p32)
        self.step = 0
        self.loss_dev = torch.zeros(1, dtype=torch.float64, device=device)
        self._ws = {}

    def _dims(self):
        return (ctypes.c_int32 * 3)(*self.shape)

    def _workspace(self, train: bool):
        if train not in self._ws:
            from .spdhg import aligned_workspace
            nb = ctypes.c_size_t()
            _chk(lib().spdhg_ws_workspace_bytes(self._dims(), int(train), ctypes.byref(nb)))
            self._ws[train] = aligned_workspace(nb.value, self.device)
        return self._ws[train]

    def pack(self):
        """Packed BF16 weights from the FP32 masters (after editing w32 directly)."""
        _chk(lib().spdhg_ws_pack(_p(self.p32), _p(self.w16blob), _s()))

    def forward(self, img: torch.Tensor, scale: float) -> torch.Tensor:
        """Network output image from `img` ([ny][nx][nz] FP32, z fastest) scaled by
        `scale` into the network's range."""
        out = torch.empty_like(img)
        _, addr, nb = self._workspace(False)
        _chk(lib().spdhg_ws_infer(self._dims(), _p(self.p32), _p(self.w16blob), float(scale),
                                  _p(img), _p(out), ctypes.c_void_p(addr), nb, _s()))
        return out

    def gradients(self, img: torch.Tensor, target: torch.Tensor, scale: float):
        """Loss 0.5 |net(img) - target|^2 (scaled range) and its gradient with respect to
        every weight ([tap][co][ci], FP32) and bias."""
        grads = torch.empty_like(self.p32)
        _, addr, nb = self._workspace(True)
        _chk(lib().spdhg_ws_gradients(self._dims(), _p(self.p32), _p(self.w16blob),
                                      float(scale), _p(img), _p(target), _p(grads),
                                      _p(self.loss_dev), ctypes.c_void_p(addr), nb, _s()))
        _, _, offs = param_layout()
        out = {}
        for name, ci, co, _ in LAYERS:
            ow, ob, _ = offs[name]
            out[f"{name}.w"] = grads[ow:ow + 27 * ci * co].view(27, co, ci)
            out[f"{name}.b"] = grads[ob:ob + co]
        return float(self.loss_dev.item()), out

    def train_step(self, img: torch.Tensor, target: torch.Tensor, scale: float,
                   lr: float = 1e-3) -> float:
        """One Adam step on 0.5 |net(img) - target|^2 (in the scaled range); returns the
        loss before the step."""
        self.step += 1
        _, addr, nb = self._workspace(True)
        _chk(lib().spdhg_ws_train_step(self._dims(), _p(self.p32), _p(self.w16blob),
                                       _p(self.m), _p(self.v), self.step, float(lr),
                                       float(scale), _p(img), _p(target), _p(self.loss_dev),
                                       ctypes.c_void_p(addr), nb, _s()))
        return float(self.loss_dev.item())


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
