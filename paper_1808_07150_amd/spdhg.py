"""ctypes binding of libspdhg.so (include/spdhg.h).  Argument marshalling only: every
step of the reconstruction runs in the library's HIP kernels; PyTorch provides device
memory and the stream.  The binding fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspdhg.so")
MAX_SEG = 128

SPDHG_OK = 0
ERRORS = {-1: "SPDHG_E_ARG", -2: "SPDHG_E_SHAPE", -3: "SPDHG_E_DOMAIN", -4: "SPDHG_E_HIP",
          -5: "SPDHG_E_WORKSPACE", -6: "SPDHG_E_STATE", -7: "SPDHG_E_NOTIMPL"}

PRIOR = {"none": 0, "tv": 1, "atv": 2, "dtv": 3, "tgv": 4}
SAMPLING = {"uniform": 0, "balanced": 1, "custom": 2}

EXPORTED = ["spdhg_last_error", "spdhg_subset_bins", "spdhg_op_workspace_bytes",
            "spdhg_project", "spdhg_project_noalloc", "spdhg_backproject",
            "spdhg_normalised_backprojection", "spdhg_nnz",
            "spdhg_workspace_bytes", "spdhg_init", "spdhg_iterate", "spdhg_epoch",
            "spdhg_epoch_graph", "spdhg_graph_create", "spdhg_graph_epoch",
            "spdhg_graph_destroy", "spdhg_batch_epoch", "spdhg_pdhg_iterate", "spdhg_em_iterate",
            "spdhg_set_tuning", "spdhg_autotune", "spdhg_set_gather", "spdhg_get_tuning",
            "spdhg_set_walk",
            "spdhg_info",
            "spdhg_objective", "spdhg_gap", "spdhg_buffer", "spdhg_block_info", "spdhg_state_bytes",
            "spdhg_save_state", "spdhg_load_state", "spdhg_set_profiling",
            "spdhg_set_profiling_kinds", "spdhg_profile",
            "spdhg_destroy"]
PROF_KINDS = ("fwd", "bwd", "prior")


class SpdhgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class CGeom(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("vx", ctypes.c_double), ("vy", ctypes.c_double), ("vz", ctypes.c_double),
                ("n_rad", ctypes.c_int32), ("d_rad", ctypes.c_double),
                ("n_ang", ctypes.c_int32), ("n_seg", ctypes.c_int32),
                ("seg_planes", ctypes.c_int32 * MAX_SEG),
                ("seg_tan", ctypes.c_double * MAX_SEG),
                ("seg_pitch", ctypes.c_int32 * MAX_SEG),
                ("det_radius", ctypes.c_double), ("nonarc", ctypes.c_int32),
                ("oblique_s", ctypes.c_int32), ("span", ctypes.c_int32)]


class CParams(ctypes.Structure):
    _fields_ = [("n_subsets", ctypes.c_int32), ("prior", ctypes.c_int32),
                ("sampling", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("eta", ctypes.c_double),
                ("gamma_d", ctypes.c_double), ("gamma", ctypes.c_double),
                ("rho", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("power_iters", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("alpha1", ctypes.c_double), ("p_prior", ctypes.c_double),
                ("p_tgv_n", ctypes.c_double)]


_lib = None


def load_library() -> ctypes.CDLL:
    """Load the in-tree libspdhg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as "
                          f"g; g.build()'` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    G, Pm = ctypes.POINTER(CGeom), ctypes.POINTER(CParams)
    lib.spdhg_last_error.restype = ctypes.c_char_p
    lib.spdhg_last_error.argtypes = []
    lib.spdhg_subset_bins.restype = i64
    lib.spdhg_subset_bins.argtypes = [G, i32, i32]
    lib.spdhg_op_workspace_bytes.argtypes = [G, ctypes.POINTER(ctypes.c_size_t)]
    for name in ("spdhg_project", "spdhg_backproject"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [G, i32, i32, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.spdhg_project_noalloc.argtypes = [G, i32, i32, vp, vp, vp, vp]
    lib.spdhg_normalised_backprojection.argtypes = [G, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.spdhg_nnz.argtypes = [G, i32, i32, ctypes.POINTER(ctypes.c_double), vp,
                              ctypes.c_size_t, vp]
    lib.spdhg_workspace_bytes.argtypes = [G, Pm, ctypes.POINTER(ctypes.c_size_t)]
    lib.spdhg_init.argtypes = [ctypes.POINTER(vp), G, Pm, vp, vp, vp, vp, vp, vp,
                               ctypes.c_size_t, vp]
    lib.spdhg_iterate.argtypes = [vp, i64, vp]
    lib.spdhg_epoch.argtypes = [vp, i32, vp]
    lib.spdhg_epoch_graph.argtypes = [vp, i32, vp]
    lib.spdhg_em_iterate.argtypes = [vp, i64, vp]
    lib.spdhg_pdhg_iterate.argtypes = [vp, i64, vp]
    lib.spdhg_batch_epoch.argtypes = [ctypes.POINTER(vp), i32, i32, i32, i32, vp]
    lib.spdhg_graph_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp)]
    lib.spdhg_graph_epoch.argtypes = [vp, i32, vp]
    lib.spdhg_graph_destroy.argtypes = [vp]
    lib.spdhg_set_tuning.argtypes = [vp, i32]
    lib.spdhg_set_walk.argtypes = [vp, i32]
    lib.spdhg_autotune.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double), vp]
    lib.spdhg_set_gather.argtypes = [vp, i32]
    lib.spdhg_get_tuning.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.spdhg_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.spdhg_objective.argtypes = [vp, vp, vp, vp]
    lib.spdhg_gap.argtypes = [vp, ctypes.c_double, vp, vp]
    lib.spdhg_buffer.argtypes = [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(i64)]
    lib.spdhg_block_info.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    lib.spdhg_state_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.spdhg_save_state.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.spdhg_load_state.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.spdhg_set_profiling.argtypes = [vp, i32]
    lib.spdhg_set_profiling_kinds.argtypes = [vp, i32]
    lib.spdhg_profile.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    lib.spdhg_destroy.argtypes = [vp]
    for name in EXPORTED[2:]:
        if getattr(lib, name).restype is not ctypes.c_int64:
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != SPDHG_OK:
        raise SpdhgError(rc, load_library().spdhg_last_error().decode())


def cgeom(g) -> CGeom:
    """spdhg_geom from any object with the geometry fields (e.g. synth.Geometry)."""
    s = CGeom()
    s.nx, s.ny, s.nz = g.nx, g.ny, g.nz
    s.vx, s.vy, s.vz = g.vx, g.vy, g.vz
    s.n_rad, s.d_rad, s.n_ang = g.n_rad, g.d_rad, g.n_ang
    s.n_seg = len(g.seg_planes)
    if s.n_seg > MAX_SEG:
        raise ValueError(f"at most {MAX_SEG} segments")
    pitch = getattr(g, "seg_pitch", ()) or (1,) * s.n_seg
    for i, (n, t, pt) in enumerate(zip(g.seg_planes, g.seg_tan, pitch)):
        s.seg_planes[i] = n
        s.seg_tan[i] = t
        s.seg_pitch[i] = pt
    s.det_radius = float(getattr(g, "det_radius", 0.0))
    s.nonarc = int(bool(getattr(g, "nonarc", False)))
    s.oblique_s = int(bool(getattr(g, "oblique_s", False)))
    s.span = int(getattr(g, "span", 0))
    return s


def cparams(n_subsets: int, prior: str = "tv", sampling: str = "uniform", precond: bool = True,
            alpha: float = 0.1, eta: float = 1e-2, gamma_d: float = 1.0, gamma: float = 1.0,
            rho: float = 0.99, seed: int = 0, power_iters: int = 100,
            alpha1: float = 0.0, em: bool = False, p_prior: float = 0.5,
            p_tgv_n: float = 0.0, split_T: bool = False,
            compensated: bool = False) -> CParams:
    p = CParams()
    p.n_subsets = n_subsets
    p.prior = PRIOR[prior]
    p.sampling = SAMPLING[sampling]
    p.precond = 1 if precond else 0
    p.alpha, p.eta, p.gamma_d, p.gamma, p.rho = alpha, eta, gamma_d, gamma, rho
    p.seed = seed & 0xFFFFFFFFFFFFFFFF
    p.power_iters = power_iters
    p.alpha1 = alpha1
    # SPDHG_FLAG_EM, SPDHG_FLAG_TGV_SPLIT_T, SPDHG_FLAG_COMPENSATED
    p.flags = (1 if em else 0) | (2 if split_T else 0) | (4 if compensated else 0)
    p.p_prior = p_prior
    p.p_tgv_n = p_tgv_n
    return p


def _ptr(t: Optional[torch.Tensor], dtype=torch.float32):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the HIP device")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"tensor must be contiguous {dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def subset_bins(g, n_subsets: int, subset: int) -> int:
    return int(load_library().spdhg_subset_bins(ctypes.byref(cgeom(g)), n_subsets, subset))


def op_workspace_bytes(g) -> int:
    n = ctypes.c_size_t(0)
    _check(load_library().spdhg_op_workspace_bytes(ctypes.byref(cgeom(g)), ctypes.byref(n)))
    return int(n.value)


def aligned_workspace(nbytes: int, device) -> Tuple[torch.Tensor, int, int]:
    """A torch uint8 tensor holding a 256-byte aligned region of nbytes: (tensor, address,
    bytes).  Torch owns the memory; keep the tensor alive while the library uses it."""
    t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    base = t.data_ptr()
    return t, (base + 255) & ~255, int(nbytes)


def op_workspace(g, device) -> Tuple[torch.Tensor, int, int]:
    """Workspace of the stand-alone operator calls for geometry g."""
    return aligned_workspace(op_workspace_bytes(g), device)


def _ws_args(g, device, ws):
    if ws is None:
        ws = op_workspace(g, device)
    return ws, ctypes.c_void_p(ws[1]), ctypes.c_size_t(ws[2])


def spdhg_project(g, n_subsets: int, subset: int, mult: Optional[torch.Tensor],
                  x: torch.Tensor, y_out: torch.Tensor, stream=None, ws=None) -> torch.Tensor:
    """y_out = A_i x (spdhg_project).  `ws` is an op_workspace(g, device) triple, or None
    for a fresh one."""
    n = subset_bins(g, n_subsets, subset)
    if y_out.numel() != n or x.numel() != g.nx * g.ny * g.nz:
        raise ValueError("size mismatch")
    keep, wp, wn = _ws_args(g, x.device, ws)
    _check(load_library().spdhg_project(ctypes.byref(cgeom(g)), n_subsets, subset, _ptr(mult),
                                        _ptr(x), _ptr(y_out), wp, wn, _stream(stream)))
    return y_out


def spdhg_backproject(g, n_subsets: int, subset: int, mult: Optional[torch.Tensor],
                      y: torch.Tensor, x_out: torch.Tensor, stream=None, ws=None) -> torch.Tensor:
    """x_out = A_i^T y (spdhg_backproject)."""
    n = subset_bins(g, n_subsets, subset)
    if y.numel() != n or x_out.numel() != g.nx * g.ny * g.nz:
        raise ValueError("size mismatch")
    keep, wp, wn = _ws_args(g, y.device, ws)
    _check(load_library().spdhg_backproject(ctypes.byref(cgeom(g)), n_subsets, subset,
                                            _ptr(mult), _ptr(y), _ptr(x_out), wp, wn,
                                            _stream(stream)))
    return x_out


def normalised_backprojection(g, b: torch.Tensor, mult: torch.Tensor, out: torch.Tensor,
                              stats: torch.Tensor, stream=None, ws=None) -> torch.Tensor:
    """out = (A^T b) / (A^T 1) (0 where A^T 1 = 0); stats (3 float64 on the device) =
    [sum, count, count / sum] over the positive voxels."""
    if b.numel() != g.n_bins or mult.numel() != g.n_bins or out.numel() != g.n_vox:
        raise ValueError("size mismatch")
    if stats.numel() < 3:
        raise ValueError("stats needs 3 doubles")
    keep, wp, wn = _ws_args(g, b.device, ws)
    _check(load_library().spdhg_normalised_backprojection(
        ctypes.byref(cgeom(g)), _ptr(b), _ptr(mult), _ptr(out), _ptr(stats, torch.float64), wp,
        wn, _stream(stream)))
    return out


def spdhg_nnz(g, n_subsets: int, subset: int, stream=None, ws=None, device=None) -> int:
    """Nonzero count of A_i (taps inside the image with nonzero weight)."""
    out = ctypes.c_double()
    keep, wp, wn = _ws_args(g, device or torch.device("cuda", torch.cuda.current_device()), ws)
    _check(load_library().spdhg_nnz(ctypes.byref(cgeom(g)), n_subsets, subset,
                                    ctypes.byref(out), wp, wn, _stream(stream)))
    return int(out.value)


class Reconstruction:
    """One SPDHG reconstruction (spdhg_init ... spdhg_destroy).  The workspace is a
    torch uint8 tensor; b, r, mult, side and x are borrowed and must stay alive."""

    BUFFERS = {"y": 0, "z": 1, "T": 2, "sigma": 3, "prior_dual": 4, "w": 5, "q2": 6, "zw": 7,
               "z_lo": 8, "x_lo": 9}

    def __init__(self, g, params: CParams, b, r, mult, x, side=None, stream=None):
        lib = load_library()
        self.g = g
        self.params = params
        self._keep = (b, r, mult, x, side)
        self.x = x
        gs = cgeom(g)
        nbytes = ctypes.c_size_t(0)
        _check(lib.spdhg_workspace_bytes(ctypes.byref(gs), ctypes.byref(params),
                                         ctypes.byref(nbytes)))
        self.ws, aligned, _ = aligned_workspace(nbytes.value, x.device)
        ctx = ctypes.c_void_p()
        _check(lib.spdhg_init(ctypes.byref(ctx), ctypes.byref(gs), ctypes.byref(params),
                              _ptr(b), _ptr(r), _ptr(mult), _ptr(side), _ptr(x),
                              ctypes.c_void_p(aligned), nbytes.value, _stream(stream)))
        self.ctx = ctx

    def iterate(self, n_iters: int, stream=None):
        _check(load_library().spdhg_iterate(self.ctx, int(n_iters), _stream(stream)))

    def pdhg_iterate(self, n_iters: int, stream=None):
        """Deterministic PDHG iterations (Algorithm 1); the context must have one data block."""
        _check(load_library().spdhg_pdhg_iterate(self.ctx, int(n_iters), _stream(stream)))

    def em_iterate(self, n_subiters: int, stream=None):
        """EM-type sub-iterations (eq. OSEM on the context's subsets; MLEM with one subset)
        on the image; needs cparams(..., em=True)."""
        _check(load_library().spdhg_em_iterate(self.ctx, int(n_subiters), _stream(stream)))

    def epoch(self, n_epochs: int = 1, stream=None):
        _check(load_library().spdhg_epoch(self.ctx, int(n_epochs), _stream(stream)))

    def epoch_graph(self, n_epochs: int = 1):
        """spdhg_epoch as launches of the context's persistent HIP graph (bitwise the
        same iterations).  Launched on a side stream (created once, default priority) that
        waits for the current stream and that the current stream then waits for, so the
        call is asynchronous like epoch()."""
        cur = torch.cuda.current_stream(self.x.device)
        if getattr(self, "_graph_stream", None) is None:
            self._graph_stream = torch.cuda.Stream(device=self.x.device)
        side = self._graph_stream
        side.wait_stream(cur)
        _check(load_library().spdhg_epoch_graph(self.ctx, int(n_epochs),
                                                ctypes.c_void_p(side.cuda_stream)))
        cur.wait_stream(side)

    def set_tuning(self, fwd_split: int):
        _check(load_library().spdhg_set_tuning(self.ctx, int(fwd_split)))

    def set_walk(self, interleave: bool):
        """Forward walk's ray-to-lane mapping: False (default) runs of consecutive planes
        per lane where the geometry allows, True interleaved planes (bitwise the same)."""
        _check(load_library().spdhg_set_walk(self.ctx, int(bool(interleave))))

    def set_gather(self, gather: int):
        """Gather tiling: 0 automatic, 1 strips of 10 columns, 2 whole columns, 3 strips
        of 10 columns at four consecutive primary indices per workgroup."""
        _check(load_library().spdhg_set_gather(self.ctx, int(gather)))

    def tuning(self):
        """(ray-bundle split, gather tiling) in use."""
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(load_library().spdhg_get_tuning(self.ctx, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    def autotune(self, stream=None):
        """Time the ray-bundle splits of the subset projection and the gather tilings of
        the backprojection and keep the fastest; returns (split, ms per projection)."""
        s, ms = ctypes.c_int32(), ctypes.c_double()
        _check(load_library().spdhg_autotune(self.ctx, ctypes.byref(s), ctypes.byref(ms),
                                             _stream(stream)))
        return int(s.value), float(ms.value)

    def info(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(load_library().spdhg_info(self.ctx, ctypes.byref(a), ctypes.byref(b)))
        return int(a.value), int(b.value)

    @property
    def iters_per_epoch(self) -> int:
        return self.info()[0]

    def objective(self, x: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(4, dtype=torch.float64, device=self.x.device)
        _check(load_library().spdhg_objective(self.ctx, _ptr(x), _ptr(out, torch.float64),
                                              _stream(stream)))
        return out

    def gap(self, U: float, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """[gap, primal, dual, box term] of the current state for g = indicator of [0, U]."""
        if out is None:
            out = torch.empty(4, dtype=torch.float64, device=self.x.device)
        _check(load_library().spdhg_gap(self.ctx, float(U), _ptr(out, torch.float64),
                                        _stream(stream)))
        return out

    def buffer(self, name: str, caller_layout: bool = True) -> Optional[torch.Tensor]:
        """A copy of an internal array (y, z, T, sigma, prior_dual; TGV: w, q2, zw; with
        the compensated primal step: z_lo, x_lo, the low parts of z and the iterate).  The
        library stores images z-fastest [y][x][z] and sinograms [angle][radial][plane];
        with caller_layout the copy is returned as [z][y][x] / [angle][plane][radial]
        (fields with c components as [c][z][y][x])."""
        p, n = ctypes.c_void_p(), ctypes.c_int64()
        _check(load_library().spdhg_buffer(self.ctx, self.BUFFERS[name], ctypes.byref(p),
                                           ctypes.byref(n)))
        if not p.value or n.value == 0:
            return None
        out = torch.empty(int(n.value), dtype=torch.float32, device=self.x.device)
        torch.cuda.synchronize()
        _memcpy_d2d(out.data_ptr(), p.value, 4 * int(n.value))
        if not caller_layout:
            return out
        g = self.g
        n_planes = g.sino_shape[1] if hasattr(g, "sino_shape") else sum(g.seg_planes)
        if name in ("y", "sigma"):
            return out.view(g.n_ang, g.n_rad, n_planes).permute(0, 2, 1).contiguous()
        if name in ("prior_dual", "w", "q2", "zw"):
            c = int(n.value) // (g.nx * g.ny * g.nz)
            return out.view(c, g.ny, g.nx, g.nz).permute(0, 3, 1, 2).contiguous()
        return out.view(g.ny, g.nx, g.nz).permute(2, 0, 1).contiguous()

    def block_info(self, i: int):
        s, p, nrm = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(load_library().spdhg_block_info(self.ctx, i, ctypes.byref(s), ctypes.byref(p),
                                               ctypes.byref(nrm)))
        return s.value, p.value, nrm.value

    def state_bytes(self) -> int:
        n = ctypes.c_size_t()
        _check(load_library().spdhg_state_bytes(self.ctx, ctypes.byref(n)))
        return int(n.value)

    def save_state(self, stream=None) -> torch.Tensor:
        n = self.state_bytes()
        buf = torch.empty(n, dtype=torch.uint8, device=self.x.device)
        _check(load_library().spdhg_save_state(self.ctx, ctypes.c_void_p(buf.data_ptr()), n,
                                               _stream(stream)))
        return buf

    def load_state(self, buf: torch.Tensor, stream=None):
        _check(load_library().spdhg_load_state(self.ctx, ctypes.c_void_p(buf.data_ptr()),
                                               buf.numel(), _stream(stream)))

    def set_profiling(self, on: bool, kinds=PROF_KINDS):
        """Per-kernel timing on or off (totals cleared); `kinds`: the kernel kinds timed."""
        lib = load_library()
        _check(lib.spdhg_set_profiling_kinds(
            self.ctx, sum(1 << PROF_KINDS.index(k) for k in kinds)))
        _check(lib.spdhg_set_profiling(self.ctx, 1 if on else 0))

    def profile(self):
        """{kind: (total ms, launches)} of the kernels launched while profiling was on."""
        ms = (ctypes.c_double * len(PROF_KINDS))()
        n = (ctypes.c_int64 * len(PROF_KINDS))()
        _check(load_library().spdhg_profile(self.ctx, ms, n))
        return {k: (ms[i], int(n[i])) for i, k in enumerate(PROF_KINDS)}

    def close(self):
        if getattr(self, "ctx", None):
            load_library().spdhg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_hip = None


def _memcpy_d2d(dst: int, src: int, nbytes: int):
    """hipMemcpy device-to-device between raw pointers (blocking)."""
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    rc = _hip.hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), nbytes, 3)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")


def batch_epoch(recs, n_epochs: int = 1, n_streams: int = 4, graph: bool = False):
    """n_epochs epochs of every Reconstruction in `recs`, overlapped on worker streams
    (optionally recorded into one HIP graph).  Each result equals its solo run bitwise."""
    lib = load_library()
    arr = (ctypes.c_void_p * len(recs))(*[r.ctx for r in recs])
    dev = recs[0].x.device if recs else None
    cur = torch.cuda.current_stream(dev)
    if graph:
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(cur)
        with torch.cuda.stream(side):
            _check(lib.spdhg_batch_epoch(arr, len(recs), int(n_epochs), int(n_streams), 1,
                                         ctypes.c_void_p(side.cuda_stream)))
        cur.wait_stream(side)
    else:
        _check(lib.spdhg_batch_epoch(arr, len(recs), int(n_epochs), int(n_streams), 0,
                                     ctypes.c_void_p(cur.cuda_stream)))


class EpochGraph:
    """Persistent epoch graph (spdhg_graph_create) over Reconstructions of any shapes: one
    HIP graph, instantiated once; epoch(n) advances every problem n epochs, bitwise as solo
    spdhg_epoch calls.  Launched on a side stream (the default stream cannot run graphs
    captured elsewhere) that the current stream then waits for."""

    def __init__(self, recs):
        lib = load_library()
        self.recs = list(recs)
        arr = (ctypes.c_void_p * len(self.recs))(*[r.ctx for r in self.recs])
        g = ctypes.c_void_p()
        _check(lib.spdhg_graph_create(arr, len(self.recs), ctypes.byref(g)))
        self.g = g
        self.dev = self.recs[0].x.device
        self.side = torch.cuda.Stream(device=self.dev)

    def epoch(self, n_epochs: int = 1):
        cur = torch.cuda.current_stream(self.dev)
        self.side.wait_stream(cur)
        _check(load_library().spdhg_graph_epoch(self.g, int(n_epochs),
                                                ctypes.c_void_p(self.side.cuda_stream)))
        cur.wait_stream(self.side)

    def close(self):
        if getattr(self, "g", None):
            torch.cuda.synchronize(self.dev)
            load_library().spdhg_graph_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
