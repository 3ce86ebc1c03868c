"""Python binding of libgramct (include/gramct.h).

Argument marshalling only: every step runs in the HIP kernels of
libgramct.so.  Device memory comes from torch tensors (on the current
device); every call is issued on torch's current stream.  There is no CPU
fallback: if the library is missing, importing this module raises.

Function names mirror the C ABI without the ``gct_`` prefix
(``gram_build`` calls ``gct_gram_build`` and so on).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgramct.so")

GCT_OK, GCT_EINVAL, GCT_EHIP, GCT_ENOTCONV, GCT_EBREAKDOWN = 0, -1, -2, -3, -4
F32, F64 = 0, 1
OP_GRAM_BUILD, OP_GRAM_SPECTRUM, OP_GRAM_APPLY, OP_PREFILTER, OP_BACKPROJECT, OP_FORWARD, OP_CG = range(7)


class GramctError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gramct error {code}: {msg}")
        self.code = code


class _Geometry(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("lambda_x", ctypes.c_double * 2),
                ("n_angles", ctypes.c_int32), ("theta", ctypes.POINTER(ctypes.c_double)),
                ("lambda_y", ctypes.c_double), ("M", ctypes.c_int32),
                ("zeta_blur", ctypes.c_double), ("prefilter_K", ctypes.c_int32)]


class _PlanInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("n_angles", ctypes.c_int32), ("M", ctypes.c_int32),
                ("prefilter_K", ctypes.c_int32), ("fft_size", ctypes.c_int32),
                ("gram_elems", ctypes.c_int64), ("spectrum_elems", ctypes.c_int64),
                ("image_elems", ctypes.c_int64), ("sino_elems", ctypes.c_int64),
                ("prefiltered_elems", ctypes.c_int64), ("gram_symmetry", ctypes.c_int32)]


class _CGResult(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("rel_res", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("rel_res0", ctypes.c_double),
                ("fell_back", ctypes.c_int32)]


class _BatchInfo(ctypes.Structure):
    _fields_ = [("slices", ctypes.c_int32), ("groups", ctypes.c_int32),
                ("image_elems", ctypes.c_int64), ("gram_elems", ctypes.c_int64),
                ("spectrum_elems", ctypes.c_int64)]


class _UNetConfig(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("base_channels", ctypes.c_int32),
                ("height", ctypes.c_int32), ("width", ctypes.c_int32), ("max_batch", ctypes.c_int32)]


class _UNetLayer(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("taps", ctypes.c_int32), ("in_channels", ctypes.c_int32),
                ("out_channels", ctypes.c_int32), ("weight_offset", ctypes.c_int64),
                ("bias_offset", ctypes.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    L.gct_last_error.restype = ctypes.c_char_p
    L.gct_plan_create.argtypes = [ctypes.POINTER(_Geometry), ctypes.POINTER(vp)]
    L.gct_plan_create_detector.argtypes = [ctypes.POINTER(_Geometry), i32, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(vp)]
    L.gct_plan_destroy.argtypes = [vp]
    L.gct_plan_get_info.argtypes = [vp, ctypes.POINTER(_PlanInfo)]
    L.gct_plan_device_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.gct_batch_device_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.gct_workspace_size.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.gct_workspace_size.restype = ctypes.c_size_t
    L.gct_gram_build.argtypes = [vp, ctypes.c_int, vp, vp]
    L.gct_gram_spectrum.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    L.gct_gram_apply.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, vp]
    L.gct_gram_apply_static.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    L.gct_prefilter.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.gct_backproject_boxspline.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    L.gct_forward_project.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.gct_cg_solve.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.c_int, dbl, i32, i32,
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_CGResult), vp, vp]
    L.gct_sd_solve.argtypes = L.gct_cg_solve.argtypes
    L.gct_plan_autotune.argtypes = [vp, ctypes.c_int, vp, vp, i32, ctypes.POINTER(i32), vp]
    L.gct_plan_set_fft_elems.argtypes = [vp, ctypes.c_int, i32]
    L.gct_plan_set_pass_elems.argtypes = [vp, ctypes.c_int, i32, i32]
    L.gct_plan_get_pass_elems.argtypes = [vp, ctypes.c_int, ctypes.POINTER(i32)]
    L.gct_plan_get_bp_shape.argtypes = [vp, ctypes.c_int, ctypes.POINTER(i32)]
    L.gct_batch_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp)]
    L.gct_batch_destroy.argtypes = [vp]
    L.gct_batch_get_info.argtypes = [vp, ctypes.POINTER(_BatchInfo), ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]
    L.gct_batch_workspace_size.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.gct_batch_workspace_size.restype = ctypes.c_size_t
    L.gct_batch_gram_build.argtypes = [vp, ctypes.c_int, vp, vp]
    L.gct_batch_gram_spectrum.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp]
    L.gct_batch_gram_apply.argtypes = [vp, ctypes.c_int, vp, vp, vp, vp, vp]
    L.gct_batch_cg_solve.argtypes = [vp, ctypes.c_int, vp, vp, vp, dbl, i32, i32,
                                     ctypes.POINTER(_CGResult), vp, vp]
    L.gct_batch_cg_solve_x0.argtypes = [vp, ctypes.c_int, vp, vp, vp, dbl, i32, i32,
                                        ctypes.POINTER(_CGResult), vp, vp]
    L.gct_batch_autotune.argtypes = [vp, ctypes.c_int, vp, vp, i32, ctypes.POINTER(i32), vp]
    L.gct_batch_get_pass_elems.argtypes = [vp, ctypes.c_int, ctypes.POINTER(i32)]
    L.gct_host_boxspline_eval.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int, dbl,
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_double)]
    L.gct_host_bp_weights.argtypes = [ctypes.POINTER(_Geometry), ctypes.c_int, dbl,
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int)]
    L.gct_host_degree.argtypes = [dbl, dbl]
    L.gct_host_degree.restype = ctypes.c_int
    flt = ctypes.c_float
    L.gct_unet_create.argtypes = [ctypes.POINTER(_UNetConfig), ctypes.POINTER(vp)]
    L.gct_unet_destroy.argtypes = [vp]
    L.gct_unet_param_count.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.gct_unet_layer_count.argtypes = [vp, ctypes.POINTER(i32)]
    L.gct_unet_layer_info.argtypes = [vp, i32, ctypes.POINTER(_UNetLayer)]
    L.gct_unet_set_params.argtypes = [vp, vp, vp]
    L.gct_unet_get_params.argtypes = [vp, vp, vp]
    L.gct_unet_get_grads.argtypes = [vp, vp, vp]
    L.gct_unet_get_moments.argtypes = [vp, vp, vp, vp]
    L.gct_unet_set_moments.argtypes = [vp, vp, vp, vp]
    L.gct_unet_forward.argtypes = [vp, i32, vp, flt, flt, vp, vp]
    L.gct_unet_backward.argtypes = [vp, i32, vp, vp, vp, vp]
    L.gct_unet_adam_step.argtypes = [vp, flt, flt, flt, flt, i32, vp]
    return L


lib = _load()


def _check(rc):
    if rc != GCT_OK:
        raise GramctError(rc, lib.gct_last_error().decode())
    return rc


def _dt(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _ptr(t: torch.Tensor, n: int | None = None, dtype=None) -> int:
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if n is not None and t.numel() < n:
        raise ValueError(f"tensor has {t.numel()} elements, need {n}")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _geometry_struct(N, theta, M, ly, zeta, lx, K):
    th = np.ascontiguousarray(theta, dtype=np.float64)
    g = _Geometry()
    g.N, g.n_angles, g.M, g.prefilter_K = int(N), int(th.size), int(M), int(K)
    g.lambda_x[0], g.lambda_x[1] = float(lx[0]), float(lx[1])
    g.lambda_y, g.zeta_blur = float(ly), float(zeta)
    g.theta = th.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return g, th


@dataclass
class PlanInfo:
    N: int
    n_angles: int
    M: int
    prefilter_K: int
    fft_size: int
    gram_elems: int
    spectrum_elems: int
    image_elems: int
    sino_elems: int
    prefiltered_elems: int
    gram_symmetry: int  # 8: one octant of Gram taps evaluated; 2: half of them


class Plan:
    """gct_plan: geometry of Sec. 2 and the per-angle tables on the device.
    The detector kernel is the blur box of width zeta, or `boxes`, a list of
    (width, height) pairs (gct_plan_create_detector)."""

    def __init__(self, N, theta, M, ly=1.0, zeta=0.0, lx=(1.0, 1.0), K=40, boxes=None):
        g, th = _geometry_struct(N, theta, M, ly, zeta, lx, K)
        h = ctypes.c_void_p()
        if boxes:
            P = ctypes.POINTER(ctypes.c_double)
            w = np.ascontiguousarray([b[0] for b in boxes], dtype=np.float64)
            ht = np.ascontiguousarray([b[1] for b in boxes], dtype=np.float64)
            _check(lib.gct_plan_create_detector(ctypes.byref(g), len(boxes), w.ctypes.data_as(P),
                                                ht.ctypes.data_as(P), ctypes.byref(h)))
        else:
            _check(lib.gct_plan_create(ctypes.byref(g), ctypes.byref(h)))
        self.boxes = [tuple(map(float, b)) for b in boxes] if boxes else None
        self._h = h
        self.theta = th
        self.N, self.M, self.ly, self.zeta, self.lx, self.K = int(N), int(M), float(ly), float(zeta), tuple(lx), int(K)
        pi = _PlanInfo()
        _check(lib.gct_plan_get_info(self._h, ctypes.byref(pi)))
        self.info = PlanInfo(*[getattr(pi, f[0]) for f in _PlanInfo._fields_])

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.gct_plan_destroy(h)
            self._h = None

    def workspace_size(self, op: int, dtype=torch.float32) -> int:
        return int(lib.gct_workspace_size(self._h, op, F32 if dtype == torch.float32 else F64))

    def device_bytes(self) -> int:
        """Bytes of device memory the plan's tables hold."""
        v = ctypes.c_int64()
        _check(lib.gct_plan_device_bytes(self._h, ctypes.byref(v)))
        return int(v.value)

    def workspace(self, op: int, dtype=torch.float32, device=None) -> torch.Tensor:
        n = max(self.workspace_size(op, dtype), 256)
        return torch.empty(n, dtype=torch.uint8, device=device or "cuda")


def gram_build(plan: Plan, G: torch.Tensor):
    _check(lib.gct_gram_build(plan.handle, _dt(G), _ptr(G, plan.info.gram_elems), _stream()))
    return G


def gram_spectrum(plan: Plan, G: torch.Tensor, Ghat: torch.Tensor, ws: torch.Tensor):
    dt = _dt(G)
    _check(lib.gct_gram_spectrum(plan.handle, dt, _ptr(G, plan.info.gram_elems),
                                 _ptr(Ghat, plan.info.spectrum_elems, G.dtype),
                                 _ptr(ws, plan.workspace_size(OP_GRAM_SPECTRUM, G.dtype)), _stream()))
    return Ghat


def gram_apply(plan: Plan, Ghat: torch.Tensor, c: torch.Tensor, y: torch.Tensor, ws: torch.Tensor):
    dt = _dt(c)
    _check(lib.gct_gram_apply(plan.handle, dt, _ptr(Ghat, plan.info.spectrum_elems, c.dtype),
                              _ptr(c, plan.info.image_elems), _ptr(y, plan.info.image_elems, c.dtype),
                              _ptr(ws, plan.workspace_size(OP_GRAM_APPLY, c.dtype)), _stream()))
    return y


def gram_apply_static(plan: Plan, Ghat: torch.Tensor, c: torch.Tensor, y: torch.Tensor):
    """gram_apply with the library's static scratch (no workspace)."""
    _check(lib.gct_gram_apply_static(plan.handle, _dt(c), _ptr(Ghat, plan.info.spectrum_elems, c.dtype),
                                     _ptr(c, plan.info.image_elems), _ptr(y, plan.info.image_elems, c.dtype),
                                     _stream()))
    return y


def prefilter(plan: Plan, g: torch.Tensor, p: torch.Tensor):
    _check(lib.gct_prefilter(plan.handle, _dt(g), _ptr(g, plan.info.sino_elems),
                             _ptr(p, plan.info.prefiltered_elems, g.dtype), _stream()))
    return p


def backproject_boxspline(plan: Plan, g: torch.Tensor, b: torch.Tensor, ws: torch.Tensor):
    _check(lib.gct_backproject_boxspline(plan.handle, _dt(g), _ptr(g, plan.info.sino_elems),
                                         _ptr(b, plan.info.image_elems, g.dtype),
                                         _ptr(ws, plan.workspace_size(OP_BACKPROJECT, g.dtype)),
                                         _stream()))
    return b


def forward_project(plan: Plan, c: torch.Tensor, g: torch.Tensor):
    _check(lib.gct_forward_project(plan.handle, _dt(c), _ptr(c, plan.info.image_elems),
                                   _ptr(g, plan.info.sino_elems, c.dtype), _stream()))
    return g


@dataclass
class CGResult:
    iters: int
    status: int
    rel_res: float
    rel_res_true: float
    rel_res0: float
    fell_back: int
    history: np.ndarray


def cg_solve(plan: Plan, Ghat: torch.Tensor, b: torch.Tensor, x: torch.Tensor, ws: torch.Tensor,
             use_x0: bool = False, rtol: float = 1e-4, max_iter: int = 1000,
             check_every: int = 8, raise_on_error: bool = False) -> CGResult:
    """Blocks until the solve ends.  Returns the result; GCT_ENOTCONV /
    GCT_EBREAKDOWN are reported in .status unless raise_on_error."""
    return _solve(lib.gct_cg_solve, plan, Ghat, b, x, ws, use_x0, rtol, max_iter, check_every, raise_on_error)


def sd_solve(plan: Plan, Ghat: torch.Tensor, b: torch.Tensor, x: torch.Tensor, ws: torch.Tensor,
             use_x0: bool = False, rtol: float = 1e-4, max_iter: int = 1000,
             check_every: int = 8, raise_on_error: bool = False) -> CGResult:
    """Steepest descent (the paper's solver); arguments and result as
    cg_solve (ws: a CG workspace)."""
    return _solve(lib.gct_sd_solve, plan, Ghat, b, x, ws, use_x0, rtol, max_iter, check_every, raise_on_error)


def _solve(fn, plan, Ghat, b, x, ws, use_x0, rtol, max_iter, check_every, raise_on_error) -> CGResult:
    dt = _dt(b)
    hist = np.zeros(max_iter + 1)
    res = _CGResult()
    rc = fn(plan.handle, dt, _ptr(Ghat, plan.info.spectrum_elems, b.dtype),
                          _ptr(b, plan.info.image_elems), _ptr(x, plan.info.image_elems, b.dtype),
                          int(bool(use_x0)), float(rtol), int(max_iter), int(check_every),
                          hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(res),
                          _ptr(ws, plan.workspace_size(OP_CG, b.dtype)), _stream())
    if rc not in (GCT_OK, GCT_ENOTCONV, GCT_EBREAKDOWN) or (raise_on_error and rc != GCT_OK):
        _check(rc)
    return CGResult(res.iters, res.status, res.rel_res, res.rel_res_true, res.rel_res0,
                    res.fell_back, hist[: res.iters + 1].copy())


def plan_autotune(plan: Plan, Ghat: torch.Tensor, ws: torch.Tensor, reps: int = 3):
    """Pick the fastest elements-per-thread of the apply passes for Ghat's
    dtype; returns the apply's choice as (row passes, column pass).  ws: a CG
    workspace of the plan."""
    ch = ctypes.c_int32(0)
    _check(lib.gct_plan_autotune(plan.handle, _dt(Ghat), _ptr(Ghat, plan.info.spectrum_elems),
                                 _ptr(ws, plan.workspace_size(OP_CG, Ghat.dtype)), int(reps),
                                 ctypes.byref(ch), _stream()))
    return plan_get_pass_elems(plan, Ghat.dtype)[:2]


def plan_set_fft_elems(plan: Plan, elems: int, dtype=torch.float32):
    """Force the elements per thread of every transform pass (0: default)."""
    _check(lib.gct_plan_set_fft_elems(plan.handle, F32 if dtype == torch.float32 else F64, int(elems)))


def plan_set_pass_elems(plan: Plan, rows: int, cols: int, dtype=torch.float32):
    """Force the elements per thread of the row passes and of the column
    pass separately (0: default)."""
    _check(lib.gct_plan_set_pass_elems(plan.handle, F32 if dtype == torch.float32 else F64, int(rows), int(cols)))


def plan_get_pass_elems(plan: Plan, dtype=torch.float32):
    """(apply rows, apply cols, CG rows, CG cols) elements per thread."""
    out = (ctypes.c_int32 * 4)()
    _check(lib.gct_plan_get_pass_elems(plan.handle, F32 if dtype == torch.float32 else F64, out))
    return tuple(int(v) for v in out)


def plan_get_bp_shape(plan: Plan, dtype=torch.float32):
    """Back-projection launch shape: (angles per chunk of the tiled kernel,
    0 when the per-angle kernel runs; angle groups; per-angle tile side, 0
    when the tiled kernel runs; breakpoints held in registers by the tiled
    kernel, 0 when searched in memory or when it does not run)."""
    out = (ctypes.c_int32 * 4)()
    _check(lib.gct_plan_get_bp_shape(plan.handle, F32 if dtype == torch.float32 else F64, out))
    return tuple(int(v) for v in out)


# ---------------------------------------------------------------------------
# Batches of independent slices
# ---------------------------------------------------------------------------
class Batch:
    """gct_batch over existing plans (kept alive by this object).  Data
    arrays are packed: slice i occupies [offset_i, offset_i + size_i)."""

    def __init__(self, plans):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib.gct_batch_create(arr, len(self.plans), ctypes.byref(h)))
        self._h = h
        info = _BatchInfo()
        S = len(self.plans)
        self.image_offsets = np.zeros(S, np.int64)
        self.gram_offsets = np.zeros(S, np.int64)
        self.spectrum_offsets = np.zeros(S, np.int64)
        _check(lib.gct_batch_get_info(h, ctypes.byref(info), self.image_offsets.ctypes.data,
                                      self.gram_offsets.ctypes.data, self.spectrum_offsets.ctypes.data))
        self.slices, self.groups = info.slices, info.groups
        self.image_elems, self.gram_elems, self.spectrum_elems = (info.image_elems, info.gram_elems,
                                                                  info.spectrum_elems)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.gct_batch_destroy(h)
            self._h = None

    def workspace_size(self, op: int, dtype=torch.float32) -> int:
        return int(lib.gct_batch_workspace_size(self._h, op, F32 if dtype == torch.float32 else F64))

    def device_bytes(self) -> int:
        """Bytes of device memory the batch's maps and descriptors hold."""
        v = ctypes.c_int64()
        _check(lib.gct_batch_device_bytes(self._h, ctypes.byref(v)))
        return int(v.value)

    def workspace(self, op: int, dtype=torch.float32) -> torch.Tensor:
        return torch.empty(max(self.workspace_size(op, dtype), 256), dtype=torch.uint8, device="cuda")

    def image(self, packed: torch.Tensor, i: int) -> torch.Tensor:
        N = self.plans[i].N
        o = int(self.image_offsets[i])
        return packed[o:o + N * N].view(N, N)


def batch_gram_build(batch: Batch, G: torch.Tensor):
    _check(lib.gct_batch_gram_build(batch.handle, _dt(G), _ptr(G, batch.gram_elems), _stream()))
    return G


def batch_gram_spectrum(batch: Batch, G: torch.Tensor, Ghat: torch.Tensor, ws: torch.Tensor):
    _check(lib.gct_batch_gram_spectrum(batch.handle, _dt(G), _ptr(G, batch.gram_elems),
                                       _ptr(Ghat, batch.spectrum_elems, G.dtype),
                                       _ptr(ws, batch.workspace_size(OP_GRAM_SPECTRUM, G.dtype)),
                                       _stream()))
    return Ghat


def batch_gram_apply(batch: Batch, Ghat: torch.Tensor, c: torch.Tensor, y: torch.Tensor,
                     ws: torch.Tensor):
    _check(lib.gct_batch_gram_apply(batch.handle, _dt(c), _ptr(Ghat, batch.spectrum_elems, c.dtype),
                                    _ptr(c, batch.image_elems), _ptr(y, batch.image_elems, c.dtype),
                                    _ptr(ws, batch.workspace_size(OP_GRAM_APPLY, c.dtype)), _stream()))
    return y


def batch_cg_solve(batch: Batch, Ghat: torch.Tensor, b: torch.Tensor, x: torch.Tensor,
                   ws: torch.Tensor, rtol: float = 1e-4, max_iter: int = 1000,
                   check_every: int = 8, use_x0: bool = False) -> list:
    """CG on every slice, from zero or (use_x0) from the iterates in x."""
    res = (_CGResult * batch.slices)()
    fn = lib.gct_batch_cg_solve_x0 if use_x0 else lib.gct_batch_cg_solve
    rc = fn(batch.handle, _dt(b), _ptr(Ghat, batch.spectrum_elems, b.dtype),
                                _ptr(b, batch.image_elems), _ptr(x, batch.image_elems, b.dtype),
                                float(rtol), int(max_iter), int(check_every), res,
                                _ptr(ws, batch.workspace_size(OP_CG, b.dtype)), _stream())
    if rc not in (GCT_OK, GCT_ENOTCONV, GCT_EBREAKDOWN):
        _check(rc)
    return [CGResult(r.iters, r.status, r.rel_res, r.rel_res_true, r.rel_res0, r.fell_back,
                     np.zeros(0)) for r in res]


def batch_autotune(batch: Batch, Ghat: torch.Tensor, ws: torch.Tensor, reps: int = 3) -> list:
    chosen = (ctypes.c_int32 * batch.groups)()
    _check(lib.gct_batch_autotune(batch.handle, _dt(Ghat), _ptr(Ghat, batch.spectrum_elems),
                                  _ptr(ws, batch.workspace_size(OP_CG, Ghat.dtype)), int(reps),
                                  chosen, _stream()))
    return list(chosen)


def batch_get_pass_elems(batch: Batch, dtype=torch.float32) -> list:
    """[(row passes, column pass)] elements per thread per FFT size."""
    out = (ctypes.c_int32 * (2 * batch.groups))()
    _check(lib.gct_batch_get_pass_elems(batch.handle, F32 if dtype == torch.float32 else F64, out))
    return [(int(out[2 * i]), int(out[2 * i + 1])) for i in range(batch.groups)]


# C-ABI names
gct_gram_build = gram_build
gct_gram_spectrum = gram_spectrum
gct_gram_apply = gram_apply
gct_gram_apply_static = gram_apply_static
gct_prefilter = prefilter
gct_backproject_boxspline = backproject_boxspline
gct_forward_project = forward_project
gct_cg_solve = cg_solve
gct_sd_solve = sd_solve
gct_batch_gram_build = batch_gram_build
gct_batch_gram_spectrum = batch_gram_spectrum
gct_batch_gram_apply = batch_gram_apply
gct_batch_cg_solve = batch_cg_solve
gct_batch_autotune = batch_autotune


# ---------------------------------------------------------------------------
# Host-only helpers (include/gramct_host.h)
# ---------------------------------------------------------------------------
def host_boxspline_eval(dirs, x, scale=1.0) -> np.ndarray:
    d = np.ascontiguousarray(dirs, dtype=np.float64)
    xs = np.ascontiguousarray(np.atleast_1d(x), dtype=np.float64)
    out = np.zeros_like(xs)
    P = ctypes.POINTER(ctypes.c_double)
    _check(lib.gct_host_boxspline_eval(d.ctypes.data_as(P), d.size, float(scale),
                                       xs.ctypes.data_as(P), xs.size, out.ctypes.data_as(P)))
    return out


def host_bp_weights(N, theta, M, angle, t, ly=1.0, zeta=0.0, lx=(1.0, 1.0), K=40):
    g, th = _geometry_struct(N, theta, M, ly, zeta, lx, K)
    w = np.zeros(64)
    jlo, nw = ctypes.c_int(), ctypes.c_int()
    _check(lib.gct_host_bp_weights(ctypes.byref(g), int(angle), float(t),
                                   w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   ctypes.byref(jlo), ctypes.byref(nw)))
    del th
    return jlo.value, w[: nw.value].copy()


def host_degree(theta: float, zeta: float) -> int:
    return int(lib.gct_host_degree(float(theta), float(zeta)))


# ---------------------------------------------------------------------------
# Warm-start U-Net (include/gramct_unet.h)
# ---------------------------------------------------------------------------
UNET_CONV3, UNET_UPCONV, UNET_FINAL = 0, 1, 2


class UNet:
    """gct_unet: parameters, moments and activations for up to max_batch
    images of height x width live in the library's device buffers."""

    def __init__(self, levels=4, base_channels=32, height=256, width=256, max_batch=1):
        cfg = _UNetConfig(int(levels), int(base_channels), int(height), int(width), int(max_batch))
        h = ctypes.c_void_p()
        _check(lib.gct_unet_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.levels, self.base_channels = int(levels), int(base_channels)
        self.height, self.width, self.max_batch = int(height), int(width), int(max_batch)
        n = ctypes.c_int64()
        _check(lib.gct_unet_param_count(h, ctypes.byref(n)))
        self.n_params = int(n.value)
        k = ctypes.c_int32()
        _check(lib.gct_unet_layer_count(h, ctypes.byref(k)))
        self.layers = []
        for i in range(k.value):
            ly = _UNetLayer()
            _check(lib.gct_unet_layer_info(h, i, ctypes.byref(ly)))
            self.layers.append(dict(kind=ly.kind, taps=ly.taps, cin=ly.in_channels,
                                    cout=ly.out_channels, w_off=ly.weight_offset,
                                    b_off=ly.bias_offset))

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.gct_unet_destroy(h)
            self._h = None

    def _img(self, t: torch.Tensor, batch: int) -> int:
        return _ptr(t, batch * self.height * self.width, torch.float32)


def unet_set_params(net: UNet, params: torch.Tensor):
    _check(lib.gct_unet_set_params(net.handle, _ptr(params, net.n_params, torch.float32), _stream()))


def unet_get_params(net: UNet, out: torch.Tensor):
    _check(lib.gct_unet_get_params(net.handle, _ptr(out, net.n_params, torch.float32), _stream()))


def unet_get_grads(net: UNet, out: torch.Tensor):
    _check(lib.gct_unet_get_grads(net.handle, _ptr(out, net.n_params, torch.float32), _stream()))


def unet_get_moments(net: UNet, m: torch.Tensor, v: torch.Tensor):
    _check(lib.gct_unet_get_moments(net.handle, _ptr(m, net.n_params, torch.float32),
                                    _ptr(v, net.n_params, torch.float32), _stream()))


def unet_set_moments(net: UNet, m: torch.Tensor | None, v: torch.Tensor | None):
    pm = None if m is None else _ptr(m, net.n_params, torch.float32)
    pv = None if v is None else _ptr(v, net.n_params, torch.float32)
    _check(lib.gct_unet_set_moments(net.handle, pm, pv, _stream()))


def unet_forward(net: UNet, x: torch.Tensor, y: torch.Tensor, in_scale: float = 1.0,
                 out_scale: float = 1.0, batch: int | None = None):
    B = x.numel() // (net.height * net.width) if batch is None else int(batch)
    _check(lib.gct_unet_forward(net.handle, B, net._img(x, B), float(in_scale), float(out_scale),
                                net._img(y, B), _stream()))


def unet_backward(net: UNet, y: torch.Tensor, target: torch.Tensor, loss: torch.Tensor | None = None,
                  batch: int | None = None):
    B = y.numel() // (net.height * net.width) if batch is None else int(batch)
    pl = None if loss is None else _ptr(loss, 1, torch.float32)
    _check(lib.gct_unet_backward(net.handle, B, net._img(y, B), net._img(target, B), pl, _stream()))


def unet_adam_step(net: UNet, lr: float, step: int, beta1: float = 0.9, beta2: float = 0.999,
                   eps: float = 1e-8):
    _check(lib.gct_unet_adam_step(net.handle, float(lr), float(beta1), float(beta2), float(eps),
                                  int(step), _stream()))
