"""FP64 CPU oracle for the pixel-basis (box-spline) parallel-beam CT path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
library (``paper_2005_13471_amd``) never imports it, and it imports nothing
from the product: the two share no code, header, table or constant generator.

The arithmetic lives in ``oracle.c`` (plain C99 + OpenMP, double precision);
this module only compiles it and marshals numpy arrays.  Every function follows
the paper section named in its docstring:

* footprints by geometry: chord length of a ray through the pixel rectangle,
  and the blurred footprint as clipped area / zeta (Sec. 2, Sec. 4);
* Gram filter G[k] = sum over angles of the continuous-y inner product of two
  pixel footprints, by exact Gauss-Legendre quadrature (Sec. 4);
* explicit forward matrix H for tiny N (Sec. 4);
* normal operator by direct spatial summation with G (Sec. 4, last remark);
* correction filter from its definition Q(z) = 1/B(z), sinogram interpolation
  and the exact-adjoint back projection (Sec. 5);
* forward model g_s[theta, m] = (H c)(y_m) (Sec. 2);
* textbook conjugate gradients in FP64 on the normal equations.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_c_int, _c_dbl = ctypes.c_int, ctypes.c_double


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-fopenmp",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        geo = [_c_int, _c_dbl, _c_dbl, _c_int, _dp, _dp]  # N lx1 lx2 n theta detector
        L.or_footprint.argtypes = [_c_dbl] * 4 + [ctypes.c_void_p] + [_c_dbl] * 3
        L.or_footprint.restype = _c_dbl
        L.or_gram.argtypes = geo + [_dp]
        L.or_gram_at.argtypes = geo + [_c_int, _ip, _dp]
        L.or_explicit_H.argtypes = geo + [ctypes.c_void_p]
        L.or_explicit_H.restype = _c_int
        L.or_apply.argtypes = [_c_int, _dp, _dp, _dp]
        L.or_apply_at.argtypes = [_c_int, _dp, _dp, _c_int, _ip, _dp]
        L.or_max_threads.restype = _c_int
        L.or_set_threads.argtypes = [_c_int]
        L.or_bspline.argtypes = [_c_int, _c_dbl]
        L.or_bspline.restype = _c_dbl
        L.or_degree.argtypes = [_c_dbl, _c_dbl]
        L.or_degree.restype = _c_int
        L.or_prefilter_taps.argtypes = [_c_int, _c_int, _dp]
        L.or_prefilter.argtypes = [_c_int, _dp, _dp, _c_int, _c_int, _dp, _dp]
        L.or_ghat.argtypes = [_c_int, _dp, _dp, _c_dbl, _c_int, _c_int, _dp, _c_int, _dp, _dp]
        bpgeo = geo + [_c_dbl, _c_int, _c_int]  # + ly M K
        L.or_backproject.argtypes = bpgeo + [_dp, _dp]
        L.or_backproject_at.argtypes = bpgeo + [_dp, _c_int, _ip, _dp]
        L.or_forward.argtypes = geo + [_c_dbl, _c_int, _dp, _dp]
        L.or_forward_at.argtypes = geo + [_c_dbl, _c_int, _dp, _c_int, _ip, _dp]
        L.or_l2_inner.argtypes = bpgeo + [_dp, _dp]
        L.or_l2_inner.restype = _c_dbl
        L.or_cg.argtypes = [_c_int, _dp, _dp, _dp, _c_int, _c_dbl, _dp]
        L.or_cg.restype = _c_int
        L.or_sd.argtypes = [_c_int, _dp, _dp, _dp, _c_int, _c_dbl, _dp]
        L.or_sd.restype = _c_int
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def detector(zeta=0.0, boxes=None) -> np.ndarray:
    """The detector kernel as the oracle's array {nb, w0, h0, w1, h1, ...}:
    K(t) = sum_i h_i 1{|t| <= w_i / 2} (Sec. 2: boxes of different heights
    and lengths).  boxes: (width, height) pairs; else one box of width zeta
    and height 1/zeta (the paper's blur model), or none for zeta = 0."""
    if boxes:
        if zeta:
            raise ValueError("give either zeta or boxes")
        bx = [(float(w), float(h)) for w, h in boxes]
    elif zeta > 0.0:
        bx = [(float(zeta), 1.0 / float(zeta))]
    else:
        bx = []
    return _f64([len(bx)] + [v for wh in bx for v in wh])


class Geometry:
    """Problem statement of Sec. 2: N, Lambda_x = diag(lx1, lx2), the angle set,
    the detector step ly, the bin count M, the detector kernel (blur width
    zeta, or a list of (width, height) boxes) and the correction-filter
    truncation K (Sec. 5 truncates at 40)."""

    def __init__(self, N, theta, M, ly=1.0, zeta=0.0, lx=(1.0, 1.0), K=40, boxes=None):
        self.N, self.M, self.ly, self.zeta, self.K = int(N), int(M), float(ly), float(zeta), int(K)
        self.boxes = [tuple(b) for b in boxes] if boxes else None
        self.det = detector(self.zeta, self.boxes)
        self.lx1, self.lx2 = float(lx[0]), float(lx[1])
        self.theta = _f64(theta)
        self.n = int(self.theta.size)

    def _geo(self):
        return (self.N, self.lx1, self.lx2, self.n, self.theta, self.det)

    def _bpgeo(self):
        return self._geo() + (self.ly, self.M, self.K)


def footprint(c, s, y, lx=(1.0, 1.0), zeta=0.0, centre=(0.0, 0.0), boxes=None):
    """Footprint of one pixel at direction (c, s) through the detector kernel
    (blur width zeta, or boxes): chord length, or sum over boxes of height
    times clipped area."""
    L = lib()
    det = detector(zeta, boxes)
    dp = det.ctypes.data  # (det stays alive for the loop)
    return np.array([L.or_footprint(c, s, lx[0], lx[1], dp, centre[0], centre[1], float(v))
                     for v in np.atleast_1d(y)])


def gram(g: Geometry) -> np.ndarray:
    """(2N-1) x (2N-1) Gram filter, row index k2 + N - 1, column k1 + N - 1."""
    W = 2 * g.N - 1
    out = np.zeros(W * W)
    lib().or_gram(*g._geo(), out)
    return out.reshape(W, W)


def gram_at(g: Geometry, taps) -> np.ndarray:
    """G at the given taps, an (n, 2) array of (k1, k2)."""
    taps = _i32(np.asarray(taps).reshape(-1, 2))
    out = np.zeros(taps.shape[0])
    lib().or_gram_at(*g._geo(), taps.shape[0], taps.reshape(-1), out)
    return out


def explicit_H(g: Geometry) -> np.ndarray:
    L = lib()
    rows = L.or_explicit_H(*g._geo(), None)
    H = np.zeros((rows, g.N * g.N))
    L.or_explicit_H(*g._geo(), H.ctypes.data_as(ctypes.c_void_p))
    return H


def apply(G: np.ndarray, c: np.ndarray) -> np.ndarray:
    N = c.shape[0]
    y = np.zeros(N * N)
    lib().or_apply(N, _f64(G).reshape(-1), _f64(c).reshape(-1), y)
    return y.reshape(N, N)


def apply_at(G: np.ndarray, c: np.ndarray, idx) -> np.ndarray:
    N = c.shape[0]
    idx = _i32(idx)
    y = np.zeros(idx.size)
    lib().or_apply_at(N, _f64(G).reshape(-1), _f64(c).reshape(-1), idx.size, idx, y)
    return y


def bspline(d: int, x):
    L = lib()
    return np.array([L.or_bspline(int(d), float(v)) for v in np.atleast_1d(x)])


def degree(theta: float, zeta: float) -> int:
    return int(lib().or_degree(float(theta), float(zeta)))


def prefilter_taps(d: int, K: int = 40) -> np.ndarray:
    q = np.zeros(2 * K + 1)
    lib().or_prefilter_taps(int(d), int(K), q)
    return q


def prefilter(g: Geometry, sino: np.ndarray) -> np.ndarray:
    p = np.zeros((g.n, g.M + 2 * g.K))
    lib().or_prefilter(g.n, g.theta, g.det, g.M, g.K, _f64(sino).reshape(-1), p)
    return p


def ghat(g: Geometry, sino: np.ndarray, y) -> np.ndarray:
    y = _f64(np.atleast_1d(y))
    out = np.zeros((g.n, y.size))
    lib().or_ghat(g.n, g.theta, g.det, g.ly, g.M, g.K, _f64(sino).reshape(-1), y.size, y, out)
    return out


def backproject(g: Geometry, sino: np.ndarray) -> np.ndarray:
    b = np.zeros(g.N * g.N)
    lib().or_backproject(*g._bpgeo(), _f64(sino).reshape(-1), b)
    return b.reshape(g.N, g.N)


def backproject_at(g: Geometry, sino: np.ndarray, idx) -> np.ndarray:
    idx = _i32(idx)
    b = np.zeros(idx.size)
    lib().or_backproject_at(*g._bpgeo(), _f64(sino).reshape(-1), idx.size, idx, b)
    return b


def forward(g: Geometry, img: np.ndarray) -> np.ndarray:
    s = np.zeros(g.n * g.M)
    lib().or_forward(*g._geo(), g.ly, g.M, _f64(img).reshape(-1), s)
    return s.reshape(g.n, g.M)


def forward_at(g: Geometry, img: np.ndarray, idx) -> np.ndarray:
    idx = _i32(idx)
    s = np.zeros(idx.size)
    lib().or_forward_at(*g._geo(), g.ly, g.M, _f64(img).reshape(-1), idx.size, idx, s)
    return s


def l2_inner(g: Geometry, img: np.ndarray, sino: np.ndarray) -> float:
    return float(lib().or_l2_inner(*g._bpgeo(), _f64(img).reshape(-1), _f64(sino).reshape(-1)))


def sd(G: np.ndarray, b: np.ndarray, x0=None, maxit=100, rtol=1e-4):
    """Steepest descent, the paper's solver (Sec. 6.2).  Returns (x, iters,
    residual history ||r_k||/||b||)."""
    N = b.shape[0]
    x = np.zeros(N * N) if x0 is None else _f64(x0).reshape(-1).copy()
    hist = np.zeros(maxit + 1)
    it = lib().or_sd(N, _f64(G).reshape(-1), _f64(b).reshape(-1), x, int(maxit), float(rtol), hist)
    return x.reshape(N, N), it, hist[: it + 1]


def cg(G: np.ndarray, b: np.ndarray, x0=None, maxit=100, rtol=1e-4):
    """Returns (x, iters, residual history ||r_k||/||b||)."""
    N = b.shape[0]
    x = np.zeros(N * N) if x0 is None else _f64(x0).reshape(-1).copy()
    hist = np.zeros(maxit + 1)
    it = lib().or_cg(N, _f64(G).reshape(-1), _f64(b).reshape(-1), x, int(maxit), float(rtol), hist)
    return x.reshape(N, N), it, hist[: it + 1]


def max_threads() -> int:
    """Threads the oracle's parallel loops use (OpenMP's current maximum)."""
    return int(lib().or_max_threads())


def set_threads(n: int) -> None:
    """Run the oracle's parallel loops on n threads from now on."""
    lib().or_set_threads(int(n))

