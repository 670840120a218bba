"""CPU oracle for the running-sum Gaussian filter.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the product
library: the fit, the rescaling, the integer weights and the filters are all
re-derived here from Elboher & Werman (arXiv 1107.4958) in plain C
(``rsg_oracle.c``, FP64 / exact int64), loaded through ctypes.

What each function follows:

* :func:`phi` -- Section 4.1, the 1/f^2 autocorrelation model.
* :func:`fit` / :func:`eval_partition` -- Section 4.1 Eq. "mahal" (quadratic
  form error with A_jk = Phi_{j-k}) and Section 4.2 (exhaustive partition
  search at sigma0 = 100/pi over 100 samples).
* :func:`boxes` -- Section 4.2 Eq. "scale1" / "scale2" plus unit-DC
  normalisation, FP32 weights and exact integer uint8 weights.
* :func:`box_filter` -- Section 3 (Eq. "kerdec-1", "S_i", "ciwi", "indep")
  applied separably (Section 3.4), by direct summation of every box.
* :func:`gauss_filter` -- direct convolution with the sampled Gaussian, the
  accuracy reference.

The readings taken where the paper is silent or garbled are listed in the
header of ``rsg_oracle.c``.
"""
from __future__ import annotations

import ctypes
import functools
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rsg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SIGMA0 = 100.0 / math.pi     # Section 4.2
N_HALF = 100                 # samples t = 0..99 on the positive half
PHI_PERIOD = 200             # DFT period: the full support [-pi sigma0, pi sigma0)
PHI_DC = 16.5                # Section 4.1: completed DC value of the spectrum

REPLICATE = 0
ZERO = 1
REFLECT = 2      # half-sample symmetric: ... c b a | a b c d | d c b ...

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile rsg_oracle.c with gcc into liboracle.so (in-tree)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        D = ctypes.c_double
        I = ctypes.c_int
        P = ctypes.c_void_p
        lib.orc_phi.argtypes = [I, D, P]
        lib.orc_phi.restype = None
        lib.orc_eval_partition.argtypes = [I, D, I, I, D, I, P, P, P]
        lib.orc_fit.argtypes = [I, D, I, I, D, I, P, P, P]
        lib.orc_scale.argtypes = [D, D, I, P, P, P, P, P]
        lib.orc_quant_u8.argtypes = [I, P, P, P, P, P]
        lib.orc_box_f64.argtypes = [P, I, I, I, I, P, P, I, P]
        lib.orc_box3_f64.argtypes = [P, I, I, I, I, I, P, P, I, P]
        lib.orc_box_u8.argtypes = [P, I, I, I, I, P, P, ctypes.c_int64, I, P]
        lib.orc_gauss_f64.argtypes = [P, I, I, I, D, I, P]
        lib.orc_box_f64_points.argtypes = [P, I, I, I, I, P, P, I, I, P, P, P, P]
        lib.orc_box_u8_points.argtypes = [P, I, I, I, I, P, P, ctypes.c_int64, I, I, P, P, P, P]
        lib.orc_gauss_f64_points.argtypes = [P, I, I, I, D, I, I, P, P, P, P]
        for f in ("orc_eval_partition", "orc_fit", "orc_scale", "orc_quant_u8", "orc_box_f64",
                  "orc_box_u8", "orc_gauss_f64", "orc_box_f64_points", "orc_box_u8_points", "orc_gauss_f64_points",
                  "orc_box3_f64"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
        return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def phi(N: int = PHI_PERIOD, dc: float = PHI_DC) -> np.ndarray:
    """Phi(l), l = 0..N-1: real inverse DFT of S(u) = 1/min(u, N-u)^2, S(0) = dc."""
    out = np.zeros(N, dtype=np.float64)
    _load().orc_phi(N, dc, _ptr(out))
    return out


def eval_partition(p, *, use_qf=True, nh=N_HALF, sigma0=SIGMA0, N=PHI_PERIOD, dc=PHI_DC):
    """Least-squares constants and error E2 of one partition (inclusive p)."""
    p = np.ascontiguousarray(p, dtype=np.int32)
    k = len(p)
    c = np.zeros(k, dtype=np.float64)
    err = np.zeros(1, dtype=np.float64)
    rc = _load().orc_eval_partition(nh, sigma0, int(use_qf), N, dc, k, _ptr(p), _ptr(c), _ptr(err))
    if rc != 0:
        raise ValueError("invalid partition %r" % (p.tolist(),))
    return c, float(err[0])


def fit(k: int, *, use_qf=True, nh=N_HALF, sigma0=SIGMA0, N=PHI_PERIOD, dc=PHI_DC):
    """Exhaustive search over all partitions (Section 4.2).  Returns (p, c, E2)."""
    return _fit_cached(int(k), bool(use_qf), int(nh), float(sigma0), int(N), float(dc))


@functools.lru_cache(maxsize=None)
def _fit_cached(k, use_qf, nh, sigma0, N, dc):
    p = np.zeros(k, dtype=np.int32)
    c = np.zeros(k, dtype=np.float64)
    err = np.zeros(1, dtype=np.float64)
    rc = _load().orc_fit(nh, sigma0, int(use_qf), N, dc, k, _ptr(p), _ptr(c), _ptr(err))
    if rc != 0:
        raise ValueError("fit failed for k=%d" % k)
    return tuple(int(v) for v in p), tuple(float(v) for v in c), float(err[0])


def scale(sigma: float, p, c, sigma0: float = SIGMA0):
    """Eq. scale1/scale2 + unit-DC normalisation.  Returns (r, w, w32)."""
    p = np.ascontiguousarray(p, dtype=np.int32)
    c = np.ascontiguousarray(c, dtype=np.float64)
    k = len(p)
    r = np.zeros(k, dtype=np.int32)
    w = np.zeros(k, dtype=np.float64)
    w32 = np.zeros(k, dtype=np.float32)
    rc = _load().orc_scale(float(sigma), sigma0, k, _ptr(p), _ptr(c), _ptr(r), _ptr(w), _ptr(w32))
    if rc != 0:
        raise ValueError("scale failed for sigma=%r" % sigma)
    return r, w, w32


def quant_u8(r, w):
    """Integer weights m, DC denominator G and shift s for the exact uint8 path."""
    r = np.ascontiguousarray(r, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    k = len(r)
    m = np.zeros(k, dtype=np.int64)
    G = np.zeros(1, dtype=np.int64)
    s = np.zeros(1, dtype=np.int32)
    rc = _load().orc_quant_u8(k, _ptr(r), _ptr(w), _ptr(m), _ptr(G), _ptr(s))
    if rc != 0:
        raise ValueError("no integer weight scale fits for r=%r" % (r.tolist(),))
    return m, int(G[0]), int(s[0])


def direct_half_samples(sigma: float, k: int) -> int:
    """Half samples M of the direct fit at sigma: the Section 4.2 support
    [-pi sigma, pi sigma) holds ceil(pi sigma) samples t = 0..M-1 on the
    positive half (100 at sigma0), and at least k so that k distinct
    half-widths exist."""
    return max(int(math.ceil(math.pi * sigma - 1e-9)), int(k))


def boxes_direct(sigma: float, k: int) -> dict:
    """Direct fit at sigma (a reading: the paper fits once at sigma0 and
    rescales, Section 4.2): the same exhaustive search of the quadratic form
    (Section 4.1, Eq. mahal) run on the Gaussian of s.d. sigma itself, over M
    half samples with Phi on period 2M.  The half-widths are the partition
    (r = p), the slice weights w_i = c_i - c_{i+1} are normalised to unit DC
    gain, and the FP32 and uint8 forms follow as for the rescaled fit."""
    M = direct_half_samples(sigma, k)
    p, c, err = fit(k, nh=M, sigma0=float(sigma), N=2 * M)
    p = np.asarray(p, dtype=np.int32)
    c = np.asarray(c, dtype=np.float64)
    slices = c - np.append(c[1:], 0.0)
    r = p.copy()
    w = slices / float(np.sum(slices * (2.0 * r + 1.0)))
    w32 = w.astype(np.float32)
    try:
        m, G, s = quant_u8(r, w)
    except ValueError:
        m, G, s = None, None, None
    return dict(sigma=float(sigma), k=int(k), p=p, c=c, fit_err=err, r=r, w=w, w32=w32,
                m=m, G=G, s=s, M=M)


def boxes(sigma: float, k: int, *, use_qf=True) -> dict:
    """Everything the filter needs for one (sigma, k): the oracle's own fit."""
    p, c, err = fit(k, use_qf=use_qf)
    r, w, w32 = scale(sigma, p, c)
    try:
        m, G, s = quant_u8(r, w)
    except ValueError:
        m, G, s = None, None, None
    return dict(sigma=float(sigma), k=int(k), p=p, c=c, fit_err=err, r=r, w=w, w32=w32,
                m=m, G=G, s=s)


def _check_img(img: np.ndarray):
    if img.ndim == 2:
        return img.shape[0], img.shape[1], 1
    if img.ndim == 3:
        return img.shape
    raise ValueError("image must be HxW or HxWxC")


def box_filter(img: np.ndarray, r, w, boundary: int = REPLICATE) -> np.ndarray:
    """FP64 direct box sums with real weights w (pass w32 promoted for FP32 parity)."""
    H, W, C = _check_img(img)
    src = np.ascontiguousarray(img, dtype=np.float64)
    dst = np.empty_like(src)
    r = np.ascontiguousarray(r, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    rc = _load().orc_box_f64(_ptr(src), H, W, C, len(r), _ptr(r), _ptr(w), boundary, _ptr(dst))
    if rc != 0:
        raise ValueError("orc_box_f64 failed")
    return dst


def box_filter_3d(vol: np.ndarray, r, w, boundary: int = REPLICATE) -> np.ndarray:
    """FP64 direct box sums of a D x H x W (x C) volume along all three axes."""
    if vol.ndim not in (3, 4):
        raise ValueError("volume must be DxHxW or DxHxWxC")
    D, H, W = vol.shape[:3]
    C = vol.shape[3] if vol.ndim == 4 else 1
    src = np.ascontiguousarray(vol, dtype=np.float64)
    dst = np.empty_like(src)
    r = np.ascontiguousarray(r, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    rc = _load().orc_box3_f64(_ptr(src), D, H, W, C, len(r), _ptr(r), _ptr(w), boundary, _ptr(dst))
    if rc != 0:
        raise ValueError("orc_box3_f64 failed")
    return dst


def box_filter_u8(img: np.ndarray, r, m, G: int, boundary: int = REPLICATE) -> np.ndarray:
    """Exact integer box filter for uint8 images, rounded half up once."""
    H, W, C = _check_img(img)
    src = np.ascontiguousarray(img, dtype=np.uint8)
    dst = np.empty_like(src)
    r = np.ascontiguousarray(r, dtype=np.int32)
    m = np.ascontiguousarray(m, dtype=np.int64)
    rc = _load().orc_box_u8(_ptr(src), H, W, C, len(r), _ptr(r), _ptr(m), int(G), boundary, _ptr(dst))
    if rc != 0:
        raise ValueError("orc_box_u8 failed")
    return dst


def gauss_filter(img: np.ndarray, sigma: float, boundary: int = REPLICATE) -> np.ndarray:
    """Sampled-Gaussian direct convolution (|t| <= ceil(6 sigma)), FP64."""
    H, W, C = _check_img(img)
    src = np.ascontiguousarray(img, dtype=np.float64)
    dst = np.empty_like(src)
    rc = _load().orc_gauss_f64(_ptr(src), H, W, C, float(sigma), boundary, _ptr(dst))
    if rc != 0:
        raise ValueError("orc_gauss_f64 failed")
    return dst


def gauss_filter_points(img: np.ndarray, sigma: float, ys, xs, cs=None, boundary: int = REPLICATE):
    """orc_gauss_f64 evaluated only at the listed output positions."""
    H, W, C = _check_img(img)
    src = np.ascontiguousarray(img, dtype=np.float64)
    ys = np.ascontiguousarray(ys, dtype=np.int64)
    xs = np.ascontiguousarray(xs, dtype=np.int64)
    cs = np.zeros_like(ys) if cs is None else np.ascontiguousarray(cs, dtype=np.int64)
    out = np.zeros(len(ys), dtype=np.float64)
    rc = _load().orc_gauss_f64_points(_ptr(src), H, W, C, float(sigma), boundary, len(ys), _ptr(ys), _ptr(xs),
                                      _ptr(cs), _ptr(out))
    if rc != 0:
        raise ValueError("orc_gauss_f64_points failed")
    return out


def box_filter_points(img: np.ndarray, r, w, ys, xs, cs=None, boundary: int = REPLICATE):
    """orc_box_f64 evaluated only at the listed output positions."""
    H, W, C = _check_img(img)
    src = np.ascontiguousarray(img, dtype=np.float64)
    ys = np.ascontiguousarray(ys, dtype=np.int64)
    xs = np.ascontiguousarray(xs, dtype=np.int64)
    cs = np.zeros_like(ys) if cs is None else np.ascontiguousarray(cs, dtype=np.int64)
    out = np.zeros(len(ys), dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    _load().orc_box_f64_points(_ptr(src), H, W, C, len(r), _ptr(r), _ptr(w), boundary, len(ys),
                               _ptr(ys), _ptr(xs), _ptr(cs), _ptr(out))
    return out


def box_filter_u8_points(img: np.ndarray, r, m, G, ys, xs, cs=None, boundary: int = REPLICATE):
    """orc_box_u8 evaluated only at the listed output positions."""
    H, W, C = _check_img(img)
    src = np.ascontiguousarray(img, dtype=np.uint8)
    ys = np.ascontiguousarray(ys, dtype=np.int64)
    xs = np.ascontiguousarray(xs, dtype=np.int64)
    cs = np.zeros_like(ys) if cs is None else np.ascontiguousarray(cs, dtype=np.int64)
    out = np.zeros(len(ys), dtype=np.uint8)
    r = np.ascontiguousarray(r, dtype=np.int32)
    m = np.ascontiguousarray(m, dtype=np.int64)
    _load().orc_box_u8_points(_ptr(src), H, W, C, len(r), _ptr(r), _ptr(m), int(G), boundary,
                              len(ys), _ptr(ys), _ptr(xs), _ptr(cs), _ptr(out))
    return out


def kernel_1d(r, w) -> np.ndarray:
    """The 1D step kernel h(t) = sum_{j: |t| <= r_j} w_j on t = -r_max..r_max (Eq. ciwi)."""
    r = np.asarray(r)
    R = int(r.max())
    t = np.arange(-R, R + 1)
    h = np.zeros(2 * R + 1, dtype=np.float64)
    for rj, wj in zip(r, w):
        h[np.abs(t) <= rj] += wj
    return h


def nrms(y: np.ndarray, ref: np.ndarray) -> float:
    """Normalised RMS error ||y - ref||_2 / ||ref||_2."""
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = float(np.sqrt(np.sum(ref * ref)))
    return float(np.sqrt(np.sum((y - ref) ** 2))) / den if den > 0 else float("nan")


def psnr(y: np.ndarray, ref: np.ndarray, peak: float = 255.0) -> float:
    """Section 5: PSNR = -10 log10(MSE) with values scaled to [0, 1]."""
    d = (np.asarray(y, dtype=np.float64) - np.asarray(ref, dtype=np.float64)) / peak
    mse = float(np.mean(d * d))
    return float("inf") if mse == 0 else -10.0 * math.log10(mse)
