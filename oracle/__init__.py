"""CPU oracle for the four-directional 5x5 Sobel operator (test infrastructure).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library and its Python binding
never import this package, and this package imports nothing from them.

The arithmetic lives in ``sobel_oracle.c`` (plain nested loops, Eq. (sobel5_1)
and Eq. (sobel5_2) of Chang et al., Sec. 3.1); this module builds it with gcc
and wraps it with ctypes, returning numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "sobel_oracle.c"
_LIB = _HERE / "liboracle.so"

REPLICATE = 0
VALID = 1
ZERO = 2           # pixels outside the image read 0 (uint8 path)
REFLECT101 = 3     # mirror about the edge pixel without repeating it (uint8 path)

_lib = None


def build(force: bool = False) -> Path:
    """Compile the oracle with gcc (-O2, OpenMP, no intrinsics)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-o", str(tmp), str(_SRC), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not _LIB.exists():
            build()
        lib = ctypes.CDLL(str(_LIB))
        P = ctypes.c_void_p
        I = ctypes.c_int
        L = ctypes.c_long
        lib.oracle_u8.argtypes = [P, I, I, L, I, P, L, P, P, I]
        lib.oracle_u8.restype = I
        lib.oracle_u8_points.argtypes = [P, I, I, L, I, P, P, L, P, P, P]
        lib.oracle_u8_points.restype = I
        lib.oracle_f64_fwd.argtypes = [P, I, I, I, I, P, P, P, I]
        lib.oracle_f64_fwd.restype = I
        lib.oracle_f64_bwd.argtypes = [P, P, I, I, I, I, P, P, I]
        lib.oracle_f64_bwd.restype = I
        lib.oracle_f64_bwd_scale.argtypes = [P, P, I, I, I, I, P, P, I]
        lib.oracle_f64_bwd_scale.restype = I
        lib.oracle_f64_fwd_scale.argtypes = [P, I, I, I, I, P, P, I]
        lib.oracle_f64_fwd_scale.restype = I
        lib.oracle_weights.argtypes = [P]
        lib.oracle_weights.restype = None
        lib.oracle_u8_2dir.argtypes = [P, I, I, L, I, I, P, L, P, I]
        lib.oracle_u8_2dir.restype = I
        lib.oracle_round_sqrt.argtypes = [ctypes.c_int64]
        lib.oracle_round_sqrt.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _weights_arg(weights):
    if weights is None:
        return None
    w = np.ascontiguousarray(weights, dtype=np.int32).reshape(4, 5, 5)
    return w


def out_shape(h: int, w: int, border: int):
    return (h - 4, w - 4) if border == VALID else (h, w)


def weights() -> np.ndarray:
    """The literal Eq. (sobel5_1) table, shape (4, 5, 5), plane order Gx, Gd, Gy, Gdt."""
    out = np.zeros((4, 5, 5), dtype=np.int32)
    _load().oracle_weights(_ptr(out))
    return out


def round_sqrt(s: int) -> int:
    return int(_load().oracle_round_sqrt(int(s)))


def sobel_u8(img: np.ndarray, border: int = REPLICATE, *, weights=None,
             want_mag: bool = True, want_dir: bool = True, nthreads: int = 0):
    """uint8 image (H, W) or (H, pitch) view -> (mag uint8 (Ho, Wo), dir int32 (4, Ho, Wo)).

    ``img`` may be a 2-D view whose rows are strided (pitch = img.strides[0]).
    """
    if img.dtype != np.uint8 or img.ndim != 2 or img.strides[1] != 1:
        raise ValueError("img must be a 2-D uint8 array with unit column stride")
    h, w = img.shape
    pitch = img.strides[0]
    ho, wo = out_shape(h, w, border)
    mag = np.empty((ho, wo), np.uint8) if want_mag else None
    d = np.empty((4, ho, wo), np.int32) if want_dir else None
    wt = _weights_arg(weights)
    base = img.ctypes.data_as(ctypes.c_void_p)
    rc = _load().oracle_u8(base, w, h, pitch, border, _ptr(mag), wo, _ptr(d),
                           _ptr(wt), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_u8 rejected its arguments (rc=%d)" % rc)
    return mag, d


def sobel_u8_2dir(img: np.ndarray, size: int, border: int = REPLICATE, *,
                  want_mag: bool = True, want_dir: bool = True, nthreads: int = 0):
    """Two-directional operator: (mag uint8 (Ho, Wo), dir int32 (2, Ho, Wo): Gx, Gy).

    size 3: Eq. (sobel3_1) with Eq. (sobel3_2); VALID shrinks by 2.
    size 5: the 0 and 90 deg filters of Eq. (sobel5_1); VALID shrinks by 4.
    """
    if img.dtype != np.uint8 or img.ndim != 2 or img.strides[1] != 1:
        raise ValueError("img must be a 2-D uint8 array with unit column stride")
    h, w = img.shape
    r = size // 2
    ho, wo = (h - 2 * r, w - 2 * r) if border == VALID else (h, w)
    mag = np.empty((max(ho, 0), max(wo, 0)), np.uint8) if want_mag else None
    d = np.empty((2, max(ho, 0), max(wo, 0)), np.int32) if want_dir else None
    rc = _load().oracle_u8_2dir(img.ctypes.data_as(ctypes.c_void_p), w, h, img.strides[0], border,
                                int(size), _ptr(mag), max(wo, 1), _ptr(d), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_u8_2dir rejected its arguments (rc=%d)" % rc)
    return mag, d


def sobel_u8_points(img: np.ndarray, ys, xs, border: int = REPLICATE, *, weights=None):
    """Responses at listed output pixels: (mag uint8 (n,), dir int32 (n, 4))."""
    if img.dtype != np.uint8 or img.ndim != 2 or img.strides[1] != 1:
        raise ValueError("img must be a 2-D uint8 array with unit column stride")
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    n = ys.size
    h, w = img.shape
    mag = np.empty(n, np.uint8)
    d = np.empty((n, 4), np.int32)
    wt = _weights_arg(weights)
    rc = _load().oracle_u8_points(img.ctypes.data_as(ctypes.c_void_p), w, h, img.strides[0],
                                  border, _ptr(ys), _ptr(xs), n, _ptr(mag), _ptr(d), _ptr(wt))
    if rc != 0:
        raise ValueError("oracle_u8_points rejected its arguments (rc=%d)" % rc)
    return mag, d


def sobel_f64_fwd(x: np.ndarray, border: int = REPLICATE, *, weights=None,
                  want_dir: bool = False, nthreads: int = 0):
    """x (B, H, W) real -> (M float64 (B, Ho, Wo), dir float64 (B, 4, Ho, Wo) or None)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 2:
        x = x[None]
    b, h, w = x.shape
    ho, wo = out_shape(h, w, border)
    mag = np.empty((b, ho, wo), np.float64)
    d = np.empty((b, 4, ho, wo), np.float64) if want_dir else None
    wt = _weights_arg(weights)
    rc = _load().oracle_f64_fwd(_ptr(x), b, h, w, border, _ptr(mag), _ptr(d), _ptr(wt),
                                int(nthreads))
    if rc != 0:
        raise ValueError("oracle_f64_fwd rejected its arguments (rc=%d)" % rc)
    return mag, d


def sobel_f64_bwd(x: np.ndarray, g: np.ndarray, border: int = REPLICATE, *, weights=None,
                  nthreads: int = 0) -> np.ndarray:
    """Adjoint of the magnitude map: dL/dx (B, H, W) for dL/dM = g (B, Ho, Wo)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    if x.ndim == 2:
        x = x[None]
        g = g[None]
    b, h, w = x.shape
    ho, wo = out_shape(h, w, border)
    if g.shape != (b, ho, wo):
        raise ValueError("g must have shape %s" % ((b, ho, wo),))
    dx = np.empty((b, h, w), np.float64)
    wt = _weights_arg(weights)
    rc = _load().oracle_f64_bwd(_ptr(x), _ptr(g), b, h, w, border, _ptr(dx), _ptr(wt),
                                int(nthreads))
    if rc != 0:
        raise ValueError("oracle_f64_bwd rejected its arguments (rc=%d)" % rc)
    return dx


def sobel_f64_bwd_scale(x: np.ndarray, g: np.ndarray, border: int = REPLICATE, *, weights=None,
                        nthreads: int = 0) -> np.ndarray:
    """Per-input-pixel sum of |term| of the adjoint's sum (tolerance scale A(p))."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    if x.ndim == 2:
        x = x[None]
        g = g[None]
    b, h, w = x.shape
    a = np.empty((b, h, w), np.float64)
    wt = _weights_arg(weights)
    rc = _load().oracle_f64_bwd_scale(_ptr(x), _ptr(g), b, h, w, border, _ptr(a), _ptr(wt),
                                      int(nthreads))
    if rc != 0:
        raise ValueError("oracle_f64_bwd_scale rejected its arguments (rc=%d)" % rc)
    return a


def sobel_f64_fwd_scale(x: np.ndarray, border: int = REPLICATE, *, weights=None,
                        nthreads: int = 0) -> np.ndarray:
    """Per-output-pixel max_k sum_t |K_k[t] x_t| (tolerance scale of the forward)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.ndim == 2:
        x = x[None]
    b, h, w = x.shape
    ho, wo = out_shape(h, w, border)
    s = np.empty((b, ho, wo), np.float64)
    wt = _weights_arg(weights)
    rc = _load().oracle_f64_fwd_scale(_ptr(x), b, h, w, border, _ptr(s), _ptr(wt), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_f64_fwd_scale rejected its arguments (rc=%d)" % rc)
    return s
