"""ctypes binding of libsobel4x5.so (the C ABI of include/sobel4x5.h).

Argument marshalling only: every function checks tensor devices/dtypes,
converts them to raw device pointers and byte pitches, and calls the library
on torch's current HIP stream.  All arithmetic happens in the HIP kernels.
The library is required: importing this module on a machine where it cannot
be loaded raises, and there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from pathlib import Path

import numpy as np

import torch

_PKG = Path(__file__).resolve().parent
# SOBEL4X5_LIBRARY may name another build of the same library (tuning runs)
LIB_PATH = Path(os.environ.get("SOBEL4X5_LIBRARY") or (_PKG / "libsobel4x5.so"))

BORDER_REPLICATE = 0
BORDER_VALID = 1
BORDER_ZERO = 2          # pixels outside the image read 0 (uint8 path)
BORDER_REFLECT101 = 3    # mirror about the edge pixel, not repeating it (uint8 path)
DIR_NONE = 0
DIR_S16 = 1
DIR_S32 = 2
OP_4DIR_5X5 = 0     # Eq. (sobel5_1) + Eq. (sobel5_2)
OP_2DIR_5X5 = 1     # the 0 and 90 deg filters of Eq. (sobel5_1)
OP_2DIR_3X3 = 2     # Eq. (sobel3_1) + Eq. (sobel3_2)
PLAN_AUTOTUNE = 1
PLAN_NO_GRAPH = 2

OK, EINVAL, EUNSUPPORTED, EHIP, ENOMEM = 0, 1, 2, 3, 4


class SobelError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__("%s failed (%d): %s" % (where, code, detail))
        self.code = code


class Outputs(ctypes.Structure):
    _fields_ = [("mag", ctypes.c_void_p), ("mag_pitch", ctypes.c_int64),
                ("dir", ctypes.c_void_p * 4), ("dir_pitch", ctypes.c_int64),
                ("dir_type", ctypes.c_int32)]


class Image(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("mag", ctypes.c_void_p),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("src_pitch", ctypes.c_int64), ("mag_pitch", ctypes.c_int64)]


def _load() -> ctypes.CDLL:
    if not LIB_PATH.exists():
        raise ImportError("libsobel4x5.so is not built (run __graft_entry__.build() or "
                          "python -m paper_2305_00515_amd.build)")
    lib = ctypes.CDLL(str(LIB_PATH))
    P, I32, I64, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sig = {
        "sobel4x5_u8": [P, I32, I32, I64, I32, ctypes.POINTER(Outputs), P],
        "sobel4x5_validate_u8": [P, I32, I32, I64, I32, ctypes.POINTER(Outputs)],
        "sobel4x5_u8_op": [P, I32, I32, I64, I32, I32, ctypes.POINTER(Outputs), P],
        "sobel4x5_validate_u8_op": [P, I32, I32, I64, I32, I32, ctypes.POINTER(Outputs)],
        "sobel4x5_plan_create": [ctypes.POINTER(Image), I32, I32, U32, ctypes.POINTER(P)],
        "sobel4x5_plan_launch": [P, P],
        "sobel4x5_plan_info": [P] + [ctypes.POINTER(I32)] * 4,
        "sobel4x5_debug_plan_claims": [P, P, I64, ctypes.POINTER(I64), P],
        "sobel4x5_plan_destroy": [P],
        "sobel4x5_batched": [ctypes.POINTER(Image), I32, I32, P],
        "sobel4x5_batched_noalloc": [ctypes.POINTER(Image), I32, I32, P],
        "sobel4x5_validate_batch": [ctypes.POINTER(Image), I32, I32],
        "sobel4x5_plan_create_ex": [ctypes.POINTER(Image), ctypes.POINTER(Outputs), I32, I32, U32, ctypes.POINTER(P)],
        "sobel4x5_batched_ex": [ctypes.POINTER(Image), ctypes.POINTER(Outputs), I32, I32, P],
        "sobel4x5_validate_batch_ex": [ctypes.POINTER(Image), ctypes.POINTER(Outputs), I32, I32],
        "sobel4x5_f32_fwd": [P, I32, I32, I32, I64, I64, I32, P, I64, I64, P],
        "sobel4x5_f32_bwd": [P, I64, I64, P, I64, I64, I32, I32, I32, I32, P, I64, I64, P],
        "sobel4x5_validate_f32": [P, I32, I32, I32, I64, I64, I32, P, I64, I64],
        "sobel4x5_u8_weighted": [P, I32, I32, I64, I32, P, ctypes.POINTER(Outputs), P],
        "sobel4x5_validate_weights": [P, I32],
        "sobel4x5_family_weights": [I32] * 6 + [P],
        "sobel4x5_pipe_create": [I32, I32, I32, ctypes.POINTER(P)],
        "sobel4x5_pipe_run": [P, ctypes.POINTER(Image), I32, I32],
        "sobel4x5_pipe_destroy": [P],
        "sobel4x5_debug_round_mag": [P, P, I64, P],
        "sobel4x5_debug_round_mag_ex": [P, P, I64, I32, P],
        "sobel4x5_debug_round_quad": [P, P, I64, P],
        "sobel4x5_debug_copy": [P, P, I64, P],
        "sobel4x5_debug_inject_failure": [I32],
        "sobel4x5_status_string": [ctypes.c_int],
        "sobel4x5_last_error": [],
        "sobel4x5_version": [],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.sobel4x5_status_string.restype = ctypes.c_char_p
    lib.sobel4x5_last_error.restype = ctypes.c_char_p
    return lib


lib = _load()


def _check(rc: int, where: str) -> None:
    if rc != OK:
        raise SobelError(rc, where, lib.sobel4x5_last_error().decode())


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _need_cuda(t: torch.Tensor, dtype, name: str) -> None:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a GPU tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))


def _rows(t: torch.Tensor, name: str):
    """(height, width, pitch bytes) of a 2-D tensor with unit column stride."""
    if t.dim() != 2 or (t.size(1) > 1 and t.stride(1) != 1):
        raise ValueError("%s must be 2-D with unit column stride" % name)
    return t.size(0), t.size(1), t.stride(0) * t.element_size()


def out_shape(h: int, w: int, border: int, op: int = OP_4DIR_5X5):
    r = 1 if op == OP_2DIR_3X3 else 2
    return (h - 2 * r, w - 2 * r) if border == BORDER_VALID else (h, w)


def _u8_outputs(src, border, mag, want_mag, dir_type, dirs, op=OP_4DIR_5X5):
    """Outputs struct (and the tensors) for a uint8 call on src.  The
    two-directional operators take two planes (Gx, Gy) in slots 0 and 2."""
    _need_cuda(src, torch.uint8, "src")
    h, w, pitch = _rows(src, "src")
    ho, wo = out_shape(h, w, border, op)
    slots = (0, 1, 2, 3) if op == OP_4DIR_5X5 else (0, 2)
    if want_mag and mag is None:
        mag = torch.empty((max(ho, 0), max(wo, 0)), dtype=torch.uint8, device=src.device)
    out = Outputs()
    if want_mag or mag is not None:
        _need_cuda(mag, torch.uint8, "mag")
        if tuple(mag.shape) != (ho, wo):
            raise ValueError("mag must have shape %s, got %s" % ((ho, wo), tuple(mag.shape)))
        out.mag = mag.data_ptr()
        out.mag_pitch = _rows(mag, "mag")[2]
    if dir_type != DIR_NONE:
        dt = torch.int16 if dir_type == DIR_S16 else torch.int32
        if dirs is None:
            dirs = [torch.empty((ho, wo), dtype=dt, device=src.device) for _ in slots]
        pitches = set()
        if len(dirs) != len(slots):
            raise ValueError("need %d directional planes" % len(slots))
        for k, d in zip(slots, dirs):
            _need_cuda(d, dt, "dirs[%d]" % k)
            if tuple(d.shape) != (ho, wo):
                raise ValueError("dirs[%d] must have shape %s" % (k, (ho, wo)))
            out.dir[k] = d.data_ptr()
            pitches.add(_rows(d, "dirs[%d]" % k)[2])
        if len(pitches) != 1:
            raise ValueError("all directional planes must share one row pitch")
        out.dir_pitch = pitches.pop()
    out.dir_type = dir_type
    res = ((mag if (want_mag or out.mag) else None), (dirs if dir_type != DIR_NONE else None))
    return out, (h, w, pitch), res


def sobel4x5_u8(src: torch.Tensor, border: int = BORDER_REPLICATE, *, mag: torch.Tensor | None = None,
                want_mag: bool = True, dir_type: int = DIR_NONE, dirs: list | None = None):
    """uint8 image (H, W) on the GPU -> (mag uint8 (Ho, Wo) or None, [4 planes] or None).

    Planes are 0 deg Gx, 45 deg Gd, 90 deg Gy, 135 deg Gdt as int16 (DIR_S16)
    or int32 (DIR_S32).  Output tensors may be passed in (any row pitch).
    """
    out, (h, w, pitch), res = _u8_outputs(src, border, mag, want_mag, dir_type, dirs)
    _check(lib.sobel4x5_u8(src.data_ptr(), w, h, pitch, border, ctypes.byref(out), _stream(src)),
           "sobel4x5_u8")
    return res


def sobel4x5_u8_op(src: torch.Tensor, op: int, border: int = BORDER_REPLICATE, *,
                   mag: torch.Tensor | None = None, want_mag: bool = True, dir_type: int = DIR_NONE,
                   dirs: list | None = None):
    """sobel4x5_u8 for operator `op` (OP_*): the two-directional operators
    return two planes [Gx, Gy]; the 3x3 pair's VALID output is (H-2, W-2)."""
    out, (h, w, pitch), res = _u8_outputs(src, border, mag, want_mag, dir_type, dirs, op)
    _check(lib.sobel4x5_u8_op(src.data_ptr(), w, h, pitch, op, border, ctypes.byref(out), _stream(src)),
           "sobel4x5_u8_op")
    return res


def _weights_buf(weights):
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.int64).reshape(4, 5, 5))
    if np.abs(w).max() >= 2 ** 31:
        raise ValueError("weights must fit int32")
    return np.ascontiguousarray(w.astype(np.int32))


def sobel4x5_u8_weighted(src: torch.Tensor, weights, border: int = BORDER_REPLICATE, *,
                         mag: torch.Tensor | None = None, want_mag: bool = True, dir_type: int = DIR_NONE,
                         dirs: list | None = None):
    """sobel4x5_u8 with run-time integer kernels (4, 5, 5), plane order as the
    default operator; each kernel antisymmetric under a half turn."""
    wb = _weights_buf(weights)
    out, (h, w, pitch), res = _u8_outputs(src, border, mag, want_mag, dir_type, dirs)
    _check(lib.sobel4x5_u8_weighted(src.data_ptr(), w, h, pitch, border, wb.ctypes.data, ctypes.byref(out),
                                    _stream(src)), "sobel4x5_u8_weighted")
    return res


def validate_weights(weights, dir_type: int = DIR_NONE) -> None:
    """Raises SobelError unless sobel4x5_u8_weighted accepts these weights."""
    wb = _weights_buf(weights)
    _check(lib.sobel4x5_validate_weights(wb.ctypes.data, dir_type), "sobel4x5_validate_weights")


def family_weights(a: int, ab: int, an: int, am: int, anb: int, amb: int) -> np.ndarray:
    """The four kernels (4, 5, 5) of the family K(a, b, n, m), from its six
    integer weights a, a*b, a*n, a*m, a*n*b, a*m*b."""
    out = np.zeros((4, 5, 5), dtype=np.int32)
    _check(lib.sobel4x5_family_weights(a, ab, an, am, anb, amb, out.ctypes.data), "sobel4x5_family_weights")
    return out


def family_products(a, b, n, m):
    """(a, a*b, a*n, a*m, a*n*b, a*m*b) for parameters given as ints,
    fractions or decimal strings; ValueError unless all six are integers."""
    from fractions import Fraction
    A, B, N, M = (Fraction(str(v)) if not isinstance(v, Fraction) else v for v in (a, b, n, m))
    prods = (A, A * B, A * N, A * M, A * N * B, A * M * B)
    if any(p.denominator != 1 for p in prods):
        raise ValueError("the family weights must all be integers, got %s" % (tuple(str(p) for p in prods),))
    return tuple(int(p) for p in prods)


def _host_rows(a, name):
    """(height, width, pitch bytes, address) of a 2-D uint8 host array
    (numpy or CPU tensor, unit column stride)."""
    if isinstance(a, torch.Tensor):
        if a.is_cuda or a.dtype != torch.uint8 or a.dim() != 2 or (a.size(1) > 1 and a.stride(1) != 1):
            raise ValueError("%s must be a 2-D uint8 CPU tensor with unit column stride" % name)
        return a.size(0), a.size(1), a.stride(0), a.data_ptr()
    a = np.asarray(a)
    if a.dtype != np.uint8 or a.ndim != 2 or (a.shape[1] > 1 and a.strides[1] != 1):
        raise ValueError("%s must be a 2-D uint8 array with unit column stride" % name)
    return a.shape[0], a.shape[1], a.strides[0], a.ctypes.data


class Pipe:
    """Host-memory images -> host-memory magnitudes, with the copies to and
    from the device overlapped with the kernels across `depth` slots."""

    def __init__(self, max_width: int, max_height: int, depth: int = 3):
        self._h = ctypes.c_void_p()
        _check(lib.sobel4x5_pipe_create(max_width, max_height, depth, ctypes.byref(self._h)), "sobel4x5_pipe_create")

    def run(self, srcs, mags=None, border: int = BORDER_REPLICATE):
        """srcs: uint8 host images (numpy arrays or CPU tensors, pinned or
        not); mags: matching outputs or None (numpy arrays are allocated)."""
        n = len(srcs)
        if mags is None:
            mags = []
            for m in srcs:
                h, w = (m.shape[0], m.shape[1])
                ho, wo = out_shape(h, w, border)
                mags.append(np.empty((max(ho, 0), max(wo, 0)), np.uint8))
        if len(mags) != n:
            raise ValueError("srcs and mags differ in length")
        arr = (Image * max(n, 1))()
        for i, (sa, ma) in enumerate(zip(srcs, mags)):
            h, w, sp, sptr = _host_rows(sa, "srcs[%d]" % i)
            ho, wo = out_shape(h, w, border)
            mh, mw, mp, mptr = _host_rows(ma, "mags[%d]" % i)
            if (mh, mw) != (ho, wo):
                raise ValueError("mags[%d] must have shape %s" % (i, (ho, wo)))
            arr[i] = Image(sptr, mptr, w, h, sp, mp)
        _check(lib.sobel4x5_pipe_run(self._h, arr, n, border), "sobel4x5_pipe_run")
        return mags

    def close(self):
        if self._h:
            lib.sobel4x5_pipe_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _images(srcs, mags, border):
    if len(srcs) != len(mags) or not srcs:
        raise ValueError("need equally many (>= 1) sources and outputs")
    arr = (Image * len(srcs))()
    for i, (s, m) in enumerate(zip(srcs, mags)):
        _need_cuda(s, torch.uint8, "srcs[%d]" % i)
        _need_cuda(m, torch.uint8, "mags[%d]" % i)
        h, w, p = _rows(s, "srcs[%d]" % i)
        if tuple(m.shape) != out_shape(h, w, border):
            raise ValueError("mags[%d] must have shape %s" % (i, out_shape(h, w, border)))
        arr[i].src = s.data_ptr()
        arr[i].mag = m.data_ptr()
        arr[i].width = w
        arr[i].height = h
        arr[i].src_pitch = p
        arr[i].mag_pitch = _rows(m, "mags[%d]" % i)[2]
    return arr


def _images_ex(srcs, mags, border, want_mag, dir_type, dirs):
    """Descriptor and per-image outputs arrays for a batch with directional
    planes; returns (imgs, outs, [(mag or None, planes or None)])."""
    n = len(srcs)
    if not n:
        raise ValueError("need at least one source")
    mags = list(mags) if mags is not None else [None] * n
    dirs = list(dirs) if dirs is not None else [None] * n
    if len(mags) != n or len(dirs) != n:
        raise ValueError("srcs, mags and dirs differ in length")
    imgs = (Image * n)()
    outs = (Outputs * n)()
    res = []
    for i, s in enumerate(srcs):
        o, (h, w, p), r = _u8_outputs(s, border, mags[i], want_mag, dir_type, dirs[i])
        outs[i] = o
        imgs[i].src = s.data_ptr()
        imgs[i].width = w
        imgs[i].height = h
        imgs[i].src_pitch = p
        res.append(r)
    return imgs, outs, res


class Plan:
    """A reusable batched plan over fixed (src, mag) tensor pairs.

    The tensors are referenced, not copied: keep them alive (the plan holds
    references) and do not reallocate them while the plan exists.
    """

    def __init__(self, srcs, mags, border: int = BORDER_REPLICATE, autotune: bool = False,
                 graph: bool = True, dir_type: int = DIR_NONE, dirs=None):
        """With dir_type, `dirs` holds each image's four planes (mags entries
        may then be None for no magnitude)."""
        self.device = list(srcs)[0].device
        flags = (PLAN_AUTOTUNE if autotune else 0) | (0 if graph else PLAN_NO_GRAPH)
        h = ctypes.c_void_p()
        if dir_type == DIR_NONE:
            self._keep = (list(srcs), list(mags))
            self._arr = _images(self._keep[0], self._keep[1], border)
            _check(lib.sobel4x5_plan_create(self._arr, len(self._arr), border, flags, ctypes.byref(h)),
                   "sobel4x5_plan_create")
        else:
            want = [m is not None for m in mags]
            if len(set(want)) != 1:
                raise ValueError("give a magnitude for every image or for none")
            self._arr, self._outs, res = _images_ex(list(srcs), mags, border, want[0], dir_type, dirs)
            self._keep = (list(srcs), res)
            _check(lib.sobel4x5_plan_create_ex(self._arr, self._outs, len(self._arr), border, flags,
                                               ctypes.byref(h)), "sobel4x5_plan_create_ex")
        self._h = h

    def launch(self) -> None:
        _check(lib.sobel4x5_plan_launch(self._h, _stream(self._keep[0][0])), "sobel4x5_plan_launch")

    def info(self) -> dict:
        vals = [ctypes.c_int32() for _ in range(4)]
        _check(lib.sobel4x5_plan_info(self._h, *[ctypes.byref(v) for v in vals]), "sobel4x5_plan_info")
        return dict(zip(("px_per_lane", "rows_per_tile", "waves_per_group", "grid"),
                        (v.value for v in vals)))

    def claims(self):
        """One launch that also counts how many waves took each tile of the
        work table (sobel4x5_debug_plan_claims): an int32 tensor of one count
        per tile, all 1 when no tile was skipped or taken twice."""
        n = ctypes.c_int64()
        _check(lib.sobel4x5_debug_plan_claims(self._h, None, 0, ctypes.byref(n), None), "sobel4x5_debug_plan_claims")
        c = torch.zeros(max(1, n.value), dtype=torch.int32, device=self.device)
        _check(lib.sobel4x5_debug_plan_claims(self._h, c.data_ptr(), c.numel(), ctypes.byref(n),
                                              _stream(self._keep[0][0])), "sobel4x5_debug_plan_claims")
        return c[: n.value]

    def close(self) -> None:
        if getattr(self, "_h", None):
            _check(lib.sobel4x5_plan_destroy(self._h), "sobel4x5_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None) and torch is not None:
                torch.cuda.synchronize(self.device)
                lib.sobel4x5_plan_destroy(self._h)
                self._h = None
        except Exception:
            pass


def sobel4x5_batched(srcs, mags=None, border: int = BORDER_REPLICATE, *, want_mag: bool = True,
                     dir_type: int = DIR_NONE, dirs=None):
    """Magnitudes of many uint8 images of uneven sizes in one persistent launch.

    With dir_type (DIR_S16 / DIR_S32) every image also gets its four
    directional planes, and the result is a list of (mag or None, [planes]).
    """
    if dir_type != DIR_NONE or not want_mag:
        imgs, outs, res = _images_ex(list(srcs), mags, border, want_mag, dir_type, dirs)
        _check(lib.sobel4x5_batched_ex(imgs, outs, len(imgs), border, _stream(srcs[0])), "sobel4x5_batched_ex")
        return res
    if mags is None:
        mags = []
        for s in srcs:
            ho, wo = out_shape(s.size(0), s.size(1), border)
            mags.append(torch.empty((ho, wo), dtype=torch.uint8, device=s.device))
    arr = _images(list(srcs), list(mags), border)
    _check(lib.sobel4x5_batched(arr, len(arr), border, _stream(srcs[0])), "sobel4x5_batched")
    return mags


def sobel4x5_batched_noalloc(srcs, mags=None, border: int = BORDER_REPLICATE):
    """sobel4x5_batched through the allocation-free entry point: its tables
    live in the library's fixed device buffer (calls that overlap on one
    device race).  Output tensors are allocated here unless `mags` is given."""
    if mags is None:
        mags = []
        for s in srcs:
            ho, wo = out_shape(s.size(0), s.size(1), border)
            mags.append(torch.empty((ho, wo), dtype=torch.uint8, device=s.device))
    arr = _images(list(srcs), list(mags), border)
    _check(lib.sobel4x5_batched_noalloc(arr, len(arr), border, _stream(srcs[0])), "sobel4x5_batched_noalloc")
    return mags


def _f32_geom(t: torch.Tensor, name: str):
    if t.dim() == 2:
        t = t.unsqueeze(0)
    if t.dim() != 3 or (t.size(2) > 1 and t.stride(2) != 1):
        raise ValueError("%s must be (B, H, W) or (H, W) with unit column stride" % name)
    return t, t.size(0), t.size(1), t.size(2), t.stride(1) * 4, t.stride(0) * 4


def sobel4x5_f32_fwd(x: torch.Tensor, border: int = BORDER_REPLICATE, out: torch.Tensor | None = None):
    """fp32 magnitude M (B, Ho, Wo) of x (B, H, W) (or (H, W))."""
    _need_cuda(x, torch.float32, "x")
    x3, b, h, w, pitch, bstride = _f32_geom(x, "x")
    ho, wo = out_shape(h, w, border)
    if out is None:
        out = torch.empty((b, ho, wo), dtype=torch.float32, device=x.device)
    _need_cuda(out, torch.float32, "out")
    o3, _, _, _, op, ob = _f32_geom(out, "out")
    if tuple(o3.shape) != (b, ho, wo):
        raise ValueError("out must have shape %s" % ((b, ho, wo),))
    _check(lib.sobel4x5_f32_fwd(x3.data_ptr(), b, w, h, pitch, bstride, border, o3.data_ptr(), op, ob,
                                _stream(x)), "sobel4x5_f32_fwd")
    return out if x.dim() == 3 else out.view(ho, wo)


def sobel4x5_f32_bwd(x: torch.Tensor, grad_mag: torch.Tensor, border: int = BORDER_REPLICATE,
                     out: torch.Tensor | None = None):
    """dL/dx (B, H, W) given dL/dM (B, Ho, Wo)."""
    _need_cuda(x, torch.float32, "x")
    _need_cuda(grad_mag, torch.float32, "grad_mag")
    x3, b, h, w, pitch, bstride = _f32_geom(x, "x")
    g3, gb, gh, gw, gp, gbs = _f32_geom(grad_mag, "grad_mag")
    if (gb, gh, gw) != (b,) + out_shape(h, w, border):
        raise ValueError("grad_mag shape does not match the output shape")
    if out is None:
        out = torch.empty((b, h, w), dtype=torch.float32, device=x.device)
    _need_cuda(out, torch.float32, "out")
    o3, _, _, _, op, ob = _f32_geom(out, "out")
    if tuple(o3.shape) != (b, h, w):
        raise ValueError("out must have shape %s" % ((b, h, w),))
    _check(lib.sobel4x5_f32_bwd(x3.data_ptr(), pitch, bstride, g3.data_ptr(), gp, gbs, b, w, h, border,
                                o3.data_ptr(), op, ob, _stream(x)), "sobel4x5_f32_bwd")
    return out if x.dim() == 3 else out.view(h, w)


def debug_round_mag(S: torch.Tensor, method: int = 0) -> torch.Tensor:
    """The library's uint8 rounding min(255, round(sqrt(S))) of int32 values
    S: method 0 by the fp32 square root, 1 by the LDS table."""
    _need_cuda(S, torch.int32, "S")
    S = S.contiguous()
    out = torch.empty(S.shape, dtype=torch.uint8, device=S.device)
    _check(lib.sobel4x5_debug_round_mag_ex(S.data_ptr(), out.data_ptr(), S.numel(), int(method), _stream(S)),
           "sobel4x5_debug_round_mag_ex")
    return out


def debug_round_quad(q: torch.Tensor) -> torch.Tensor:
    """The four-directional kernels' rounding of int16 quadruples
    (E1, E2, Hp, Hm), shape [n, 4]: min(255, round(sqrt(S))) with
    S = 2 (E1^2 + E2^2 + Hp^2 + Hm^2), through the saturated int16 sum and
    the LDS table."""
    _need_cuda(q, torch.int16, "q")
    if q.dim() != 2 or q.shape[1] != 4:
        raise ValueError("q must have shape [n, 4]")
    q = q.contiguous()
    out = torch.empty(q.shape[0], dtype=torch.uint8, device=q.device)
    _check(lib.sobel4x5_debug_round_quad(q.data_ptr(), out.data_ptr(), q.shape[0], _stream(q)),
           "sobel4x5_debug_round_quad")
    return out


def debug_inject_failure(nth_call: int) -> None:
    """Make the nth_call-th guarded HIP call of the library report a runtime
    failure (0 disarms); tests of the error paths only."""
    _check(lib.sobel4x5_debug_inject_failure(int(nth_call)), "sobel4x5_debug_inject_failure")


def debug_copy(src: torch.Tensor, dst: torch.Tensor) -> None:
    """Plain 128-bit streaming copy of src into dst (same byte size)."""
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("contiguous GPU tensors required")
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n:
        raise ValueError("size mismatch")
    _check(lib.sobel4x5_debug_copy(src.data_ptr(), dst.data_ptr(), n, _stream(src)), "sobel4x5_debug_copy")


def status_string(code: int) -> str:
    return lib.sobel4x5_status_string(code).decode()


def version() -> int:
    return lib.sobel4x5_version()
