"""CPU-only checks of the C ABI: the library loads, exports every declared
entry point, and rejects bad arguments on the host before any launch."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sobel4x5.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sobel4x5_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("sobel4x5_u8", "sobel4x5_batched", "sobel4x5_f32_fwd", "sobel4x5_f32_bwd",
                 "sobel4x5_plan_create", "sobel4x5_plan_launch", "sobel4x5_plan_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol(sobel_lib):
    lib = ctypes.CDLL(str(sobel_lib.LIB_PATH))
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_and_status_strings(sobel_lib):
    assert sobel_lib.version() >= 100
    assert sobel_lib.status_string(0) == "ok"
    assert sobel_lib.status_string(1) == "invalid argument"
    assert sobel_lib.status_string(99) == "unknown status"


FAKE = 0x10000000   # never dereferenced: validation only


def v_u8(api, src=FAKE, w=64, h=32, pitch=64, border=0, mag=FAKE + (1 << 24), mag_pitch=64,
         dir_type=0, dirs=None, dir_pitch=0):
    out = api.Outputs()
    out.mag = mag
    out.mag_pitch = mag_pitch
    out.dir_type = dir_type
    out.dir_pitch = dir_pitch
    for k in range(4):
        out.dir[k] = (dirs[k] if dirs else 0)
    return api.lib.sobel4x5_validate_u8(src, w, h, pitch, border, ctypes.byref(out))


def test_validate_u8(sobel_lib):
    api = sobel_lib
    assert v_u8(api) == 0
    assert v_u8(api, src=0) == api.EINVAL
    assert v_u8(api, w=0) == api.EINVAL
    assert v_u8(api, h=-1) == api.EINVAL
    assert v_u8(api, pitch=63) == api.EINVAL
    assert v_u8(api, border=4) == api.EINVAL
    assert v_u8(api, border=-1) == api.EINVAL
    for b in (2, 3):                                          # ZERO, REFLECT101: H x W output
        assert v_u8(api, border=b) == 0
        assert v_u8(api, border=b, w=1, h=1, pitch=1, mag_pitch=1) == 0
        assert v_u8(api, border=b, mag_pitch=63) == api.EINVAL
    assert v_u8(api, border=1, w=4) == api.EINVAL            # VALID needs >= 5
    assert v_u8(api, border=1, w=5, h=5, pitch=5, mag_pitch=1) == 0
    assert v_u8(api, mag_pitch=10) == api.EINVAL
    assert v_u8(api, mag=FAKE + 100) == api.EINVAL            # overlaps src
    assert v_u8(api, mag=0) == api.EINVAL                     # nothing requested
    dirs = [FAKE + (k + 2) * (1 << 24) for k in range(4)]
    assert v_u8(api, mag=0, dir_type=1, dirs=dirs, dir_pitch=128) == 0
    assert v_u8(api, mag=0, dir_type=2, dirs=dirs, dir_pitch=128) == api.EINVAL   # pitch < 4*64
    assert v_u8(api, mag=0, dir_type=3, dirs=dirs, dir_pitch=256) == api.EINVAL
    assert v_u8(api, mag=0, dir_type=1, dirs=dirs[:3] + [0], dir_pitch=128) == api.EINVAL
    same = [dirs[0]] * 4
    assert v_u8(api, mag=0, dir_type=1, dirs=same, dir_pitch=128) == api.EINVAL  # overlap
    assert v_u8(api, w=1, h=1, pitch=1, mag_pitch=1) == 0
    msg = api.lib.sobel4x5_last_error().decode()
    assert isinstance(msg, str)


def v_op(api, op, src=FAKE, w=64, h=32, pitch=64, border=0, mag=FAKE + (1 << 24), mag_pitch=64,
         dir_type=0, dirs=None, dir_pitch=0):
    out = api.Outputs()
    out.mag = mag
    out.mag_pitch = mag_pitch
    out.dir_type = dir_type
    out.dir_pitch = dir_pitch
    for k in range(4):
        out.dir[k] = (dirs[k] if dirs else 0)
    return api.lib.sobel4x5_validate_u8_op(src, w, h, pitch, op, border, ctypes.byref(out))


def test_validate_u8_op(sobel_lib):
    api = sobel_lib
    for op in (0, 1, 2):
        assert v_op(api, op) == 0
    assert v_op(api, 3) == api.EINVAL
    assert v_op(api, -1) == api.EINVAL
    # VALID: the 3x3 pair needs 3x3 and shrinks by 2, the 5x5 operators need 5x5
    assert v_op(api, 2, border=1, w=3, h=3, pitch=3, mag_pitch=1) == 0
    assert v_op(api, 2, border=1, w=2, h=3, pitch=3, mag_pitch=1) == api.EINVAL
    assert v_op(api, 1, border=1, w=4, h=5, pitch=5, mag_pitch=1) == api.EINVAL
    assert v_op(api, 2, border=1, w=10, h=4, pitch=10, mag_pitch=8) == 0
    assert v_op(api, 2, border=1, w=10, h=4, pitch=10, mag_pitch=7) == api.EINVAL
    # two-directional operators read dir[0] and dir[2] only
    dirs = [FAKE + (k + 2) * (1 << 24) for k in range(4)]
    two = [dirs[0], 0, dirs[2], 0]
    assert v_op(api, 1, mag=0, dir_type=1, dirs=two, dir_pitch=128) == 0
    assert v_op(api, 2, mag=0, dir_type=2, dirs=two, dir_pitch=256) == 0
    assert v_op(api, 0, mag=0, dir_type=1, dirs=two, dir_pitch=128) == api.EINVAL
    assert v_op(api, 2, mag=0, dir_type=1, dirs=[dirs[0], 0, 0, 0], dir_pitch=128) == api.EINVAL
    assert v_op(api, 2, mag=0, dir_type=1, dirs=[dirs[0], 0, dirs[0], 0], dir_pitch=128) == api.EINVAL


def test_validate_batch(sobel_lib):
    api = sobel_lib
    arr = (api.Image * 3)()
    for i in range(3):
        arr[i].src = FAKE + i * (1 << 24)
        arr[i].mag = FAKE + (10 + i) * (1 << 24)
        arr[i].width, arr[i].height = 100 + i, 50
        arr[i].src_pitch = 256
        arr[i].mag_pitch = 256
    assert api.lib.sobel4x5_validate_batch(arr, 3, 0) == 0
    assert api.lib.sobel4x5_validate_batch(arr, 0, 0) == api.EINVAL
    assert api.lib.sobel4x5_validate_batch(arr, 3, 5) == api.EINVAL
    arr[1].mag = arr[0].mag + 10                     # two outputs overlap
    assert api.lib.sobel4x5_validate_batch(arr, 3, 0) == api.EINVAL
    arr[1].mag = arr[2].src                          # output overlaps another image's input
    assert api.lib.sobel4x5_validate_batch(arr, 3, 0) == api.EINVAL
    arr[1].mag = FAKE + 11 * (1 << 24)
    arr[2].width = 300                               # pitch too small
    assert api.lib.sobel4x5_validate_batch(arr, 3, 0) == api.EINVAL
    arr[2].width = 102
    for b in (2, 3):
        assert api.lib.sobel4x5_validate_batch(arr, 3, b) == 0


def test_validate_batch_with_outputs(sobel_lib):
    """Per-image outputs: directional planes take part in every overlap check,
    and imgs[i].mag is ignored."""
    api = sobel_lib
    n = 3
    arr = (api.Image * n)()
    outs = (api.Outputs * n)()
    for i in range(n):
        arr[i].src = FAKE + i * (1 << 24)
        arr[i].mag = 0                                  # ignored with outputs
        arr[i].width, arr[i].height = 100, 50
        arr[i].src_pitch = 128
        outs[i].mag = FAKE + (10 + i) * (1 << 24)
        outs[i].mag_pitch = 128
        outs[i].dir_type = 1
        outs[i].dir_pitch = 256
        for k in range(4):
            outs[i].dir[k] = FAKE + (20 + 4 * i + k) * (1 << 24)
    v = api.lib.sobel4x5_validate_batch_ex
    assert v(arr, outs, n, 0) == 0
    assert v(arr, None, n, 0) == api.EINVAL             # plain batch: mag must be given
    outs[2].dir[3] = outs[0].dir[1] + 64                # planes of two images overlap
    assert v(arr, outs, n, 0) == api.EINVAL
    outs[2].dir[3] = arr[1].src                         # a plane overlaps an input
    assert v(arr, outs, n, 0) == api.EINVAL
    outs[2].dir[3] = FAKE + 40 * (1 << 24)
    outs[1].dir_pitch = 100                             # pitch below 2 * width
    assert v(arr, outs, n, 0) == api.EINVAL
    outs[1].dir_pitch = 256
    outs[0].mag = 0                                     # planes only
    assert v(arr, outs, n, 3) == 0
    outs[0].dir_type = 0                                # nothing requested for image 0
    assert v(arr, outs, n, 0) == api.EINVAL


def test_validate_f32(sobel_lib):
    api = sobel_lib
    f = api.lib.sobel4x5_validate_f32
    src, out = FAKE, FAKE + (1 << 26)
    assert f(src, 2, 64, 32, 256, 256 * 32, 0, out, 256, 256 * 32) == 0
    assert f(src, 2, 64, 32, 256, 256 * 31, 0, out, 256, 256 * 32) == api.EINVAL   # bstride
    assert f(src, 2, 64, 32, 255, 256 * 32, 0, out, 256, 256 * 32) == api.EINVAL   # pitch % 4
    assert f(src + 2, 2, 64, 32, 256, 256 * 32, 0, out, 256, 256 * 32) == api.EINVAL
    assert f(src, 2, 64, 32, 256, 256 * 32, 0, src + 64, 256, 256 * 32) == api.EINVAL  # overlap
    assert f(src, 1, 4, 4, 16, 0, 1, out, 16, 0) == api.EINVAL                     # VALID < 5
    assert f(src, 0, 8, 8, 32, 0, 0, out, 32, 0) == 0                               # empty batch
    for b in (2, 3):                                                                  # ZERO, REFLECT101
        assert f(src, 2, 64, 32, 256, 256 * 32, b, out, 256, 256 * 32) == 0
        assert f(src, 1, 1, 1, 4, 0, b, out, 4, 0) == 0                              # any H, W >= 1
    assert f(src, 2, 64, 32, 256, 256 * 32, 4, out, 256, 256 * 32) == api.EINVAL     # no such rule


def test_plan_handles_are_checked(sobel_lib):
    api = sobel_lib
    assert api.lib.sobel4x5_plan_launch(None, None) == api.EINVAL
    assert api.lib.sobel4x5_plan_destroy(None) == api.EINVAL
    bogus = ctypes.create_string_buffer(256)
    assert api.lib.sobel4x5_plan_destroy(ctypes.cast(bogus, ctypes.c_void_p)) == api.EINVAL


def test_debug_round_mag_rejects_bad_args(sobel_lib):
    api = sobel_lib
    assert api.lib.sobel4x5_debug_round_mag(None, None, 5, None) == api.EINVAL
    assert api.lib.sobel4x5_debug_round_mag(None, None, -1, None) == api.EINVAL


def test_pipe_arguments_are_checked_before_any_gpu_work(sobel_lib):
    import ctypes
    lib = sobel_lib.lib
    h = ctypes.c_void_p()
    assert lib.sobel4x5_pipe_create(64, 64, 0, ctypes.byref(h)) == sobel_lib.EINVAL     # depth 0
    assert lib.sobel4x5_pipe_create(64, 64, 17, ctypes.byref(h)) == sobel_lib.EINVAL    # depth > 16
    assert lib.sobel4x5_pipe_create(0, 64, 2, ctypes.byref(h)) == sobel_lib.EINVAL
    assert lib.sobel4x5_pipe_create(64, 64, 2, None) == sobel_lib.EINVAL
    assert lib.sobel4x5_pipe_run(None, None, 0, 0) == sobel_lib.EINVAL
    assert lib.sobel4x5_pipe_destroy(None) == sobel_lib.EINVAL


def _fake_batch(api, n, w, h):
    arr = (api.Image * n)()
    span = w * h
    for i in range(n):
        arr[i].src = FAKE + 2 * i * span
        arr[i].mag = FAKE + (2 * i + 1) * span
        arr[i].width, arr[i].height = w, h
        arr[i].src_pitch = arr[i].mag_pitch = w
    return arr


def test_noalloc_limits_are_rejected_before_any_gpu_call(sobel_lib):
    """The allocation-free batched call takes at most
    SOBEL4X5_NOALLOC_MAX_IMAGES images and SOBEL4X5_NOALLOC_MAX_TILES
    wave-tiles; a batch beyond either (or an invalid one) returns EINVAL
    from host checks alone -- this runs without a GPU."""
    api = sobel_lib
    f = api.lib.sobel4x5_batched_noalloc
    assert f(_fake_batch(api, 1025, 16, 16), 1025, 0, None) == api.EINVAL       # > 1024 images
    assert b"1024" in api.lib.sobel4x5_last_error()
    # 8192^2 with 32-row tiles: 896 wave-tiles an image at 16 px/lane (1792
    # at 8), so 147 of them exceed 65536 under either tile width
    assert f(_fake_batch(api, 147, 8192, 8192), 147, 0, None) == api.EINVAL
    assert b"65536" in api.lib.sobel4x5_last_error()
    bad = _fake_batch(api, 4, 64, 64)
    bad[2].mag = bad[1].src                                                    # output overlaps an input
    assert f(bad, 4, 0, None) == api.EINVAL
    assert f(None, 1, 0, None) == api.EINVAL
