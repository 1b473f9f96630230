"""The allocation-free batched entry point against the allocating one.

sobel4x5_batched_noalloc runs the batched kernel with its tables in the
library's fixed device buffer.  Through the C ABI, two calls in a row on one
stream -- the second with fewer, smaller images, so that whatever the first
call left in the buffer would show -- must give the same bytes as
sobel4x5_batched, and those the oracle's.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_2305_00515_amd import synth

pytestmark = pytest.mark.gpu


def _batch(sizes, seed0, gpu):
    imgs = [synth.rect_image(h, w, seed0 + i) for i, (h, w) in enumerate(sizes)]
    return imgs, [torch.from_numpy(m).to(gpu) for m in imgs]


def _abi_images(api, srcs, mags):
    arr = (api.Image * len(srcs))()
    for i, (s, m) in enumerate(zip(srcs, mags)):
        arr[i].src = s.data_ptr()
        arr[i].mag = m.data_ptr()
        arr[i].height, arr[i].width = s.shape
        arr[i].src_pitch = s.stride(0)
        arr[i].mag_pitch = m.stride(0)
    return arr


@pytest.mark.parametrize("border", [0, 1, 2, 3])
def test_noalloc_matches_the_allocating_call_twice(oracle_mod, sobel_lib, gpu, border):
    api = sobel_lib
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    first = [(300, 517), (1030, 260), (64, 64), (129, 4000), (777, 1111), (5, 9), (2048, 1536), (33, 700)]
    second = [(200, 150), (70, 1030), (9, 5)]
    for sizes, seed in ((first, 500), (second, 600)):
        imgs, srcs = _batch(sizes, seed, gpu)
        ref = [torch.full(api.out_shape(h, w, border), 0xA5, dtype=torch.uint8, device=gpu) for h, w in sizes]
        got = [torch.full(api.out_shape(h, w, border), 0x5A, dtype=torch.uint8, device=gpu) for h, w in sizes]
        a_ref = _abi_images(api, srcs, ref)
        a_got = _abi_images(api, srcs, got)
        assert api.lib.sobel4x5_batched(a_ref, len(sizes), border, stream) == 0
        assert api.lib.sobel4x5_batched_noalloc(a_got, len(sizes), border, stream) == 0, \
            api.lib.sobel4x5_last_error()
        torch.cuda.synchronize()
        for i, (m, r, g) in enumerate(zip(imgs, ref, got)):
            assert torch.equal(r, g), "image %d of %s differs from sobel4x5_batched" % (i, sizes)
            if i < 3:
                want = oracle_mod.sobel_u8(m, border=border, want_dir=False)[0]
                assert np.array_equal(g.cpu().numpy(), want), "image %d of %s differs from the oracle" % (i, sizes)


def test_noalloc_repeats_on_one_buffer(sobel_lib, gpu):
    """Many calls in a row on one stream (each copies its tables into the
    same buffer after the previous launch): the last result equals the
    first, and the queue counters left by each launch do not leak into the
    next."""
    api = sobel_lib
    sizes = [(513, 1025), (100, 3000), (4000, 130)]
    imgs, srcs = _batch(sizes, 700, gpu)
    first = api.sobel4x5_batched_noalloc(srcs)
    torch.cuda.synchronize()
    outs = [torch.empty_like(m) for m in first]
    for _ in range(20):
        api.sobel4x5_batched_noalloc(srcs, outs)
    torch.cuda.synchronize()
    for a, b in zip(first, outs):
        assert torch.equal(a, b)
