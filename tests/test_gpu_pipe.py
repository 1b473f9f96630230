"""GPU: the host pipeline (host images -> host magnitudes) equals the oracle."""
import numpy as np
import pytest

from paper_2305_00515_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("depth", [1, 3])
def test_pipe_pageable_and_pinned(oracle_mod, sobel_lib, gpu, depth):
    sizes = [(120, 333), (64, 1025), (5, 5), (300, 200), (77, 1920), (1, 9), (250, 640)]
    imgs = [synth.rect_image(h, w, 900 + i) for i, (h, w) in enumerate(sizes)]
    # half the images in pinned CPU tensors (direct copies), half as numpy
    # arrays (pageable: staged), outputs mixed the same way, with row padding
    srcs, mags = [], []
    for i, m in enumerate(imgs):
        h, w = m.shape
        if i % 2:
            t = torch.empty((h, w + 7), dtype=torch.uint8, pin_memory=True)[:, :w]
            t.copy_(torch.from_numpy(m))
            srcs.append(t)
            mags.append(torch.full((h, w + 3), 0x5A, dtype=torch.uint8, pin_memory=True)[:, :w])
        else:
            srcs.append(m)
            mags.append(np.full((h, w), 0x5A, np.uint8))
    p = sobel_lib.Pipe(1920, 300, depth)
    for _ in range(2):                      # the pipeline is reusable
        out = p.run(srcs, mags)
        for i, (m, o) in enumerate(zip(imgs, out)):
            got = o.numpy() if isinstance(o, torch.Tensor) else o
            assert np.array_equal(got, oracle_mod.sobel_u8(m, want_dir=False)[0]), i
    # valid border, outputs allocated by the binding
    out = p.run(srcs[:3], border=sobel_lib.BORDER_VALID)
    for m, o in zip(imgs[:3], out):
        assert np.array_equal(o, oracle_mod.sobel_u8(m, 1, want_dir=False)[0])
    p.close()


def test_pipe_rejects_oversized_images(sobel_lib, gpu):
    p = sobel_lib.Pipe(64, 64, 2)
    with pytest.raises(sobel_lib.SobelError):
        p.run([np.zeros((65, 10), np.uint8)])
    with pytest.raises(sobel_lib.SobelError):
        p.run([np.zeros((10, 65), np.uint8)])
    p.close()


# The guarded HIP calls of one run of 6 images through 3 slots: per image a
# host-to-device copy, a launch and a device-to-host copy, a wait for the
# slot before each of images 3..5, and a final wait per slot (24 in all).
@pytest.mark.parametrize("nth", [1, 2, 3, 5, 9, 13, 17])
def test_pipe_failure_leaves_nothing_pending(oracle_mod, sobel_lib, gpu, nth):
    """A runtime failure injected at the nth guarded call: the run reports
    EHIP, nothing writes that run's outputs after it returned (pinned
    outputs receive their copies straight from the device), and the next
    run, with another and shorter image array, is exact."""
    sizes = [(100, 300), (64, 500), (50, 50), (120, 200), (80, 640), (30, 90)]
    imgs = [synth.rect_image(h, w, 950 + i) for i, (h, w) in enumerate(sizes)]
    srcs, mags = [], []
    for i, m in enumerate(imgs):
        h, w = m.shape
        if i % 2:
            t = torch.empty((h, w), dtype=torch.uint8, pin_memory=True)
            t.copy_(torch.from_numpy(m))
            srcs.append(t)
            mags.append(torch.full((h, w), 0x5A, dtype=torch.uint8, pin_memory=True))
        else:
            srcs.append(m)
            mags.append(np.full((h, w), 0x5A, np.uint8))
    p = sobel_lib.Pipe(640, 120, 3)
    sobel_lib.debug_inject_failure(nth)
    try:
        with pytest.raises(sobel_lib.SobelError) as e:
            p.run(srcs, mags)
    finally:
        sobel_lib.debug_inject_failure(0)
    assert e.value.code == sobel_lib.EHIP
    for m in mags:
        m[...] = 0x5A
    imgs2 = [synth.rect_image(40, 70, 990), synth.rect_image(90, 33, 991)]
    out = p.run(imgs2)
    torch.cuda.synchronize()
    for m, o in zip(imgs2, out):
        assert np.array_equal(o, oracle_mod.sobel_u8(m, want_dir=False)[0])
    for i, m in enumerate(mags):
        got = m.numpy() if isinstance(m, torch.Tensor) else m
        assert (got == 0x5A).all(), "output of image %d of the failed run was written after it returned" % i
    p.close()
