"""GPU parity of the batched persistent path (plans, hipGraph, autotune)."""
import numpy as np
import pytest

from paper_2305_00515_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def upload(img, dev, pitch):
    h, w = img.shape
    flat = torch.zeros(((h - 1) * pitch + w,), dtype=torch.uint8, device=dev)
    v = flat.as_strided((h, w), (pitch, 1))
    v.copy_(torch.from_numpy(np.ascontiguousarray(img)))
    return v


def make_batch(sizes, dev, seed0=1000, border=0, pitch_fn=lambda w: synth.round_up(w, 256)):
    imgs = [synth.rect_image(h, w, seed0 + i) for i, (h, w) in enumerate(sizes)]
    srcs = [upload(m, dev, pitch_fn(m.shape[1])) for m in imgs]
    mags = []
    for (h, w) in sizes:
        ho, wo = (h, w) if border == 0 else (h - 4, w - 4)
        mags.append(torch.full((ho, wo), 0x5A, dtype=torch.uint8, device=dev))
    return imgs, srcs, mags


def check_all(oracle_mod, imgs, mags, border=0):
    torch.cuda.synchronize()
    for i, (img, m) in enumerate(zip(imgs, mags)):
        om, _ = oracle_mod.sobel_u8(img, border, want_dir=False)
        got = m.cpu().numpy()
        assert np.array_equal(got, om), "image %d %s differs in %d pixels" % (i, img.shape, int((got != om).sum()))


SMALL = [(1, 1), (2, 300), (300, 2), (5, 5), (17, 250), (128, 128), (64, 1000), (333, 257),
         (700, 129), (1000, 1000), (7, 4096), (129, 555)]


@pytest.mark.parametrize("border", [0, 1])
def test_small_mixed_batch(oracle_mod, sobel_lib, gpu, border):
    sizes = [s for s in SMALL if border == 0 or min(s) >= 5]
    imgs, srcs, mags = make_batch(sizes, gpu, border=border)
    plan = sobel_lib.Plan(srcs, mags, border)
    plan.launch()
    check_all(oracle_mod, imgs, mags, border)
    # replays reset their queue: clear outputs and launch three more times
    for _ in range(3):
        for m in mags:
            m.fill_(0)
        plan.launch()
        check_all(oracle_mod, imgs, mags, border)
    plan.close()


def test_one_shot_and_cache(oracle_mod, sobel_lib, gpu):
    imgs, srcs, mags = make_batch(SMALL, gpu)
    sobel_lib.sobel4x5_batched(srcs, mags)
    check_all(oracle_mod, imgs, mags)
    for m in mags:
        m.fill_(0)
    sobel_lib.sobel4x5_batched(srcs, mags)          # cached plan
    check_all(oracle_mod, imgs, mags)


def test_batch_of_one_and_duplicates(oracle_mod, sobel_lib, gpu):
    imgs, srcs, mags = make_batch([(400, 900)], gpu)
    sobel_lib.Plan(srcs, mags).launch()
    check_all(oracle_mod, imgs, mags)
    # the same source image twice, two outputs
    m2 = [torch.zeros_like(mags[0]), torch.zeros_like(mags[0])]
    sobel_lib.Plan([srcs[0], srcs[0]], m2).launch()
    check_all(oracle_mod, imgs * 2, m2)


def test_unaligned_images(oracle_mod, sobel_lib, gpu):
    sizes = [(50, 61), (33, 200), (80, 1001)]
    imgs, srcs, mags = make_batch(sizes, gpu, pitch_fn=lambda w: w + 1)
    sobel_lib.Plan(srcs, mags, graph=False).launch()
    check_all(oracle_mod, imgs, mags)


def test_autotune_is_bit_exact(oracle_mod, sobel_lib, gpu, tmp_path, monkeypatch):
    monkeypatch.setenv("SOBEL4X5_TUNE_CACHE", str(tmp_path / "tune.txt"))
    sizes = synth.batch_sizes(16, 5, 128, 1500)
    imgs, srcs, mags = make_batch(sizes, gpu)
    plan = sobel_lib.Plan(srcs, mags, autotune=True)
    info = plan.info()
    assert info["px_per_lane"] in (8, 16) and info["rows_per_tile"] >= 8
    for m in mags:
        m.fill_(0)
    plan.launch()
    check_all(oracle_mod, imgs, mags)
    assert (tmp_path / "tune.txt").exists()
    plan2 = sobel_lib.Plan(srcs, mags, autotune=True)      # served from the cache file
    assert plan2.info()["rows_per_tile"] == info["rows_per_tile"]


def test_config3_full_batch_every_pixel(oracle_mod, sobel_lib, gpu):
    """256 images, sides uniform in [128, 4096]: one persistent graph launch,
    every pixel of every image against the oracle."""
    sizes = synth.batch_sizes(256, 77)
    imgs = [synth.rect_image(h, w, 1000 + i) for i, (h, w) in enumerate(sizes)]
    srcs = [upload(m, gpu, synth.round_up(m.shape[1], 256)) for m in imgs]
    mags = [torch.zeros((h, w), dtype=torch.uint8, device=gpu) for (h, w) in sizes]
    plan = sobel_lib.Plan(srcs, mags)
    plan.launch()
    torch.cuda.synchronize()
    for i, (img, m) in enumerate(zip(imgs, mags)):
        om, _ = oracle_mod.sobel_u8(img, want_dir=False)
        got = m.cpu().numpy()
        assert np.array_equal(got, om), "image %d %s: %d pixels differ" % (i, img.shape, int((got != om).sum()))
    plan.close()


def test_config3_planes_every_value(oracle_mod, sobel_lib, gpu):
    """Magnitudes plus four int16 planes for 32 images of the same size
    distribution (the bench's plane workload, in the static-grid form), every
    value against the oracle."""
    sizes = synth.batch_sizes(32, 78)
    imgs = [synth.rect_image(h, w, 3000 + i) for i, (h, w) in enumerate(sizes)]
    srcs = [upload(m, gpu, synth.round_up(m.shape[1], 256)) for m in imgs]
    mags = [torch.zeros((h, w), dtype=torch.uint8, device=gpu) for (h, w) in sizes]
    dirs = [[torch.zeros((h, w), dtype=torch.int16, device=gpu) for _ in range(4)] for (h, w) in sizes]
    plan = sobel_lib.Plan(srcs, mags, dir_type=1, dirs=dirs)
    plan.launch()
    torch.cuda.synchronize()
    for i, img in enumerate(imgs):
        om, od = oracle_mod.sobel_u8(img)
        assert np.array_equal(mags[i].cpu().numpy(), om), "image %d magnitude" % i
        got = np.stack([d.cpu().numpy() for d in dirs[i]]).astype(np.int32)
        assert np.array_equal(got, od), "image %d planes: %d values differ" % (i, int((got != od).sum()))
    plan.close()


def test_edge_tiles_fast_path(oracle_mod, sobel_lib, gpu):
    """Aligned images whose first and last tile columns are complete: the
    edge tiles take the fast path with mask fix-ups of the group halo."""
    sizes = [(130, 512), (97, 1024), (64, 1027), (200, 2048), (33, 515), (128, 4096)]
    imgs, srcs, mags = make_batch(sizes, gpu)
    sobel_lib.Plan(srcs, mags).launch()
    check_all(oracle_mod, imgs, mags)


def test_one_shot_calls_on_two_streams(oracle_mod, sobel_lib, gpu):
    """The same one-shot batch on two streams without a wait in between:
    each stream gets a cached plan of its own (a plan's work queue admits one
    launch at a time), so a later launch on one stream still covers every
    tile."""
    imgs, srcs, mags = make_batch(SMALL, gpu)
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(3):
        with torch.cuda.stream(a):
            sobel_lib.sobel4x5_batched(srcs, mags)
        with torch.cuda.stream(b):
            sobel_lib.sobel4x5_batched(srcs, mags)
    torch.cuda.synchronize()
    check_all(oracle_mod, imgs, mags)
    for m in mags:
        m.fill_(0)
    torch.cuda.synchronize()
    with torch.cuda.stream(a):
        sobel_lib.sobel4x5_batched(srcs, mags)
    torch.cuda.synchronize()
    check_all(oracle_mod, imgs, mags)


@pytest.mark.parametrize("static", ["0", "1"])
@pytest.mark.parametrize("planes", [False, True])
def test_every_tile_taken_once(oracle_mod, sobel_lib, gpu, monkeypatch, static, planes):
    """Work-queue check (sobel4x5_debug_plan_claims): in both grid forms every
    tile of the plan's table is taken by exactly one wave, on three claim
    launches interleaved with graph launches of the same plan (the persistent
    queue resets itself between launches); the outputs stay exact."""
    monkeypatch.setenv("SOBEL4X5_BATCH_STATIC", static)
    sizes = SMALL + [(2048, 3000), (1500, 517)]
    imgs, srcs, mags = make_batch(sizes, gpu, seed0=4000)
    dirs = ([[torch.zeros(m.shape, dtype=torch.int16, device=gpu) for _ in range(4)] for m in imgs]
            if planes else None)
    plan = sobel_lib.Plan(srcs, mags, dir_type=1, dirs=dirs) if planes else sobel_lib.Plan(srcs, mags)
    for rep in range(3):
        c = plan.claims()
        torch.cuda.synchronize()
        counts = c.cpu().numpy()
        assert counts.size > 0
        assert (counts == 1).all(), "rep %d: %d tiles skipped, %d taken more than once" % (
            rep, int((counts == 0).sum()), int((counts > 1).sum()))
        plan.launch()
    check_all(oracle_mod, imgs, mags)
    plan.close()
