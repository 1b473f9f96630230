"""GPU parity of the ZERO and REFLECT101 borders against the CPU oracle
(bit-exact), on every uint8 entry point: single image (fast, edge-strip,
ragged and byte paths), the two-directional operators, run-time weights,
batches (with and without directional planes) and the host pipeline.
Also the batched directional planes under every border."""
import numpy as np
import pytest

from paper_2305_00515_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REPLICATE, VALID, ZERO, REFLECT101 = 0, 1, 2, 3
NEW = (ZERO, REFLECT101)


def dev_image(img, dev, pitch=None, offset=0):
    h, w = img.shape
    pitch = w if pitch is None else pitch
    flat = torch.full((offset + max(h - 1, 0) * pitch + w + 64,), 0xA5, dtype=torch.uint8, device=dev)
    view = flat.as_strided((h, w), (pitch, 1), offset)
    view.copy_(torch.from_numpy(np.ascontiguousarray(img)))
    return view


def out_hw(h, w, border, r=2):
    return (h - 2 * r, w - 2 * r) if border == VALID else (h, w)


def check_single(oracle_mod, api, img, dev, border, dir_type=0, pitch=None, offset=0):
    src = dev_image(img, dev, pitch, offset)
    mag, dirs = api.sobel4x5_u8(src, border, dir_type=dir_type)
    torch.cuda.synchronize()
    om, od = oracle_mod.sobel_u8(np.ascontiguousarray(img), border)
    m = mag.cpu().numpy()
    assert np.array_equal(m, om), "border %d: magnitude differs (%d px)" % (border, int((m != om).sum()))
    if dirs is not None:
        d = np.stack([x.cpu().numpy() for x in dirs]).astype(np.int32)
        assert np.array_equal(d, od), "border %d: planes differ (%d values)" % (border, int((d != od).sum()))


@pytest.mark.parametrize("border", NEW)
@pytest.mark.parametrize("h,w", [(1, 1), (1, 2), (2, 1), (2, 2), (2, 3), (3, 3), (3, 4), (4, 7), (5, 5),
                                 (7, 15), (16, 17), (33, 256), (20, 257), (40, 1000), (9, 1920), (300, 4099)])
def test_single_size_sweep(oracle_mod, sobel_lib, gpu, border, h, w):
    img = synth.rect_image(h, w, h * 7919 + w + 11 * border)
    check_single(oracle_mod, sobel_lib, img, gpu, border, 2)
    check_single(oracle_mod, sobel_lib, img, gpu, border, 0)


@pytest.mark.parametrize("border", NEW)
@pytest.mark.parametrize("w", [512, 513, 514, 515, 1024, 1025, 1026, 1027, 2048, 2051])
def test_single_edge_strips(oracle_mod, sobel_lib, gpu, border, w):
    """Aligned rows: the edge strips take the fast path with the border's
    halo selectors (0..3 valid bytes in the right halo dword); ragged widths
    add the slow strip with its in-register fix-ups."""
    img = synth.rect_image(45, w, 31 * w + border)
    p = synth.round_up(w, 16)
    check_single(oracle_mod, sobel_lib, img, gpu, border, 0, pitch=p)
    check_single(oracle_mod, sobel_lib, img, gpu, border, 1, pitch=p)
    low = (img % 3).astype(np.uint8)            # unsaturated magnitudes near the edges
    check_single(oracle_mod, sobel_lib, low, gpu, border, 0, pitch=p)


@pytest.mark.parametrize("border", NEW)
def test_single_unaligned_rows(oracle_mod, sobel_lib, gpu, border):
    img = synth.rect_image(37, 1001, 5 + border)
    for pitch, off in ((1001, 0), (1002, 1), (1024, 3)):
        check_single(oracle_mod, sobel_lib, img, gpu, border, 0, pitch=pitch, offset=off)
    check_single(oracle_mod, sobel_lib, img, gpu, border, 1, pitch=1002, offset=1)


@pytest.mark.parametrize("border", NEW)
def test_single_patterns(oracle_mod, sobel_lib, gpu, border):
    h, w = 70, 530
    y, x = np.mgrid[0:h, 0:w]
    pats = [np.full((h, w), 255, np.uint8), np.full((h, w), 3, np.uint8),
            (((x + y) % 2) * 255).astype(np.uint8), ((x * 7 + y * 13) % 256).astype(np.uint8)]
    for p in pats:
        check_single(oracle_mod, sobel_lib, p, gpu, border, 2, pitch=544)


@pytest.mark.parametrize("border", NEW)
def test_single_full_size(oracle_mod, sobel_lib, gpu, border):
    n = 8192
    img = synth.rect_image(n, n, 3)
    src = dev_image(img, gpu)
    mag = sobel_lib.sobel4x5_u8(src, border)[0]
    torch.cuda.synchronize()
    om, _ = oracle_mod.sobel_u8(img, border, want_dir=False)
    assert np.array_equal(mag.cpu().numpy(), om)


@pytest.mark.parametrize("border", NEW)
@pytest.mark.parametrize("op,size", [(1, 5), (2, 3)])
def test_two_directional_operators(oracle_mod, sobel_lib, gpu, border, op, size):
    for (h, w, pitch) in ((1, 1, 1), (2, 3, 3), (3, 3, 3), (17, 63, 64), (45, 1027, 1040), (64, 2048, 2048),
                          (33, 1001, 1002)):
        img = synth.rect_image(h, w, 3 * h + w + op)
        src = dev_image(img, gpu, pitch)
        mag, dirs = sobel_lib.sobel4x5_u8_op(src, op, border, dir_type=1)
        torch.cuda.synchronize()
        om, od = oracle_mod.sobel_u8_2dir(img, size, border)
        assert np.array_equal(mag.cpu().numpy(), om), (h, w)
        d = np.stack([x.cpu().numpy() for x in dirs]).astype(np.int32)
        assert np.array_equal(d, od), (h, w)


@pytest.mark.parametrize("border", NEW)
def test_run_time_weights(oracle_mod, sobel_lib, gpu, border):
    w = sobel_lib.family_weights(*sobel_lib.family_products(1, 3, 5, 10))
    for (h, wd) in ((1, 1), (2, 2), (5, 9), (40, 300), (129, 1000)):
        img = synth.rect_image(h, wd, 7 * h + wd)
        src = dev_image(img, gpu)
        mag, dirs = sobel_lib.sobel4x5_u8_weighted(src, w, border, dir_type=2)
        torch.cuda.synchronize()
        om, od = oracle_mod.sobel_u8(img, border, weights=w)
        assert np.array_equal(mag.cpu().numpy(), om), (h, wd)
        assert np.array_equal(np.stack([x.cpu().numpy() for x in dirs]), od), (h, wd)


def batch_images():
    sizes = [(1, 1), (2, 2), (1, 7), (5, 3), (64, 64), (300, 200), (130, 520), (77, 1030), (513, 129), (40, 2048)]
    return [synth.rect_image(h, w, 1000 + i) for i, (h, w) in enumerate(sizes)]


@pytest.mark.parametrize("border", NEW)
def test_batched_magnitudes(oracle_mod, sobel_lib, gpu, border):
    imgs = batch_images()
    srcs = [dev_image(m, gpu, synth.round_up(m.shape[1], 16)) for m in imgs]
    mags = sobel_lib.sobel4x5_batched(srcs, border=border)
    torch.cuda.synchronize()
    for m, g in zip(imgs, mags):
        assert np.array_equal(g.cpu().numpy(), oracle_mod.sobel_u8(m, border, want_dir=False)[0]), m.shape


@pytest.mark.parametrize("border", [REPLICATE, VALID, ZERO, REFLECT101])
@pytest.mark.parametrize("dir_type", [1, 2])
def test_batched_directional_planes(oracle_mod, sobel_lib, gpu, border, dir_type):
    imgs = [m for m in batch_images() if border != VALID or min(m.shape) >= 5]
    srcs = [dev_image(m, gpu, synth.round_up(m.shape[1], 16)) for m in imgs]
    res = sobel_lib.sobel4x5_batched(srcs, border=border, dir_type=dir_type)
    torch.cuda.synchronize()
    for m, (g, planes) in zip(imgs, res):
        om, od = oracle_mod.sobel_u8(m, border)
        assert np.array_equal(g.cpu().numpy(), om), m.shape
        d = np.stack([x.cpu().numpy() for x in planes]).astype(np.int32)
        assert np.array_equal(d, od), m.shape


@pytest.mark.parametrize("static", ["0", "1"])
@pytest.mark.parametrize("planes", [False, True])
def test_batched_grid_forms(oracle_mod, sobel_lib, gpu, monkeypatch, static, planes):
    """Both grid forms of the batched kernel, for magnitudes and for planes:
    the persistent grid with its work queue (which the last wave resets for
    the next launch) and the static grid of one wave per tile, each plan
    replayed three times with the outputs poisoned in between."""
    monkeypatch.setenv("SOBEL4X5_BATCH_STATIC", static)
    imgs = batch_images()
    srcs = [dev_image(m, gpu, synth.round_up(m.shape[1], 16)) for m in imgs]
    mags = [torch.empty(m.shape, dtype=torch.uint8, device=gpu) for m in imgs]
    dirs = [[torch.empty(m.shape, dtype=torch.int16, device=gpu) for _ in range(4)] for m in imgs] if planes else None
    plan = (sobel_lib.Plan(srcs, mags, REFLECT101, dir_type=1, dirs=dirs) if planes
            else sobel_lib.Plan(srcs, mags, REFLECT101))
    for _ in range(3):
        for t in mags:
            t.fill_(7)
        for ps in dirs or []:
            for t in ps:
                t.fill_(7)
        plan.launch()
        torch.cuda.synchronize()
        for i, m in enumerate(imgs):
            om, od = oracle_mod.sobel_u8(m, REFLECT101)
            assert np.array_equal(mags[i].cpu().numpy(), om), m.shape
            if planes:
                assert np.array_equal(np.stack([x.cpu().numpy() for x in dirs[i]]).astype(np.int32), od), m.shape
    plan.close()


def test_batched_planes_only_unaligned_and_autotuned_plan(oracle_mod, sobel_lib, gpu, tmp_path, monkeypatch):
    """Planes without magnitudes, unaligned sources (byte path), and an
    autotuned plan whose candidate shapes are checked on every plane."""
    monkeypatch.setenv("SOBEL4X5_TUNE_CACHE", str(tmp_path / "tune.txt"))
    imgs = batch_images()[3:]
    srcs = [dev_image(m, gpu, m.shape[1] + 1, 1) for m in imgs]
    res = sobel_lib.sobel4x5_batched(srcs, border=REFLECT101, want_mag=False, dir_type=1)
    torch.cuda.synchronize()
    for m, (g, planes) in zip(imgs, res):
        assert g is None
        _, od = oracle_mod.sobel_u8(m, REFLECT101)
        assert np.array_equal(np.stack([x.cpu().numpy() for x in planes]).astype(np.int32), od)
    srcs = [dev_image(m, gpu, synth.round_up(m.shape[1], 16)) for m in imgs]
    mags = [torch.empty(m.shape, dtype=torch.uint8, device=gpu) for m in imgs]
    dirs = [[torch.empty(m.shape, dtype=torch.int16, device=gpu) for _ in range(4)] for m in imgs]
    plan = sobel_lib.Plan(srcs, mags, ZERO, autotune=True, dir_type=1, dirs=dirs)
    for _ in range(2):
        for t in mags:
            t.fill_(7)
        for ps in dirs:
            for t in ps:
                t.fill_(7)
        plan.launch()
        torch.cuda.synchronize()
        for m, g, ps in zip(imgs, mags, dirs):
            om, od = oracle_mod.sobel_u8(m, ZERO)
            assert np.array_equal(g.cpu().numpy(), om)
            assert np.array_equal(np.stack([x.cpu().numpy() for x in ps]).astype(np.int32), od)
    # a second plan is served from the cache file, grid form included
    plan2 = sobel_lib.Plan(srcs, mags, ZERO, autotune=True, dir_type=1, dirs=dirs)
    assert plan2.info() == plan.info()
    for t in mags:
        t.fill_(7)
    plan2.launch()
    torch.cuda.synchronize()
    for m, g in zip(imgs, mags):
        assert np.array_equal(g.cpu().numpy(), oracle_mod.sobel_u8(m, ZERO)[0])
    plan2.close()
    plan.close()


@pytest.mark.parametrize("border", NEW)
def test_pipeline(oracle_mod, sobel_lib, gpu, border):
    imgs = batch_images()[4:]
    pipe = sobel_lib.Pipe(2048, 600, 2)
    outs = pipe.run(imgs, border=border)
    pipe.close()
    for m, o in zip(imgs, outs):
        assert np.array_equal(o, oracle_mod.sobel_u8(m, border, want_dir=False)[0]), m.shape


@pytest.mark.parametrize("border", NEW)
def test_fp32_pitched_buffers_through_the_c_abi(oracle_mod, sobel_lib, gpu, border):
    """The fp32 pair under the new borders on row-pitched, batch-strided
    buffers (rows padded to 80 floats, images 7 rows apart), called through
    the C ABI with raw pointers; pixels of the padding stay untouched."""
    api = sobel_lib
    b, h, w, wp, hp = 2, 33, 70, 80, 40
    x = np.stack([synth.rect_image(h, w, 60 + i) for i in range(b)]).astype(np.float32) / np.float32(255)
    xs = torch.full((b, hp, wp), 7.0, device=gpu)
    xs[:, :h, :w] = torch.from_numpy(x).to(gpu)
    m = torch.full((b, hp, wp), -1.0, device=gpu)
    g = np.random.default_rng(3).standard_normal((b, h, w)).astype(np.float32)
    gs = torch.full((b, hp, wp), 9.0, device=gpu)
    gs[:, :h, :w] = torch.from_numpy(g).to(gpu)
    dx = torch.full((b, hp, wp), -2.0, device=gpu)
    pitch, bstride = wp * 4, hp * wp * 4
    rc = api.lib.sobel4x5_f32_fwd(xs.data_ptr(), b, w, h, pitch, bstride, border, m.data_ptr(), pitch, bstride, None)
    assert rc == 0
    rc = api.lib.sobel4x5_f32_bwd(xs.data_ptr(), pitch, bstride, gs.data_ptr(), pitch, bstride, b, w, h, border,
                                  dx.data_ptr(), pitch, bstride, None)
    assert rc == 0
    torch.cuda.synchronize()
    M, D = m.cpu().numpy(), dx.cpu().numpy()
    Mr, _ = oracle_mod.sobel_f64_fwd(x.astype(np.float64), border)
    s = oracle_mod.sobel_f64_fwd_scale(x.astype(np.float64), border)
    assert np.all(np.abs(M[:, :h, :w] - Mr) <= 1e-5 * np.maximum(Mr, s) + 1e-30)
    ref = oracle_mod.sobel_f64_bwd(x.astype(np.float64), g.astype(np.float64), border)
    A = oracle_mod.sobel_f64_bwd_scale(x.astype(np.float64), g.astype(np.float64), border)
    assert np.all(np.abs(D[:, :h, :w] - ref) <= 1e-5 * A + 1e-30)
    assert np.all(M[:, h:, :] == -1.0) and np.all(M[:, :, w:] == -1.0)
    assert np.all(D[:, h:, :] == -2.0) and np.all(D[:, :, w:] == -2.0)


def test_batched_mixed_outputs_through_the_c_abi(oracle_mod, sobel_lib, gpu):
    """One batch whose images ask for different outputs: magnitude only,
    int16 planes only, magnitude + int32 planes, magnitude + int16 planes
    (the C ABI's per-image sobel4x5_outputs)."""
    api = sobel_lib
    imgs = batch_images()[2:8]
    kinds = [(True, 0), (False, 1), (True, 2), (True, 1), (False, 2), (True, 0)]
    border = REFLECT101
    n = len(imgs)
    srcs = [dev_image(m, gpu, synth.round_up(m.shape[1], 16)) for m in imgs]
    arr = (api.Image * n)()
    outs = (api.Outputs * n)()
    keep = []
    for i, (m, s, (want_mag, dt)) in enumerate(zip(imgs, srcs, kinds)):
        o, (h, w, p), res = api._u8_outputs(s, border, None, want_mag, dt, None)
        outs[i] = o
        arr[i].src = s.data_ptr()
        arr[i].width, arr[i].height, arr[i].src_pitch = w, h, p
        keep.append(res)
    api._check(api.lib.sobel4x5_batched_ex(arr, outs, n, border, api._stream(srcs[0])), "sobel4x5_batched_ex")
    torch.cuda.synchronize()
    for m, (want_mag, dt), (g, planes) in zip(imgs, kinds, keep):
        om, od = oracle_mod.sobel_u8(m, border)
        if want_mag:
            assert np.array_equal(g.cpu().numpy(), om), m.shape
        else:
            assert g is None
        if dt:
            d = np.stack([x.cpu().numpy() for x in planes]).astype(np.int32)
            assert np.array_equal(d, od), m.shape
        else:
            assert planes is None
