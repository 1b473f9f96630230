"""GPU parity of the matrix-core form of the four-directional uint8
magnitude (u8_mfma.hpp, selected with SOBEL4X5_U8_MFMA=1) against the CPU
oracle: bit-exact, every border rule, ragged sizes, pitches and offsets."""
import numpy as np
import pytest

from paper_2305_00515_amd import synth
from test_gpu_u8 import dev_image, oracle_bands, run

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture
def mfma(monkeypatch):
    monkeypatch.setenv("SOBEL4X5_U8_MFMA", "1")


def check_mag(oracle_mod, api, img, dev, border, **kw):
    mag, _, _ = run(api, img, dev, border, 0, **kw)
    om, _ = oracle_mod.sobel_u8(np.ascontiguousarray(img), border, want_dir=False)
    bad = int((mag != om).sum())
    assert bad == 0, "border %d, %s: %d pixels differ" % (border, img.shape, bad)


# tile edges: 32-row tiles of 128 columns, 16-byte input pieces from 12
# columns left of the tile; widths and heights on both sides of each
@pytest.mark.parametrize("h,w", [(1, 1), (2, 3), (4, 4), (5, 5), (7, 13), (31, 127), (32, 128), (33, 129),
                                 (36, 140), (63, 255), (64, 256), (65, 257), (100, 1000), (37, 4099),
                                 (300, 700), (129, 1921)])
def test_sizes_all_borders(oracle_mod, sobel_lib, gpu, mfma, h, w):
    img = synth.rect_image(h, w, h * 211 + w)
    for border in (0, 1, 2, 3):
        if border == 1 and (h < 5 or w < 5):
            continue
        check_mag(oracle_mod, sobel_lib, img, gpu, border)


@pytest.mark.parametrize("w", [61, 200, 1001])
def test_pitch_and_offset(oracle_mod, sobel_lib, gpu, mfma, w):
    img = synth.rect_image(70, w, w + 5)
    for pitch in (w, w + 3, synth.round_up(w, 256)):
        for off in (0, 1, 7):
            check_mag(oracle_mod, sobel_lib, img, gpu, 0, pitch=pitch, offset=off, mag_pitch=w + (off % 2))


def test_no_writes_outside_outputs(sobel_lib, gpu, mfma):
    img = synth.rect_image(50, 300, 5)
    _, _, flat = run(sobel_lib, img, gpu, mag_pitch=320)
    f = flat.cpu().numpy()
    rows = f[: 50 * 320].reshape(50, 320)
    assert np.all(rows[:, 300:] == 0x5A)
    assert np.all(f[50 * 320:] == 0x5A)


def test_extreme_patterns(oracle_mod, sobel_lib, gpu, mfma):
    h, w = 70, 530
    y, x = np.mgrid[0:h, 0:w]
    for p in [np.full((h, w), 255, np.uint8), np.zeros((h, w), np.uint8),
              (((x + y) % 2) * 255).astype(np.uint8), (((x // 3 + y // 5) % 2) * 255).astype(np.uint8)]:
        for border in (0, 2, 3):
            check_mag(oracle_mod, sobel_lib, p, gpu, border)


@pytest.mark.parametrize("border", [0, 1, 2, 3])
def test_full_size_every_pixel(oracle_mod, sobel_lib, gpu, mfma, border):
    """8192^2 replicate (the benchmarked shape) and 4096^2 under the other
    rules, every pixel against the oracle."""
    n = 8192 if border == 0 else 4096
    img = synth.rect_image(n, n, 3 + border)
    src = dev_image(img, gpu)
    mag = sobel_lib.sobel4x5_u8(src, border)[0]
    torch.cuda.synchronize()
    m = mag.cpu().numpy()
    del mag
    if border == 1:
        # VALID: output rows [y0, y1) read input rows [y0, y1 + 4)
        for y0 in range(0, n - 4, 2048):
            y1 = min(n - 4, y0 + 2048)
            om, _ = oracle_mod.sobel_u8(np.ascontiguousarray(img[y0:y1 + 4]), 1, want_dir=False)
            bad = int((m[y0:y1] != om).sum())
            assert bad == 0, "rows %d..%d: %d pixels differ" % (y0, y1, bad)
        return
    for y0, y1, om, _ in oracle_bands(img, border=border):
        bad = int((m[y0:y1] != om).sum())
        assert bad == 0, "rows %d..%d: %d pixels differ" % (y0, y1, bad)


def test_repeated_calls_match_default_path(sobel_lib, gpu, monkeypatch):
    """Two images in a row through the matrix-core form equal the default
    kernel's output (both launches reuse every wave's LDS tile)."""
    for seed, (h, w) in enumerate([(1080, 1920), (700, 333)]):
        img = synth.field_image(h, w, seed)
        monkeypatch.setenv("SOBEL4X5_U8_MFMA", "1")
        a, _, _ = run(sobel_lib, img, gpu)
        monkeypatch.setenv("SOBEL4X5_U8_MFMA", "0")
        b, _, _ = run(sobel_lib, img, gpu)
        assert np.array_equal(a, b)
