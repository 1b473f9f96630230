"""GPU parity of sobel4x5_u8_weighted against the CPU oracle: bit-exact."""
from fractions import Fraction

import numpy as np
import pytest

from paper_2305_00515_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FAMILIES = [(1, 2, 4, 6), (1, 1, 2, 3), (2, Fraction(3, 2), 2, 3), (1, 3, 5, 10)]


def antisym_random(rng, amp):
    """Four random integer 5x5 kernels, antisymmetric under a half turn."""
    w = rng.integers(-amp, amp + 1, size=(4, 5, 5))
    return w - w[:, ::-1, ::-1]                      # k - rot180(k): antisymmetric


def run(api, img, dev, weights, border, dir_type, pitch=None):
    h, w = img.shape
    pitch = w if pitch is None else pitch
    flat = torch.full(((h - 1) * pitch + w + 64,), 0xA5, dtype=torch.uint8, device=dev)
    src = flat.as_strided((h, w), (pitch, 1))
    src.copy_(torch.from_numpy(img))
    mag, dirs = api.sobel4x5_u8_weighted(src, weights, border, dir_type=dir_type)
    torch.cuda.synchronize()
    d = None if dirs is None else np.stack([x.cpu().numpy() for x in dirs]).astype(np.int64)
    return mag.cpu().numpy(), d


@pytest.mark.parametrize("abnm", FAMILIES)
def test_family_parity(oracle_mod, sobel_lib, gpu, abnm):
    w = sobel_lib.family_weights(*sobel_lib.family_products(*abnm))
    dt = sobel_lib.DIR_S16 if np.abs(w).sum(axis=(1, 2)).max() <= 128 else sobel_lib.DIR_S32
    for (h, wd) in [(97, 301), (5, 5), (1, 7), (64, 1030)]:
        img = synth.rect_image(h, wd, h * 31 + wd)
        for border in (0, 1):
            if border and (h < 5 or wd < 5):
                continue
            mag, d = run(sobel_lib, img, gpu, w, border, dt)
            om, od = oracle_mod.sobel_u8(img, border, weights=w)
            assert np.array_equal(mag, om), (abnm, h, wd, border)
            assert np.array_equal(d, od), (abnm, h, wd, border)


def test_random_antisymmetric_kernels(oracle_mod, sobel_lib, gpu):
    rng = np.random.default_rng(11)
    for trial in range(4):
        w = antisym_random(rng, 3 + 40 * trial)
        img = synth.rect_image(70, 211, 500 + trial)
        low = (img % 4).astype(np.uint8)              # low amplitude: unsaturated magnitudes
        for im in (img, low):
            mag, d = run(sobel_lib, im, gpu, w, 0, sobel_lib.DIR_S32, pitch=213)
            om, od = oracle_mod.sobel_u8(im, 0, weights=w)
            assert np.array_equal(mag, om) and np.array_equal(d, od), trial


def test_weights_at_the_int16_limit(oracle_mod, sobel_lib, gpu):
    """Antisymmetry puts each weight twice into sum |k| <= 32768, so |k| <=
    16384: the largest kernels the host accepts, with weights of +-16384 and
    a mix of signs that fills the whole budget, under all four borders."""
    rng = np.random.default_rng(5)
    w = np.zeros((4, 5, 5), np.int64)
    w[0, 0, 0], w[0, 4, 4] = 16384, -16384                      # one pair at the limit
    w[1, 1, 3], w[1, 3, 1] = -16384, 16384
    for k in (2, 3):                                            # 12 random pairs, sum |k| = 32768
        v = rng.integers(1, 2000, 12).astype(np.float64)
        v = np.floor(v / v.sum() * 16384).astype(np.int64)
        v[0] += 16384 - v.sum()
        v *= rng.choice([-1, 1], 12)
        taps = [(i, j) for i in range(3) for j in range(5) if (i, j) < (2, 2)]
        for (i, j), x in zip(taps, v):
            w[k, i, j], w[k, 4 - i, 4 - j] = x, -x
    assert np.abs(w).sum(axis=(1, 2)).max() == 32768 and np.abs(w).max() == 16384
    img = synth.rect_image(37, 130, 77)
    low = (img % 3).astype(np.uint8)
    for border in (0, 1, 2, 3):
        for im in (img, low):
            mag, d = run(sobel_lib, im, gpu, w.astype(np.int32), border, sobel_lib.DIR_S32)
            om, od = oracle_mod.sobel_u8(im, border, weights=w.astype(np.int32))
            assert np.array_equal(mag, om) and np.array_equal(d, od), border


def test_default_weights_match_fast_path(sobel_lib, gpu):
    """The weighted path with Eq. (sobel5_1) equals the packed default path."""
    img = synth.field_image(300, 1000, 9)
    src = torch.from_numpy(img).to(gpu)
    w = sobel_lib.family_weights(1, 2, 4, 6, 8, 12)
    m1, d1 = sobel_lib.sobel4x5_u8(src, dir_type=sobel_lib.DIR_S16)
    m2, d2 = sobel_lib.sobel4x5_u8_weighted(src, w, dir_type=sobel_lib.DIR_S16)
    torch.cuda.synchronize()
    assert torch.equal(m1, m2)
    assert all(torch.equal(a, b) for a, b in zip(d1, d2))


def test_weighted_rejects_bad_weights(sobel_lib, gpu):
    src = torch.zeros((16, 16), dtype=torch.uint8, device=gpu)
    w = sobel_lib.family_weights(1, 2, 4, 6, 8, 12)
    bad = w.copy()
    bad[0, 2, 2] = 1                                   # centre tap of an antisymmetric kernel is 0
    with pytest.raises(sobel_lib.SobelError):
        sobel_lib.sobel4x5_u8_weighted(src, bad)
    big = sobel_lib.family_weights(*sobel_lib.family_products(1, 3, 5, 10))
    with pytest.raises(sobel_lib.SobelError):
        sobel_lib.sobel4x5_u8_weighted(src, big, dir_type=sobel_lib.DIR_S16)


# Magnitudes alone with weights that fit int8 take the matrix-core form
# (SOBEL4X5_W_MFMA=0 forces the kernel above): both paths, unclamped
# (sum |k| <= 181 per kernel) and clamped sums, every border rule.
@pytest.mark.parametrize("path", ["1", "0"])
@pytest.mark.parametrize("amp", [1, 3, 20, 63])
def test_magnitude_only_both_paths(oracle_mod, sobel_lib, gpu, monkeypatch, path, amp):
    monkeypatch.setenv("SOBEL4X5_W_MFMA", path)
    rng = np.random.default_rng(100 + amp)
    w = antisym_random(rng, amp)
    assert np.abs(w).max() <= 127
    for (h, wd) in [(1, 1), (5, 5), (33, 129), (97, 301), (64, 1030), (40, 4099)]:
        img = synth.rect_image(h, wd, h * 17 + wd + amp)
        low = (img % 4).astype(np.uint8)
        for im in (img, low):
            for border in (0, 1, 2, 3):
                if border == 1 and (h < 5 or wd < 5):
                    continue
                mag, _ = run(sobel_lib, im, gpu, w, border, 0)
                om, _ = oracle_mod.sobel_u8(im, border, weights=w, want_dir=False)
                assert np.array_equal(mag, om), (amp, h, wd, border, int((mag != om).sum()))


@pytest.mark.parametrize("abnm", FAMILIES)
def test_family_magnitudes_full_size(oracle_mod, sobel_lib, gpu, abnm):
    """The family's magnitudes at 4096^2 (the matrix-core form whenever the
    weights fit int8), every pixel against the oracle."""
    w = sobel_lib.family_weights(*sobel_lib.family_products(*abnm))
    img = synth.rect_image(4096, 4096, 9)
    mag, _ = run(sobel_lib, img, gpu, w, 0, 0)
    om, _ = oracle_mod.sobel_u8(img, 0, weights=w, want_dir=False)
    assert np.array_equal(mag, om), int((mag != om).sum())
