"""Pins for the oracle's ZERO and REFLECT101 borders (uint8 path).

ZERO reads 0 outside the image; REFLECT101 mirrors about the edge pixel
without repeating it (d c b | a b c d | c b a).  The oracle is checked
against scipy.ndimage (modes 'constant' and 'mirror'), torch's reflect and
zero padding followed by conv2d, symmetry closed forms, and the interior
(where no tap leaves the image, every border rule agrees).  Tiny images,
whose reflection repeats, are included.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi

from paper_2305_00515_amd import synth

REPLICATE, VALID, ZERO, REFLECT101 = 0, 1, 2, 3
SCIPY_MODE = {ZERO: "constant", REFLECT101: "mirror"}
SHAPES = [(1, 1), (1, 2), (2, 1), (2, 2), (2, 3), (3, 3), (3, 5), (4, 4), (5, 7), (9, 6), (33, 47)]


@pytest.mark.parametrize("border", [ZERO, REFLECT101])
@pytest.mark.parametrize("h,w", SHAPES)
def test_four_directions_match_scipy(oracle_mod, border, h, w):
    img = synth.rect_image(h, w, 100 + 7 * h + w)
    K = oracle_mod.weights().astype(np.float64)
    mag, d = oracle_mod.sobel_u8(img, border)
    f = img.astype(np.float64)
    for k in range(4):
        assert np.array_equal(d[k], ndi.correlate(f, K[k], mode=SCIPY_MODE[border], cval=0.0)), k
    s = (d.astype(np.int64) ** 2).sum(axis=0)
    want = np.minimum(np.floor(np.sqrt(s.astype(np.float64)) + 0.5), 255).astype(np.uint8)
    assert np.array_equal(mag, want)


@pytest.mark.parametrize("border", [ZERO, REFLECT101])
@pytest.mark.parametrize("h,w", SHAPES)
def test_two_directions_match_scipy(oracle_mod, border, h, w):
    img = synth.field_image(h, w, 3 + h + w)
    f = img.astype(np.float64)
    mode = SCIPY_MODE[border]
    _, d3 = oracle_mod.sobel_u8_2dir(img, 3, border)
    assert np.array_equal(d3[0], ndi.sobel(f, axis=1, mode=mode, cval=0.0))
    assert np.array_equal(d3[1], ndi.sobel(f, axis=0, mode=mode, cval=0.0))
    K = oracle_mod.weights().astype(np.float64)
    _, d5 = oracle_mod.sobel_u8_2dir(img, 5, border)
    assert np.array_equal(d5[0], ndi.correlate(f, K[0], mode=mode, cval=0.0))
    assert np.array_equal(d5[1], ndi.correlate(f, K[2], mode=mode, cval=0.0))


@pytest.mark.parametrize("border,pad_mode", [(ZERO, "constant"), (REFLECT101, "reflect")])
def test_match_torch_padding(oracle_mod, border, pad_mode):
    torch = pytest.importorskip("torch")
    import torch.nn.functional as F
    img = synth.rect_image(40, 53, 17)
    K = torch.from_numpy(oracle_mod.weights().astype(np.float64))[:, None]
    x = torch.from_numpy(img.astype(np.float64))[None, None]
    xp = F.pad(x, (2, 2, 2, 2), mode=pad_mode)          # torch 'reflect' does not repeat the edge
    want = F.conv2d(xp, K)[0].numpy()                    # conv2d is a correlation
    _, d = oracle_mod.sobel_u8(img, border)
    assert np.array_equal(d, want)


@pytest.mark.parametrize("border", [ZERO, REFLECT101])
def test_interior_agrees_with_replicate(oracle_mod, border):
    img = synth.rect_image(30, 41, 5)
    _, d = oracle_mod.sobel_u8(img, border)
    _, dr = oracle_mod.sobel_u8(img, REPLICATE)
    assert np.array_equal(d[:, 2:-2, 2:-2], dr[:, 2:-2, 2:-2])
    assert not np.array_equal(d, dr)


def test_reflect101_edge_symmetry(oracle_mod):
    """Mirrored about column 0, the image is even in x there, so every filter
    that is odd in x (Gx) vanishes on column 0 and on the last column; Gy
    vanishes on the first and last row."""
    img = synth.rect_image(25, 31, 9)
    _, d = oracle_mod.sobel_u8(img, REFLECT101)
    assert np.all(d[0][:, 0] == 0) and np.all(d[0][:, -1] == 0)
    assert np.all(d[2][0, :] == 0) and np.all(d[2][-1, :] == 0)
    _, d3 = oracle_mod.sobel_u8_2dir(img, 3, REFLECT101)
    assert np.all(d3[0][:, 0] == 0) and np.all(d3[1][0, :] == 0)
    # replicate does not have this property on a generic image
    _, dr = oracle_mod.sobel_u8(img, REPLICATE)
    assert np.any(dr[0][:, 0] != 0)


def test_zero_border_on_a_constant_image(oracle_mod):
    """A constant image c under ZERO: at (y, x) each response is -c times the
    sum of the weights whose taps fall outside the image."""
    c, h, w = 7, 12, 14
    img = np.full((h, w), c, np.uint8)
    _, d = oracle_mod.sobel_u8(img, ZERO)
    K = oracle_mod.weights().astype(np.int64)
    for (y, x) in [(0, 0), (0, 5), (1, 1), (5, 0), (h - 1, w - 1), (h - 2, 3), (6, 6)]:
        for k in range(4):
            outside = sum(K[k, i, j] for i in range(5) for j in range(5)
                          if not (0 <= y + i - 2 < h and 0 <= x + j - 2 < w))
            assert d[k, y, x] == -c * outside
    _, dref = oracle_mod.sobel_u8(img, REFLECT101)
    assert not dref.any()


@pytest.mark.parametrize("border", [ZERO, REFLECT101])
def test_points_match_full(oracle_mod, border):
    img = synth.field_image(50, 70, 4)
    mag, d = oracle_mod.sobel_u8(img, border)
    rng = np.random.default_rng(1)
    ys = np.concatenate([rng.integers(0, 50, 300), [0, 0, 49, 49, 1]])
    xs = np.concatenate([rng.integers(0, 70, 300), [0, 69, 0, 69, 1]])
    pm, pd = oracle_mod.sobel_u8_points(img, ys, xs, border)
    assert np.array_equal(pm, mag[ys, xs]) and np.array_equal(pd, d[:, ys, xs].T)


def test_planted_mistake_reflect_with_edge_repeat(oracle_mod):
    """scipy's 'reflect' repeats the edge pixel (c b a | a b c): that is not
    REFLECT101 and must disagree near the border."""
    img = synth.rect_image(20, 22, 6)
    K = oracle_mod.weights().astype(np.float64)
    _, d = oracle_mod.sobel_u8(img, REFLECT101)
    wrong = ndi.correlate(img.astype(np.float64), K[0], mode="reflect")
    assert not np.array_equal(d[0], wrong)


@pytest.mark.parametrize("border", [ZERO, REFLECT101])
@pytest.mark.parametrize("h,w", [(1, 1), (2, 3), (3, 2), (4, 4), (9, 6), (33, 47)])
def test_real_valued_path_equals_the_integer_path(oracle_mod, border, h, w):
    """On integer images the fp64 responses are exact, so they equal the
    integer path's under the same border rule bit for bit."""
    img = synth.rect_image(h, w, 40 + h + w)
    _, d = oracle_mod.sobel_u8(img, border)
    M, D = oracle_mod.sobel_f64_fwd(img.astype(np.float64)[None], border, want_dir=True)
    assert np.array_equal(D[0], d.astype(np.float64))
    assert np.array_equal(M[0], np.sqrt((d.astype(np.float64) ** 2).sum(0)))


def test_real_valued_adjoint_zero_border_drops_outside_taps(oracle_mod):
    """Under ZERO the adjoint of one output pixel is the four filters cut
    off at the image edge: with g = 1 at the corner pixel only, dx is
    sum_k K_k[t] G_k / M over the in-image taps t and zero elsewhere."""
    x = np.zeros((1, 6, 7))
    x[0, 0, 2] = 1.0                     # an impulse two columns right of (0, 0)
    M, D = oracle_mod.sobel_f64_fwd(x, ZERO, want_dir=True)
    g = np.zeros_like(M)
    g[0, 0, 0] = 1.0
    dx = oracle_mod.sobel_f64_bwd(x, g, ZERO)
    K = oracle_mod.weights().astype(np.float64)
    G = D[0, :, 0, 0]
    want = np.zeros((6, 7))
    for k in range(4):
        want[:3, :3] += K[k, 2:, 2:] * G[k] / M[0, 0, 0]
    np.testing.assert_allclose(dx[0], want, rtol=1e-14, atol=1e-15)
    # the replicate rule folds the outside taps onto the edge instead
    dr = oracle_mod.sobel_f64_bwd(x, g, REPLICATE)
    assert not np.allclose(dr, dx)
