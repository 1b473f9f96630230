"""Pins for the CPU oracle: checks against what the paper and mathematics fix.

None of these tests re-types the oracle's loops.  The oracle is checked
against (a) the paper's second printing of the weights, (b) library routines
that implement the same correlation independently (scipy.ndimage,
scipy.signal, torch conv2d), (c) hand-derived closed forms (ramps, steps,
impulses, constants), (d) exact invariants (dihedral symmetries, linearity),
and (e) exact integer rounding.  Each family is chosen so that a dropped
term, a wrong sign, a swapped plane or a transposed filter fails at least one
of them (see test_planted_mistakes_are_caught).
"""
import math
import os

import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.signal as sps

from paper_2305_00515_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
PLANES = ("Gx", "Gd", "Gy", "Gdt")


def read_matrices(path):
    mats, cur, name = {}, [], None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                if name:
                    mats[name] = np.array(cur, dtype=np.int64)
                name, cur = line[1:-1], []
            else:
                cur.append([int(v) for v in line.split()])
    mats[name] = np.array(cur, dtype=np.int64)
    return mats


@pytest.fixture(scope="module")
def K_golden():
    m = read_matrices(os.path.join(GOLDEN, "eq_sobel5_1.txt"))
    return np.stack([m[p] for p in PLANES])


def param_weights(a, b, n, m):
    """Eq. (sobel5_param) (Sec. 3.2), typed from its printed matrices."""
    Kx = a * np.array([[-1, -b, 0, b, 1],
                       [-n, -n * b, 0, n * b, n],
                       [-m, -m * b, 0, m * b, m],
                       [-n, -n * b, 0, n * b, n],
                       [-1, -b, 0, b, 1]])
    Ky = a * np.array([[-1, -n, -m, -n, -1],
                       [-b, -n * b, -m * b, -n * b, -b],
                       [0, 0, 0, 0, 0],
                       [b, n * b, m * b, n * b, b],
                       [1, n, m, n, 1]])
    Kd = a * np.array([[-m, -n, -1, -b, 0],
                       [-n, -m * b, -n * b, 0, b],
                       [-1, -n * b, 0, n * b, 1],
                       [-b, 0, n * b, m * b, n],
                       [0, b, 1, n, m]])
    Kdt = a * np.array([[0, -b, -1, -n, -m],
                        [b, 0, -n * b, -m * b, -n],
                        [1, n * b, 0, -n * b, -1],
                        [n, m * b, n * b, 0, -b],
                        [m, n, 1, b, 0]])
    return np.stack([Kx, Kd, Ky, Kdt])


# ----------------------------------------------------------------------------
# (a) weights: two printings, and the paper's derived matrices
# ----------------------------------------------------------------------------

def test_weights_match_golden_typing(oracle_mod, K_golden):
    assert np.array_equal(oracle_mod.weights(), K_golden)


def test_weights_match_generalized_form(oracle_mod):
    # Eq. (sobel5_param) at (a, b, n, m) = (1, 2, 4, 6) is Eq. (sobel5_1).
    assert np.array_equal(oracle_mod.weights(), param_weights(1, 2, 4, 6))


@pytest.mark.parametrize("abnm", [(1, 2, 4, 6), (1, 1, 2, 3), (2, 3, 5, 7), (1, 2, 5, 8)])
def test_paper_diagonal_transforms(abnm):
    """Eq. (sobel5_kd+-) and Eq. (sobel5_4), Sec. 4.3 (diagonal optimisation)."""
    a, b, n, m = abnm
    Kx, Kd, Ky, Kdt = param_weights(a, b, n, m)
    Kdp = a * np.array([[-m, -n - b, -2, -n - b, -m],
                        [b - n, -m * b, -2 * n * b, -m * b, b - n],
                        [0, 0, 0, 0, 0],
                        [n - b, m * b, 2 * n * b, m * b, n - b],
                        [m, n + b, 2, n + b, m]])
    Kdm = a * np.array([[-m, b - n, 0, n - b, m],
                        [-n - b, -m * b, 0, m * b, n + b],
                        [-2, -2 * n * b, 0, 2 * n * b, 2],
                        [-n - b, -m * b, 0, m * b, n + b],
                        [-m, b - n, 0, n - b, m]])
    assert np.array_equal(Kd + Kdt, Kdp)
    assert np.array_equal(Kd - Kdt, Kdm)
    col1 = np.array([m, n + b, 2, n + b, m])
    row1 = np.array([-1, -b, 0, b, 1])
    col2 = np.array([m * b + b - n, n * b + b * b - m * b, 2 * b - 2 * n * b,
                     n * b + b * b - m * b, m * b - n + b])
    row2 = np.array([0, -1, 0, 1, 0])
    assert np.array_equal(a * (np.outer(col1, row1) - np.outer(col2, row2)), Kdm)
    # the separable K_x of Eq. (sobel5_param)
    assert np.array_equal(a * np.outer([1, n, m, n, 1], [-1, -b, 0, b, 1]), Kx)
    assert np.array_equal(Ky, Kx.T)


def test_weight_structure(oracle_mod):
    K = oracle_mod.weights().astype(np.int64)
    for k in range(4):
        assert K[k].sum() == 0
        assert np.abs(K[k]).sum() == 96
        assert np.array_equal(np.rot90(K[k], 2), -K[k])      # antisymmetric under rot180
    assert np.array_equal(K[1], K[1].T)                     # Gd symmetric
    assert np.array_equal(K[3].T, -K[3])                    # Gdt antisymmetric
    assert np.array_equal(K[3], np.fliplr(K[1]))            # Gdt = fliplr(Gd)


# ----------------------------------------------------------------------------
# (b) library routines computing the same replicate-bordered correlation
# ----------------------------------------------------------------------------

def scipy_dirs(img, K):
    I = img.astype(np.int64)
    return np.stack([ndi.correlate(I, K[k].astype(np.int64), mode="nearest") for k in range(4)])


def exact_mag(dirs):
    S = (dirs.astype(np.int64) ** 2).sum(axis=0)
    out = np.empty(S.shape, np.int64)
    flat = S.ravel()
    res = out.ravel()
    for i, s in enumerate(flat):
        r = math.isqrt(int(s))
        res[i] = min(255, r + (1 if s - r * r > r else 0))
    return out.astype(np.uint8)


@pytest.mark.parametrize("h,w", [(1, 1), (1, 7), (7, 1), (2, 3), (3, 2), (4, 4), (5, 5),
                                 (6, 8), (8, 6), (13, 17), (64, 33)])
def test_replicate_matches_scipy(oracle_mod, K_golden, h, w):
    rng = np.random.default_rng(h * 100 + w)
    img = rng.integers(0, 256, size=(h, w), dtype=np.uint8)
    mag, d = oracle_mod.sobel_u8(img)
    ref = scipy_dirs(img, K_golden)
    assert np.array_equal(d, ref)
    assert np.array_equal(mag, exact_mag(ref))


def test_tiny_images_exhaustive_shapes(oracle_mod, K_golden):
    """Every H, W in 1..8, random and extreme values, against scipy."""
    rng = np.random.default_rng(5)
    for h in range(1, 9):
        for w in range(1, 9):
            for kind in range(3):
                if kind == 0:
                    img = rng.integers(0, 256, size=(h, w), dtype=np.uint8)
                elif kind == 1:
                    img = (rng.integers(0, 2, size=(h, w)) * 255).astype(np.uint8)
                else:
                    img = rng.integers(0, 3, size=(h, w), dtype=np.uint8)
                mag, d = oracle_mod.sobel_u8(img)
                ref = scipy_dirs(img, K_golden)
                assert np.array_equal(d, ref), (h, w, kind)
                assert np.array_equal(mag, exact_mag(ref)), (h, w, kind)


def test_replicate_matches_torch_conv2d(oracle_mod, K_golden):
    torch = pytest.importorskip("torch")
    import torch.nn.functional as F
    img = synth.rect_image(96, 80, 3)
    x = torch.from_numpy(img.astype(np.float64))[None, None]
    xp = F.pad(x, (2, 2, 2, 2), mode="replicate")
    wt = torch.from_numpy(K_golden.astype(np.float64))[:, None]
    ref = F.conv2d(xp, wt)[0].numpy()               # conv2d is a correlation
    _, d = oracle_mod.sobel_u8(img)
    assert np.array_equal(d, ref.astype(np.int64))


def test_valid_matches_scipy_signal(oracle_mod, K_golden):
    img = synth.rect_image(40, 57, 9)
    mag, d = oracle_mod.sobel_u8(img, border=oracle_mod.VALID)
    I = img.astype(np.int64)
    ref = np.stack([sps.correlate2d(I, K_golden[k], mode="valid") for k in range(4)])
    assert np.array_equal(d, ref)
    mag_r, d_r = oracle_mod.sobel_u8(img)
    assert np.array_equal(d, d_r[:, 2:-2, 2:-2])
    assert np.array_equal(mag, mag_r[2:-2, 2:-2])


def test_pitch_is_honoured(oracle_mod):
    img = synth.rect_image(37, 50, 4)
    view = synth.pitched(img, 64)
    m1, d1 = oracle_mod.sobel_u8(np.ascontiguousarray(img))
    m2, d2 = oracle_mod.sobel_u8(view)
    assert np.array_equal(m1, m2) and np.array_equal(d1, d2)


def test_points_match_full(oracle_mod):
    img = synth.field_image(120, 90, 2)
    mag, d = oracle_mod.sobel_u8(img)
    rng = np.random.default_rng(0)
    ys = rng.integers(0, 120, 500)
    xs = rng.integers(0, 90, 500)
    pm, pd = oracle_mod.sobel_u8_points(img, ys, xs)
    assert np.array_equal(pm, mag[ys, xs])
    assert np.array_equal(pd, d[:, ys, xs].T)


def test_rejects_bad_arguments(oracle_mod):
    img = np.zeros((4, 4), np.uint8)
    with pytest.raises(ValueError):
        oracle_mod.sobel_u8(img, border=oracle_mod.VALID)     # VALID needs >= 5x5
    with pytest.raises(ValueError):
        oracle_mod.sobel_u8(img, border=7)


# ----------------------------------------------------------------------------
# (c) closed forms
# ----------------------------------------------------------------------------

def test_constant_images_give_zero(oracle_mod):
    for v in (0, 1, 77, 255):
        img = np.full((23, 31), v, np.uint8)
        mag, d = oracle_mod.sobel_u8(img)
        assert not d.any() and not mag.any()


@pytest.mark.parametrize("alpha,beta", [(1, 0), (0, 1), (1, 1), (2, -1), (-1, 3), (3, 2)])
def test_ramp_closed_form(oracle_mod, alpha, beta):
    """I = alpha*x + beta*y + c.  Interior responses (hand-derived):
    Gx = 128 alpha, Gy = 128 beta, Gd = 96 (alpha + beta), Gdt = 96 (beta - alpha),
    because sum_j r_j (j - 2) = 8 for r = [-1,-2,0,2,1], the smoothing column sums
    to 16, and the first moment of each diagonal filter is 96."""
    h, w = 24, 24
    y, x = np.mgrid[0:h, 0:w]
    c = 100
    img = (alpha * x + beta * y + c).astype(np.int64)
    assert img.min() >= 0 and img.max() <= 255
    _, d = oracle_mod.sobel_u8(img.astype(np.uint8))
    inner = (slice(2, h - 2), slice(2, w - 2))
    assert np.all(d[0][inner] == 128 * alpha)
    assert np.all(d[1][inner] == 96 * (alpha + beta))
    assert np.all(d[2][inner] == 128 * beta)
    assert np.all(d[3][inner] == 96 * (beta - alpha))


def test_ramp_magnitudes(oracle_mod):
    # S = 34816 (alpha^2 + beta^2): sqrt(34816) = 186.59 -> 187; (1, 1) saturates.
    y, x = np.mgrid[0:16, 0:16]
    m1, _ = oracle_mod.sobel_u8((x + 10).astype(np.uint8))
    m2, _ = oracle_mod.sobel_u8((x + y + 10).astype(np.uint8))
    assert np.all(m1[2:-2, 2:-2] == 187)
    assert np.all(m2[2:-2, 2:-2] == 255)


@pytest.mark.parametrize("height", [1, 7, 255])
def test_vertical_step(oracle_mod, height):
    """Step of height h at column x0: Gx = 16h, 48h, 48h, 16h at x0-2..x0+1,
    Gd = 13h, 35h, 35h, 13h there, Gdt = -Gd, Gy = 0 (column suffix sums)."""
    h, w, x0 = 12, 20, 9
    img = np.zeros((h, w), np.uint8)
    img[:, x0:] = height
    _, d = oracle_mod.sobel_u8(img)
    row = 6
    gx = d[0, row, x0 - 3: x0 + 3]
    gd = d[1, row, x0 - 3: x0 + 3]
    assert list(gx) == [0, 16 * height, 48 * height, 48 * height, 16 * height, 0]
    assert list(gd) == [0, 13 * height, 35 * height, 35 * height, 13 * height, 0]
    assert np.array_equal(d[3], -d[1])
    assert not d[2].any()
    # horizontal step: the transpose
    _, dt = oracle_mod.sobel_u8(np.ascontiguousarray(img.T))
    assert np.array_equal(dt[2], d[0].T)
    assert not dt[0].any()


def test_diagonal_step_45(oracle_mod):
    tab = np.loadtxt(os.path.join(GOLDEN, "step45.txt"), dtype=np.int64, comments="#")
    hgt, s = 50, 30
    n = 40
    y, x = np.mgrid[0:n, 0:n]
    img = np.where(x + y >= s, hgt, 0).astype(np.uint8)
    _, d = oracle_mod.sobel_u8(img)
    expect = {int(r[0]): r[1:] for r in tab}
    for yy in range(3, n - 3):
        for xx in range(3, n - 3):
            dd = xx + yy - s
            e = expect.get(dd, np.zeros(4, np.int64)) * hgt
            assert list(d[:, yy, xx]) == list(e), (yy, xx)
    # the 135-degree step is the left-right mirror: Gd and Gdt swap, Gx negates
    img2 = np.ascontiguousarray(img[:, ::-1])
    _, d2 = oracle_mod.sobel_u8(img2)
    assert np.array_equal(d2[3], d[1][:, ::-1])
    assert np.array_equal(d2[1], d[3][:, ::-1])


def test_impulse_response(oracle_mod, K_golden):
    """An impulse V at (y0, x0) gives G_k(y0+dy, x0+dx) = V * K_k[2-dy][2-dx]
    (correlation), which equals -V * K_k[2+dy][2+dx] since every filter is
    antisymmetric under rot180."""
    for V in (1, 2, 255):
        img = np.zeros((15, 15), np.uint8)
        img[7, 7] = V
        mag, d = oracle_mod.sobel_u8(img)
        win = d[:, 5:10, 5:10]
        assert np.array_equal(win, V * K_golden[:, ::-1, ::-1])
        assert np.array_equal(win, -V * K_golden)
        mask = np.ones_like(d[0], bool)
        mask[5:10, 5:10] = False
        assert not d[:, mask].any()
    # V = 1: S = 0 at the centre, 272 at the 8 neighbours, 38/40 on the outer ring
    img = np.zeros((9, 9), np.uint8)
    img[4, 4] = 1
    mag, d = oracle_mod.sobel_u8(img)
    S = (d.astype(np.int64) ** 2).sum(0)[2:7, 2:7]
    assert S[2, 2] == 0
    assert S[1, 1] == S[1, 2] == S[2, 1] == 272
    assert S[0, 0] == 38 and S[0, 1] == 40 and S[0, 2] == 38
    assert mag[4, 4] == 0 and mag[3, 4] == 16 and mag[2, 2] == 6 and mag[2, 3] == 6
    # V = 2 at the neighbour: S = 1088 -> round(32.98) = 33 (floor would give 32)
    img[4, 4] = 2
    mag, _ = oracle_mod.sobel_u8(img)
    assert mag[4, 5] == 33


# ----------------------------------------------------------------------------
# (d) invariants
# ----------------------------------------------------------------------------

@pytest.fixture(scope="module")
def sample_img():
    return synth.rect_image(45, 38, 11)


def test_transpose_invariant(oracle_mod, sample_img):
    m, d = oracle_mod.sobel_u8(sample_img)
    mt, dt = oracle_mod.sobel_u8(np.ascontiguousarray(sample_img.T))
    assert np.array_equal(dt[0], d[2].T)
    assert np.array_equal(dt[2], d[0].T)
    assert np.array_equal(dt[1], d[1].T)
    assert np.array_equal(dt[3], -d[3].T)
    assert np.array_equal(mt, m.T)


def test_fliplr_invariant(oracle_mod, sample_img):
    m, d = oracle_mod.sobel_u8(sample_img)
    mf, df = oracle_mod.sobel_u8(np.ascontiguousarray(sample_img[:, ::-1]))
    assert np.array_equal(df[0], -d[0][:, ::-1])
    assert np.array_equal(df[2], d[2][:, ::-1])
    assert np.array_equal(df[1], d[3][:, ::-1])
    assert np.array_equal(df[3], d[1][:, ::-1])
    assert np.array_equal(mf, m[:, ::-1])


def test_rot180_and_dihedral_magnitude(oracle_mod, sample_img):
    m, d = oracle_mod.sobel_u8(sample_img)
    mr, dr = oracle_mod.sobel_u8(np.ascontiguousarray(np.rot90(sample_img, 2)))
    assert np.array_equal(dr, -np.rot90(d, 2, axes=(1, 2)))
    for k in range(4):
        for flip in (False, True):
            t = np.rot90(sample_img, k)
            t = t[:, ::-1] if flip else t
            mt, _ = oracle_mod.sobel_u8(np.ascontiguousarray(t))
            ref = np.rot90(m, k)
            ref = ref[:, ::-1] if flip else ref
            assert np.array_equal(mt, ref), (k, flip)


def test_linearity(oracle_mod):
    rng = np.random.default_rng(3)
    a = rng.integers(0, 128, size=(30, 26), dtype=np.uint8)
    b = rng.integers(0, 128, size=(30, 26), dtype=np.uint8)
    _, da = oracle_mod.sobel_u8(a)
    _, db = oracle_mod.sobel_u8(b)
    _, dab = oracle_mod.sobel_u8((a + b).astype(np.uint8))
    assert np.array_equal(dab, da + db)
    _, dc = oracle_mod.sobel_u8((a + 100).astype(np.uint8))
    assert np.array_equal(dc, da)


# ----------------------------------------------------------------------------
# (e) rounding of the uint8 magnitude
# ----------------------------------------------------------------------------

def test_round_sqrt_exhaustive(oracle_mod):
    for s in list(range(0, 70001)) + [599270400, 2**31 - 1, 10**12]:
        r = math.isqrt(s)
        want = r + (1 if s - r * r > r else 0)
        got = oracle_mod.round_sqrt(s)
        assert got == want, s


def test_saturation_threshold(oracle_mod):
    # (254.5)^2 = 64770.25, so S = 64770 -> 254 and S = 64771 -> 255.
    assert oracle_mod.round_sqrt(64770) == 254
    assert oracle_mod.round_sqrt(64771) == 255


# ----------------------------------------------------------------------------
# planted mistakes: the pins above must catch plausible errors in the tables
# ----------------------------------------------------------------------------

def _pins_pass(oracle_mod, K_golden, weights):
    """A compact rerun of the pin families with a (possibly wrong) weight table."""
    img = synth.rect_image(20, 18, 1)
    _, d = oracle_mod.sobel_u8(img, weights=weights)
    if not np.array_equal(d, scipy_dirs(img, K_golden)):
        return False
    y, x = np.mgrid[0:16, 0:16]
    _, dr = oracle_mod.sobel_u8((x + 2 * y + 10).astype(np.uint8), weights=weights)
    inner = (slice(2, -2), slice(2, -2))
    return (np.all(dr[0][inner] == 128) and np.all(dr[2][inner] == 256)
            and np.all(dr[1][inner] == 288) and np.all(dr[3][inner] == 96))


def test_planted_mistakes_are_caught(oracle_mod, K_golden):
    good = oracle_mod.weights()
    assert _pins_pass(oracle_mod, K_golden, good)
    mutants = []
    m = good.copy(); m[[0, 2]] = m[[2, 0]]; mutants.append(m)             # swapped planes
    m = good.copy(); m[3] = -m[3]; mutants.append(m)                       # wrong sign
    m = good.copy(); m[3] = m[3].T; mutants.append(m)                      # transposed filter
    m = good.copy(); m[0, 2, 1] = 0; mutants.append(m)                     # dropped term
    m = good.copy(); m[1] = np.roll(m[1], 1, axis=1); mutants.append(m)    # off-by-one column
    m = good.copy(); m[:, :, :] = m[:, ::-1, ::-1]; mutants.append(m)      # convolution, not correlation
    for i, mt in enumerate(mutants):
        assert not _pins_pass(oracle_mod, K_golden, mt), i
