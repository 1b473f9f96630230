"""Pins for the oracle's real-valued path (forward magnitude and its adjoint).

The forward is pinned to torch's conv2d after padding (a library routine:
replicate, zero, or a reflect-101 gather whose indices come from numpy's
'reflect' pad, which also covers images smaller than the pad) and to the
oracle's own integer path on integer images.  The adjoint is pinned to
torch's reverse-mode autograd through that same library forward (fp64, safe
square root), to central finite differences, and by the adjoint dot-product
identity against the forward's own linear responses.  The two tolerance
scales are pinned by exact closed forms (constant and impulse images).
"""
import numpy as np
import pytest

from paper_2305_00515_amd import synth

torch = pytest.importorskip("torch")
import torch.nn.functional as F  # noqa: E402


def torch_forward(x, K, border):
    """Library forward: pad + conv2d (a correlation) + safe sqrt."""
    t = x[:, None]
    if border == 0:
        t = F.pad(t, (2, 2, 2, 2), mode="replicate")
    elif border == 2:
        t = F.pad(t, (2, 2, 2, 2), mode="constant", value=0.0)
    elif border == 3:
        ri = torch.from_numpy(np.pad(np.arange(x.shape[1]), 2, mode="reflect"))
        ci = torch.from_numpy(np.pad(np.arange(x.shape[2]), 2, mode="reflect"))
        t = t[:, :, ri][:, :, :, ci]
    wt = torch.from_numpy(K.astype(np.float64))[:, None]
    G = F.conv2d(t, wt)
    S = (G * G).sum(1)
    pos = S > 0
    safe = torch.where(pos, S, torch.ones_like(S))
    return torch.where(pos, torch.sqrt(safe), torch.zeros_like(S)), G


@pytest.mark.parametrize("border", [0, 1, 2, 3])
def test_f64_forward_matches_torch(oracle_mod, border):
    rng = np.random.default_rng(1)
    x = rng.random((2, 19, 23))
    M, D = oracle_mod.sobel_f64_fwd(x, border, want_dir=True)
    Mt, Gt = torch_forward(torch.from_numpy(x), oracle_mod.weights(), border)
    np.testing.assert_allclose(D, Gt.numpy(), rtol=0, atol=1e-12)
    np.testing.assert_allclose(M, Mt.numpy(), rtol=1e-14, atol=1e-12)


def test_f64_forward_equals_integer_path(oracle_mod):
    img = synth.rect_image(33, 41, 8)
    _, d = oracle_mod.sobel_u8(img)
    M, D = oracle_mod.sobel_f64_fwd(img.astype(np.float64), want_dir=True)
    assert np.array_equal(D[0], d.astype(np.float64))
    assert np.array_equal(M[0], np.sqrt((d.astype(np.float64) ** 2).sum(0)))


def test_f64_values_k_over_255_are_exact(oracle_mod):
    """Inputs k/255 rounded to fp32 are multiples of 2^-31 with |G| < 2^8, so
    every response is exact in fp64: scaling the integer responses by the
    per-pixel fp32 values reproduces them bit for bit."""
    img = synth.rect_image(28, 30, 2)
    x = (img.astype(np.float32) / np.float32(255.0)).astype(np.float64)
    _, D = oracle_mod.sobel_f64_fwd(x, want_dir=True)
    scaled = x * 2.0 ** 31
    assert np.array_equal(scaled, np.round(scaled))        # multiples of 2^-31
    _, Di = oracle_mod.sobel_f64_fwd(scaled, want_dir=True)
    assert np.array_equal(D * 2.0 ** 31, Di)


@pytest.mark.parametrize("border", [0, 1, 2, 3])
@pytest.mark.parametrize("shape", [(1, 9, 11), (2, 17, 13), (1, 5, 5), (1, 1, 7), (1, 3, 2), (1, 2, 4), (1, 4, 3)])
def test_f64_backward_matches_torch_autograd(oracle_mod, border, shape):
    b, h, w = shape
    if border == 1 and (h < 5 or w < 5):
        pytest.skip("VALID needs 5x5")
    rng = np.random.default_rng(h * 31 + w)
    x = rng.random(shape)
    x[:, : h // 2, : w // 2] = 0.25                 # a flat patch: M = 0 there
    M, _ = oracle_mod.sobel_f64_fwd(x, border)
    g = rng.standard_normal(M.shape)
    xt = torch.from_numpy(x).requires_grad_(True)
    Mt, _ = torch_forward(xt, oracle_mod.weights(), border)
    (Mt * torch.from_numpy(g)).sum().backward()
    dx = oracle_mod.sobel_f64_bwd(x, g, border)
    np.testing.assert_allclose(dx, xt.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_f64_backward_constant_image_is_zero(oracle_mod):
    x = np.full((1, 12, 14), 0.3)
    g = np.ones((1, 12, 14))
    dx = oracle_mod.sobel_f64_bwd(x, g)
    assert not dx.any()


def test_f64_backward_central_differences(oracle_mod):
    """Central FD with Richardson extrapolation on interior and border pixels,
    for loss = mean(M).  The remaining truncation term scales as h^4."""
    img = synth.rect_image(24, 20, 6)
    x = img.astype(np.float64)[None] / 255.0
    x += np.random.default_rng(0).random(x.shape) * 0.05     # no exactly flat windows
    n = x.size
    g = np.full((1, 24, 20), 1.0 / n)
    dx = oracle_mod.sobel_f64_bwd(x, g)

    def loss(z):
        return oracle_mod.sobel_f64_fwd(z)[0].sum() / n

    pts = [(0, 0), (0, 19), (23, 0), (23, 19), (1, 7), (12, 0), (12, 10), (5, 5), (22, 18)]
    for (py, px) in pts:
        def fd(hh):
            zp = x.copy(); zp[0, py, px] += hh
            zm = x.copy(); zm[0, py, px] -= hh
            return (loss(zp) - loss(zm)) / (2 * hh)
        h0 = 1e-4
        rich = (4 * fd(h0 / 2) - fd(h0)) / 3
        assert abs(rich - dx[0, py, px]) <= 1e-7 * max(1.0, abs(dx[0, py, px])), (py, px)


@pytest.mark.parametrize("border", [0, 1, 2, 3])
def test_error_scales_bound_the_results(oracle_mod, border):
    """The tolerance scales dominate the quantities they scale."""
    rng = np.random.default_rng(4)
    x = rng.random((2, 14, 17))
    M, D = oracle_mod.sobel_f64_fwd(x, border, want_dir=True)
    sf = oracle_mod.sobel_f64_fwd_scale(x, border)
    assert np.all(np.abs(D).max(axis=1) <= sf + 1e-12)
    g = rng.standard_normal(M.shape)
    dx = oracle_mod.sobel_f64_bwd(x, g, border)
    A = oracle_mod.sobel_f64_bwd_scale(x, g, border)
    assert np.all(np.abs(dx) <= A + 1e-12)
    assert np.all(A >= 0)
    # a constant image has no terms at all
    assert not oracle_mod.sobel_f64_bwd_scale(np.full((1, 8, 8), 0.7), np.ones((1, 8, 8))).any()


# ----------------------------------------------------------------------------
# Exact pins of the two tolerance scales.  The scales set how far an fp32
# result may sit from the fp64 oracle, so a mistake that inflates them (a sum
# over the four filters instead of the largest one, a tap counted twice, a
# missing absolute value, the filter applied transposed) would loosen every
# fp32 parity check.  Each pin is a closed form worked out from the printed
# matrices of Eq. (sobel5_1) (tests/golden/eq_sobel5_1.txt) for an input on
# which the definition collapses to one term.
# ----------------------------------------------------------------------------

import os  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden_weights():
    mats, cur, name = {}, [], None
    with open(os.path.join(GOLDEN, "eq_sobel5_1.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("["):
                if name:
                    mats[name] = np.array(cur, dtype=np.float64)
                name, cur = line[1:-1], []
            else:
                cur.append([float(v) for v in line.split()])
    mats[name] = np.array(cur, dtype=np.float64)
    return np.stack([mats[p] for p in ("Gx", "Gd", "Gy", "Gdt")])


@pytest.mark.parametrize("border", [0, 1, 3])
def test_fwd_scale_constant_image_is_96c(oracle_mod, border):
    """Every filter has sum |w| = 96, and a constant image c feeds c to every
    tap under REPLICATE, VALID and REFLECT101: the scale is exactly 96c."""
    K = golden_weights()
    assert np.all(np.abs(K).sum(axis=(1, 2)) == 96)
    x = np.full((2, 9, 12), 3.0)
    s = oracle_mod.sobel_f64_fwd_scale(x, border)
    assert np.all(s == 288.0)


def test_fwd_scale_zero_border_counts_only_taps_inside(oracle_mod):
    """Under ZERO a tap outside reads 0: at the corner pixel of a constant
    image only the taps (i, j) with i, j >= 2 read c, so the scale is c times
    the largest sum of |w| over that quarter of a filter."""
    K = golden_weights()
    x = np.full((1, 10, 10), 2.0)
    s = oracle_mod.sobel_f64_fwd_scale(x, 2)
    corner = 2.0 * np.abs(K[:, 2:, 2:]).sum(axis=(1, 2)).max()
    assert s[0, 0, 0] == corner
    assert np.all(s[0, 2:-2, 2:-2] == 192.0)


def test_fwd_scale_impulse_is_largest_single_tap(oracle_mod):
    """Impulse V at c: output q = c + (dy, dx) sees one nonzero tap, (2-dy,
    2-dx), so the scale is V * max_k |K_k[2-dy][2-dx]| and 0 farther away."""
    K = golden_weights()
    V, c = 5.0, 7
    x = np.zeros((1, 15, 15))
    x[0, c, c] = V
    s = oracle_mod.sobel_f64_fwd_scale(x)[0]
    want = np.zeros((15, 15))
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            want[c + dy, c + dx] = V * np.abs(K[:, 2 - dy, 2 - dx]).max()
    assert np.array_equal(s, want)
    # planted mistakes this pin catches: a sum over the filters, a doubled tap
    summed = np.zeros_like(want)
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            summed[c + dy, c + dx] = V * np.abs(K[:, 2 - dy, 2 - dx]).sum()
    assert not np.array_equal(summed, s)
    assert not np.array_equal(2 * s, s)


# (dy, dx, catches_signed, catches_transposed): whether the tap of that
# offset makes the two planted mistakes visible (they need mixed signs among
# the G_k, and unequal weights on |K_x| and |K_y| = |K_x|^T respectively)
@pytest.mark.parametrize("dy,dx,sgn,trn", [(1, -2, True, True), (-1, 1, True, False), (2, 2, False, False)])
def test_bwd_scale_single_output_closed_form(oracle_mod, dy, dx, sgn, trn):
    """Impulse image (V at c) and dL/dM nonzero (g) at one output q0 = c +
    (dy, dx) only.  Then G_k(q0) = V K_k[2-dy][2-dx], u_k = g G_k / M, and
    the scale at q0 + (i-2, j-2) is sum_k |K_k[i][j]| |u_k|; 0 elsewhere."""
    K = golden_weights()
    V, c, g0 = 3.0, 8, -0.75
    H = W = 17
    x = np.zeros((1, H, W))
    x[0, c, c] = V
    g = np.zeros((1, H, W))
    q = (c + dy, c + dx)
    g[0, q[0], q[1]] = g0
    A = oracle_mod.sobel_f64_bwd_scale(x, g)[0]
    G = V * K[:, 2 - dy, 2 - dx]
    M = np.sqrt((G * G).sum())
    u = g0 * G / M
    want = np.zeros((H, W))
    for i in range(5):
        for j in range(5):
            want[q[0] + i - 2, q[1] + j - 2] = (np.abs(K[:, i, j]) * np.abs(u)).sum()
    np.testing.assert_allclose(A, want, rtol=1e-14, atol=0)
    # planted mistakes this pin catches: signed u, transposed filters
    signed = np.zeros((H, W))
    transposed = np.zeros((H, W))
    for i in range(5):
        for j in range(5):
            signed[q[0] + i - 2, q[1] + j - 2] = (np.abs(K[:, i, j]) * u).sum()
            transposed[q[0] + i - 2, q[1] + j - 2] = (np.abs(K[:, j, i]) * np.abs(u)).sum()
    assert (np.abs(signed - A).max() > 1e-3 * A.max()) == sgn
    assert (np.abs(transposed - A).max() > 1e-3 * A.max()) == trn


@pytest.mark.parametrize("border", [0, 1, 2, 3])
def test_adjoint_dot_product(oracle_mod, border):
    """<J d, v> = <d, J^T v> for the magnitude map linearised at x.  The
    responses are linear in the image under every border rule, so J d is
    exactly sum_k G_k[x] G_k[d] / M[x], formed from the oracle's own forward
    planes (0 where M = 0, the subgradient the adjoint takes: the corners
    under REFLECT101, whose mirrored window is symmetric about its centre);
    J^T v is the oracle's adjoint."""
    rng = np.random.default_rng(17 + border)
    x = rng.random((2, 13, 16))
    d = rng.standard_normal(x.shape)
    M, Gx = oracle_mod.sobel_f64_fwd(x, border, want_dir=True)
    _, Gd = oracle_mod.sobel_f64_fwd(d, border, want_dir=True)
    assert (M > 0).mean() > 0.95
    Jd = np.where(M > 0, (Gx * Gd).sum(axis=1) / np.where(M > 0, M, 1.0), 0.0)
    v = rng.standard_normal(M.shape)
    JTv = oracle_mod.sobel_f64_bwd(x, v, border)
    lhs, rhs = float((Jd * v).sum()), float((d * JTv).sum())
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(Jd * v).sum() + np.abs(d * JTv).sum())
