"""Pins for the oracle's real-valued path (forward magnitude and its adjoint).

The forward is pinned to torch's conv2d after padding (a library routine:
replicate, zero, or a reflect-101 gather whose indices come from numpy's
'reflect' pad, which also covers images smaller than the pad) and to the
oracle's own integer path on integer images.  The adjoint is pinned to
torch's reverse-mode autograd through that same library forward (fp64, safe
square root) and to central finite differences.
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
