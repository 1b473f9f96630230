"""GPU checks of the fp32 forward/adjoint against the fp64 oracle and FD.

Tolerances (a reading of "rel. tol 1e-5" for an fp32 path, see the design
notes): forward |M - M_ref| <= 1e-5 * max(M_ref, s_f) where s_f is the
per-pixel scale max_k sum_t |K_k[t] x_t|; gradient |g - g_ref| <= 1e-5 * A
where A is the per-pixel sum of |terms| of the adjoint's sum, plus a
normwise bound ||g - g_ref|| <= 1e-5 ||g_ref||.  Plain elementwise relative
error is not meaningful where the adjoint's terms cancel.
"""
import numpy as np
import pytest

from paper_2305_00515_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


def f32_batch(b, h, w, seed):
    return np.stack([synth.rect_image(h, w, seed + i) for i in range(b)]).astype(np.float32) / np.float32(255.0)


def check_fwd(oracle_mod, x, M, border):
    Mr, _ = oracle_mod.sobel_f64_fwd(x.astype(np.float64), border)
    s = oracle_mod.sobel_f64_fwd_scale(x.astype(np.float64), border)
    err = np.abs(M.astype(np.float64) - Mr)
    assert np.all(err <= TOL * np.maximum(Mr, s) + 1e-30), float((err / np.maximum(Mr, s).clip(1e-30)).max())
    assert np.all(M[Mr == 0] == 0)          # flat windows give exactly 0


def check_bwd(oracle_mod, x, g, dx, border):
    xd, gd = x.astype(np.float64), g.astype(np.float64)
    ref = oracle_mod.sobel_f64_bwd(xd, gd, border)
    A = oracle_mod.sobel_f64_bwd_scale(xd, gd, border)
    err = np.abs(dx.astype(np.float64) - ref)
    assert np.all(err <= TOL * A + 1e-30), float((err / A.clip(1e-30)).max())
    assert np.linalg.norm(err) <= TOL * np.linalg.norm(ref)


@pytest.mark.parametrize("border", [0, 1, 2, 3])
@pytest.mark.parametrize("shape", [(1, 5, 5), (2, 37, 45), (1, 64, 64), (3, 100, 33), (1, 1, 9), (1, 7, 1),
                                   (1, 2, 3), (2, 3, 4), (1, 300, 130), (1, 70, 260),
                                   (1, 12, 116), (1, 12, 117), (1, 10, 118), (1, 9, 119), (2, 9, 233),
                                   (1, 8, 234), (1, 7, 232)])
def test_forward_backward_small(oracle_mod, sobel_lib, gpu, border, shape):
    """Every border rule, on shapes that span several column strips and row
    chunks (130, 260 columns; 300 rows), on widths around a multiple of the
    adjoint's 116-column strips (W mod 116 in {0, 1, 2, 3}: under
    REFLECT101 the mirrors W-2, W-3 of the padded columns W, W+1 then lie in
    the strip before the last one), and on images so small that the
    reflection repeats (1 to 4 rows or columns)."""
    b, h, w = shape
    if border == 1 and min(h, w) < 5:
        pytest.skip("VALID needs 5x5")
    x = f32_batch(b, h, w, 11 * h + w)
    xt = torch.from_numpy(x).to(gpu)
    M = sobel_lib.sobel4x5_f32_fwd(xt, border)
    torch.cuda.synchronize()
    check_fwd(oracle_mod, x, M.cpu().numpy(), border)
    g = np.random.default_rng(h).standard_normal(M.shape).astype(np.float32)
    dx = sobel_lib.sobel4x5_f32_bwd(xt, torch.from_numpy(g).to(gpu), border)
    torch.cuda.synchronize()
    check_bwd(oracle_mod, x, g, dx.cpu().numpy(), border)


def test_noninteger_inputs(oracle_mod, sobel_lib, gpu):
    rng = np.random.default_rng(9)
    x = rng.random((2, 70, 90)).astype(np.float32)
    x[:, 10:30, 10:40] = np.float32(0.3)      # flat patch of a non-dyadic value
    xt = torch.from_numpy(x).to(gpu)
    M = sobel_lib.sobel4x5_f32_fwd(xt)
    torch.cuda.synchronize()
    check_fwd(oracle_mod, x, M.cpu().numpy(), 0)
    g = np.full(M.shape, 1.0 / M.numel(), np.float32)
    dx = sobel_lib.sobel4x5_f32_bwd(xt, torch.from_numpy(g).to(gpu))
    torch.cuda.synchronize()
    check_bwd(oracle_mod, x, g, dx.cpu().numpy(), 0)


def test_tiny_magnitudes(oracle_mod, sobel_lib, gpu):
    """Images scaled by 2^-50 (exact) put S = M^2 between about 2^-116 and
    2^-84, on both sides of 2^-100 where the adjoint's reciprocal square root
    switches to its scaled form; every S stays a normal fp32 number."""
    x = f32_batch(2, 40, 70, 31) * np.float32(2.0 ** -50)
    xt = torch.from_numpy(x).to(gpu)
    M = sobel_lib.sobel4x5_f32_fwd(xt)
    torch.cuda.synchronize()
    Mh = M.cpu().numpy().astype(np.float64)
    check_fwd(oracle_mod, x, Mh.astype(np.float32), 0)
    S = Mh[Mh > 0] ** 2
    assert S.min() < 2.0 ** -100 < S.max()
    g = np.random.default_rng(4).standard_normal(M.shape).astype(np.float32)
    dx = sobel_lib.sobel4x5_f32_bwd(xt, torch.from_numpy(g).to(gpu))
    torch.cuda.synchronize()
    check_bwd(oracle_mod, x, g, dx.cpu().numpy(), 0)


@pytest.mark.parametrize("border", [0, 3])
def test_autograd_function(oracle_mod, sobel_lib, gpu, border):
    from paper_2305_00515_amd import sobel4x5_magnitude
    x = f32_batch(2, 48, 40, 5)
    xt = torch.from_numpy(x).to(gpu).requires_grad_(True)
    loss = sobel4x5_magnitude(xt, border).mean()
    loss.backward()
    g = np.full((2, 48, 40), 1.0 / x.size, np.float32)
    check_bwd(oracle_mod, x, g, xt.grad.cpu().numpy(), border)


def test_config4_fd_and_oracle_gradient(oracle_mod, sobel_lib, gpu):
    """32 x 1024^2, loss = mean(M): the GPU gradient at 64 random pixels (8 on
    the border) against central differences of the fp64 oracle (local: only
    the 5x5 outputs around the pixel change), Richardson-extrapolated from
    h = 1e-3; and the whole forward and gradient of all 32 images against the
    oracle's."""
    from paper_2305_00515_amd import sobel4x5_magnitude
    B, H, W = 32, 1024, 1024
    x = f32_batch(B, H, W, 2000)
    xt = torch.from_numpy(x).to(gpu).requires_grad_(True)
    loss = sobel4x5_magnitude(xt).mean()
    loss.backward()
    grad = xt.grad.cpu().numpy()
    n = B * H * W
    rng = np.random.default_rng(64)
    pts = [(int(rng.integers(B)), int(rng.integers(H)), int(rng.integers(W))) for _ in range(56)]
    pts += [(int(rng.integers(B)), 0, int(rng.integers(W))), (int(rng.integers(B)), H - 1, 5),
            (0, 0, 0), (1, H - 1, W - 1), (2, 17, 0), (3, 511, W - 1), (4, 0, W - 1), (5, H - 1, 0)]
    for (b, py, px) in pts:
        y0, y1 = max(0, py - 6), min(H, py + 7)
        x0, x1 = max(0, px - 6), min(W, px + 7)
        patch = x[b, y0:y1, x0:x1].astype(np.float64)
        # outputs whose window touches (py, px): rows/cols within 2 (clamped) of it
        oy0, oy1 = max(0, py - 2), min(H, py + 3)
        ox0, ox1 = max(0, px - 2), min(W, px + 3)
        # the patch must contain every clamped tap of those outputs: edge-touching
        # patches keep the true image border, so replicate reads agree
        assert (y0 == 0 or oy0 - 2 >= y0) and (y1 == H or oy1 + 2 <= y1)

        def local_loss(z):
            M, _ = oracle_mod.sobel_f64_fwd(z)
            return M[0, oy0 - y0:oy1 - y0, ox0 - x0:ox1 - x0].sum() / n

        def fd(hh):
            zp = patch.copy(); zp[py - y0, px - x0] += hh
            zm = patch.copy(); zm[py - y0, px - x0] -= hh
            return (local_loss(zp) - local_loss(zm)) / (2 * hh)

        h0 = 1e-3
        rich = (4 * fd(h0 / 2) - fd(h0)) / 3
        g1 = np.zeros((1,) + patch.shape)
        g1[0, oy0 - y0:oy1 - y0, ox0 - x0:ox1 - x0] = 1.0 / n
        A = oracle_mod.sobel_f64_bwd_scale(patch[None], g1)[0, py - y0, px - x0]
        assert abs(grad[b, py, px] - rich) <= TOL * A + 1e-14, (b, py, px, grad[b, py, px], rich, A)
    # the whole forward and the whole gradient of every image against the
    # oracle, at the scaled tolerances
    M = sobel_lib.sobel4x5_f32_fwd(xt.detach())
    torch.cuda.synchronize()
    check_fwd(oracle_mod, x, M.cpu().numpy(), 0)
    g = np.full((B, H, W), 1.0 / n, np.float32)
    check_bwd(oracle_mod, x, g, grad, 0)
