"""Generalised weights (Sec. 3.2, Eq. (sobel5_param)) on the CPU: the
library's family builder, weight validation, and the oracle pinned for
non-default weights by closed forms derived by hand."""
from fractions import Fraction

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
api = pytest.importorskip("paper_2305_00515_amd.api")

# (a, b, n, m) with integer a, a*b, a*n, a*m, a*n*b, a*m*b
FAMILIES = [(1, 2, 4, 6), (1, 1, 2, 3), (2, Fraction(3, 2), 2, 3), (1, 3, 5, 10), (3, Fraction(1, 3), 3, 6)]


def printed_family(a, b, n, m):
    """K_x, K_d, K_y, K_dt typed from the matrices printed in Eq. (sobel5_param)
    (K_y and K_dt from their own printed matrices, not derived)."""
    F = lambda v: Fraction(v)
    a, b, n, m = F(a), F(b), F(n), F(m)
    kx = [[-1, -b, 0, b, 1], [-n, -n * b, 0, n * b, n], [-m, -m * b, 0, m * b, m],
          [-n, -n * b, 0, n * b, n], [-1, -b, 0, b, 1]]
    ky = [[-1, -n, -m, -n, -1], [-b, -n * b, -m * b, -n * b, -b], [0] * 5,
          [b, n * b, m * b, n * b, b], [1, n, m, n, 1]]
    kd = [[-m, -n, -1, -b, 0], [-n, -m * b, -n * b, 0, b], [-1, -n * b, 0, n * b, 1],
          [-b, 0, n * b, m * b, n], [0, b, 1, n, m]]
    kdt = [[0, -b, -1, -n, -m], [b, 0, -n * b, -m * b, -n], [1, n * b, 0, -n * b, -1],
           [n, m * b, n * b, 0, -b], [m, n, 1, b, 0]]
    out = np.zeros((4, 5, 5), dtype=np.int64)
    for k, K in enumerate((kx, kd, ky, kdt)):
        for i in range(5):
            for j in range(5):
                v = a * F(K[i][j])
                assert v.denominator == 1
                out[k, i, j] = int(v)
    return out


@pytest.mark.parametrize("abnm", FAMILIES)
def test_family_builder_matches_printed_matrices(abnm):
    w = api.family_weights(*api.family_products(*abnm))
    assert np.array_equal(w, printed_family(*abnm))


def test_family_at_defaults_is_eq_sobel5_1():
    assert np.array_equal(api.family_weights(1, 2, 4, 6, 8, 12), oracle.weights())


def test_family_products_rejects_non_integer_weights():
    with pytest.raises(ValueError):
        api.family_products(1, Fraction(1, 2), 2, 3)      # a*b = 1/2
    with pytest.raises(api.SobelError):
        api.family_weights(1, 2, 4, 6, 9, 12)             # a*n*b inconsistent
    with pytest.raises(api.SobelError):
        api.family_weights(0, 2, 4, 6, 8, 12)


def test_validate_weights():
    w = api.family_weights(1, 2, 4, 6, 8, 12)
    api.validate_weights(w, api.DIR_S32)
    api.validate_weights(w, api.DIR_S16)                  # sum |k| = 96 <= 128
    bad = w.copy()
    bad[1, 0, 0] += 1                                     # breaks the half-turn antisymmetry
    with pytest.raises(api.SobelError):
        api.validate_weights(bad)
    big = api.family_weights(*api.family_products(1, 3, 5, 10))   # sum |k| = 168
    api.validate_weights(big, api.DIR_S32)
    with pytest.raises(api.SobelError):
        api.validate_weights(big, api.DIR_S16)
    huge = big * 200                                      # sum |k| > 32768
    with pytest.raises(api.SobelError):
        api.validate_weights(huge, api.DIR_S32)


@pytest.mark.parametrize("abnm", FAMILIES)
def test_oracle_ramp_closed_form(abnm):
    """I = alpha*x + beta*y: away from the border
    Gx = a*alpha*(2+2n+m)*(4+2b), Gy = a*beta*(2+2n+m)*(4+2b),
    Gd = (alpha+beta)*(4a + 4am + 6an + 2ab + 2amb + 2anb), Gdt = (beta-alpha)*(same)
    (sums of the printed taps times their offsets, worked out by hand)."""
    a, ab, an, am, anb, amb = api.family_products(*abnm)
    w = api.family_weights(a, ab, an, am, anb, amb)
    cx = (2 * a + 2 * an + am) * (4 + 2 * Fraction(ab, a))     # a(2+2n+m)(4+2b)
    cd = 4 * a + 4 * am + 6 * an + 2 * ab + 2 * amb + 2 * anb
    for alpha, beta in ((1, 0), (0, 1), (1, 1), (2, 1)):
        y, x = np.mgrid[0:24, 0:30]
        img = (alpha * x + beta * y).astype(np.uint8)
        _, d = oracle.sobel_u8(img, weights=w)
        inner = (slice(2, -2), slice(2, -2))
        assert (d[0][inner] == alpha * cx).all() and (d[2][inner] == beta * cx).all()
        assert (d[1][inner] == (alpha + beta) * cd).all() and (d[3][inner] == (beta - alpha) * cd).all()


@pytest.mark.parametrize("abnm", FAMILIES[1:])
def test_oracle_impulse_response(abnm):
    """A single pixel V at (y0, x0): G_k(y0+dy, x0+dx) = -V * k[2+dy][2+dx]
    (the correlation sees the impulse at offset (-dy, -dx); half-turn
    antisymmetry flips the sign)."""
    w = api.family_weights(*api.family_products(*abnm))
    img = np.zeros((15, 17), np.uint8)
    img[7, 8] = 3
    _, d = oracle.sobel_u8(img, weights=w)
    for k in range(4):
        assert np.array_equal(d[k][5:10, 6:11], -3 * w[k])
