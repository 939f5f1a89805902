"""Pins for the oracle's coefficient generators (CPU only).

Each test checks the oracle against something other than itself: closed forms,
an exact summation identity, a brute-force 2D Fourier integral, the far-field
constant of the fractional Laplacian, or a limit case.
"""
import math

import mpmath
import numpy as np
import pytest

from oracle import coeffs as C

ALPHAS = [1.1, 1.5, 1.9]


# ----------------------------------------------------------------- 1D a_k
@pytest.mark.parametrize("alpha", ALPHAS)
def test_riesz_partial_sums_closed_form(alpha):
    """a_0 + 2 sum_{k=1..K} a_k = 2(-1)^K Gamma(alpha) / (Gamma(alpha/2-K) Gamma(alpha/2+K+1)):
    Pascal's rule on a_k = (-1)^k binom(alpha, alpha/2+k) telescopes the sum."""
    a = C.riesz_coeffs(alpha, 60)
    b = alpha / 2
    for K in (1, 2, 5, 17, 59):
        lhs = a[0] + 2.0 * a[1:K + 1].sum()
        with mpmath.workdps(30):
            rhs = 2 * (-1) ** K * mpmath.gamma(alpha) * mpmath.rgamma(b - K) * mpmath.rgamma(b + K + 1)
        assert abs(lhs - float(rhs)) <= 2e-14, (K, lhs, float(rhs))


@pytest.mark.parametrize("alpha", ALPHAS)
def test_riesz_symbol_at_pi(alpha):
    """sum_k a_k (-1)^k e^{ik pi} = (4 sin^2(pi/2))^(alpha/2) = 2^alpha."""
    a = C.riesz_coeffs(alpha, 4096)
    k = np.arange(4096)
    # the alternating series converges like k^(-1-alpha); average two consecutive partial sums
    s = a[0] + 2.0 * np.cumsum((a * (-1.0) ** k)[1:])
    est = 0.5 * (s[-1] + s[-2])
    assert abs(est - 2.0 ** alpha) < 1e-9


@pytest.mark.parametrize("alpha", ALPHAS)
def test_riesz_far_field(alpha):
    """a_k k^(1+alpha) -> -Gamma(alpha+1) sin(pi alpha/2) / pi."""
    a = C.riesz_coeffs(alpha, 4096)
    lim = -math.gamma(alpha + 1) * math.sin(math.pi * alpha / 2) / math.pi
    assert abs(a[4000] * 4000 ** (1 + alpha) / lim - 1.0) < 1e-3


def test_riesz_alpha2_is_three_point_laplacian():
    a = C.riesz_coeffs(2.0, 6)
    np.testing.assert_allclose(a, [2.0, -1.0, 0, 0, 0, 0], atol=1e-15)


@pytest.mark.parametrize("alpha", ALPHAS)
def test_riesz_recurrence_matches(alpha):
    """Gamma(z+1) = z Gamma(z) turns the closed form into a_{k+1} = a_k (k - a/2)/(k + a/2 + 1)."""
    a = C.riesz_coeffs(alpha, 4096)
    r = np.empty_like(a)
    r[0] = math.gamma(alpha + 1) / math.gamma(alpha / 2 + 1) ** 2
    for k in range(4095):
        r[k + 1] = r[k] * (k - alpha / 2) / (k + alpha / 2 + 1)
    np.testing.assert_allclose(r, a, rtol=5e-13, atol=0)


@pytest.mark.parametrize("alpha", ALPHAS + [1.999])
def test_subordination_quadrature_reproduces_1d(alpha):
    """The quadrature used for a_ij, applied to the 1D symbol, gives the closed form a_k."""
    a = C.riesz_coeffs(alpha, 4096)
    q = C.riesz_coeffs_quadrature(alpha, 4096)
    rel = np.abs(q - a) / np.abs(a)
    assert rel[:200].max() < 1e-14
    assert rel.max() < 5e-13      # scipy's ive loses ~1e-13 at orders ~1e3


# ----------------------------------------------------------------- 2D a_ij
def _bruteforce_2d(alpha, i, j, dps=18):
    """(1/pi^2) int_[0,pi]^2 s^(alpha/2) cos(i eta) cos(j xi): the defining 2D Fourier
    integral (the symbol is even), by nested tanh-sinh quadrature in polar
    coordinates centred on the non-smooth point at the origin."""
    with mpmath.workdps(dps):
        b = mpmath.mpf(alpha) / 2
        pi = mpmath.pi

        def f(eta, xi):
            s = 4 * mpmath.sin(eta / 2) ** 2 + 4 * mpmath.sin(xi / 2) ** 2
            return s ** b * mpmath.cos(i * eta) * mpmath.cos(j * xi)

        def lower(th):
            c, s = mpmath.cos(th), mpmath.sin(th)
            return mpmath.quad(lambda r: f(r * c, r * s) * r, [0, pi / c])

        def upper(th):
            c, s = mpmath.cos(th), mpmath.sin(th)
            return mpmath.quad(lambda r: f(r * c, r * s) * r, [0, pi / s])

        return float((mpmath.quad(lower, [0, pi / 4]) + mpmath.quad(upper, [pi / 4, pi / 2])) / pi ** 2)


@pytest.mark.parametrize("alpha,ij", [(1.5, (0, 0)), (1.5, (1, 0)), (1.5, (1, 1)), (1.5, (3, 2)),
                                      (1.1, (0, 0)), (1.1, (2, 1)), (1.9, (0, 0)), (1.9, (1, 0))])
def test_2d_coeffs_vs_bruteforce_integral(alpha, ij):
    a = C.laplacian_coeffs(alpha, 8)
    ref = _bruteforce_2d(alpha, *ij)
    assert abs(a[ij] - ref) <= 1e-13 * abs(ref), (a[ij], ref)


@pytest.mark.parametrize("alpha", ALPHAS)
def test_2d_symbol_at_corner(alpha):
    """sum_{i,j in Z} a_ij e^{i(i pi + j pi)} = (4 + 4)^(alpha/2)."""
    n = 1024
    a = C.laplacian_coeffs(alpha, n)
    w = np.where(np.arange(n) == 0, 1.0, 2.0) * (-1.0) ** np.arange(n)
    w[-1] *= 0.5          # mean of the last two partial sums of the alternating series
    assert abs(w @ a @ w - 8.0 ** (alpha / 2)) < 1e-12


def _far_constant(alpha, d):
    """C_{d,alpha} of the fractional Laplacian's definition (section "Introduction")."""
    return 2 ** alpha * math.gamma((alpha + d) / 2) / (math.pi ** (d / 2) * abs(math.gamma(-alpha / 2)))


@pytest.mark.parametrize("alpha", ALPHAS)
def test_2d_row_sums_give_1d_coeffs(alpha):
    """Setting xi = 0 in the symbol: sum_{j in Z} a_ij = a_i (the 1D coefficient).  The table
    stops at |j| < n; the missing tail is estimated from the far field a ~ -C |k|^(-2-alpha)."""
    n = 2048
    a = C.laplacian_coeffs(alpha, n)
    a1 = C.riesz_coeffs(alpha, n)
    w = np.where(np.arange(n) == 0, 1.0, 2.0)
    rows = a @ w
    c2 = _far_constant(alpha, 2)
    j = np.arange(n, 400000, dtype=np.float64)
    for i in (0, 1, 2, 5, 20):
        tail = -2.0 * c2 * (np.sum((i * i + j * j) ** (-1 - alpha / 2))
                            + (400000 - 0.5) ** (-1 - alpha) / (1 + alpha))
        err = rows[i] + tail - a1[i]
        assert abs(err) < 0.01 * abs(tail) + 1e-14, (i, err, tail)


@pytest.mark.parametrize("alpha", ALPHAS)
def test_2d_far_field_constant(alpha):
    """a_ij |k|^(2+alpha) -> -C_{2,alpha} (the kernel constant of the fractional Laplacian)."""
    a = C.laplacian_coeffs(alpha, 401)
    c2 = _far_constant(alpha, 2)
    for (i, j) in [(400, 0), (300, 200), (283, 283)]:
        r = math.hypot(i, j)
        assert abs(a[i, j] * r ** (2 + alpha) / (-c2) - 1.0) < 2e-3


@pytest.mark.parametrize("alpha", ALPHAS)
def test_2d_symmetry_and_signs(alpha):
    a = C.laplacian_coeffs(alpha, 300)
    assert np.array_equal(a, a.T)
    assert a[0, 0] > 0
    off = a.copy()
    off[0, 0] = -1.0
    assert (off < 0).all()


def test_2d_alpha_near_two_is_five_point():
    a = C.laplacian_coeffs(1.9999, 16)
    assert abs(a[0, 0] - 4.0) < 5e-3
    assert abs(a[1, 0] + 1.0) < 5e-3
    off = a.copy()
    off[0, 0] = off[1, 0] = off[0, 1] = 0.0
    assert np.abs(off).max() < 5e-3
