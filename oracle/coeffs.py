"""Oracle: coefficients of the discrete fractional operators (test infrastructure).

Everything here is plain FP64 (mpmath only for the printed Gamma closed form) and
is written from the paper's definitions, section "Construction of S-ADI scheme":

* 1D fractional centred-difference coefficients a_k (closed form printed next to
  the definition of the discrete Riesz operators).
* 2D coefficients a_ij of the discrete fractional Laplacian L_h^alpha, defined as
  the Fourier coefficients of the symbol (4 sin^2(eta/2) + 4 sin^2(xi/2))^(alpha/2).

The paper gives no way to evaluate a_ij.  Reading used here (exact identity, then
numerical quadrature):

    s^beta = beta / Gamma(1-beta) * int_0^inf (1 - exp(-t s)) t^(-1-beta) dt,  0<beta<1,

with s the symbol's base and beta = alpha/2.  Since
exp(-t(2-2cos eta)) = sum_k exp(-2t) I_k(2t) exp(i k eta), the Fourier coefficients of
exp(-t s) are e^{-4t} I_i(2t) I_j(2t) and

    a_ij = beta/Gamma(1-beta) * int_0^inf (delta_i0 delta_j0 - ive(i,2t) ive(j,2t)) t^(-1-beta) dt,

ive(k,x) = e^{-x} I_k(x).  The same identity with one factor gives the 1D a_k,
which the tests compare with the closed form to pin the quadrature.

Quadrature: t = e^s and the trapezoidal rule on the WHOLE real s-line (exponentially
convergent for this analytic integrand).  Nodes inside [S_LO, S_HI] are evaluated
directly; the infinitely many nodes outside are summed in closed form from the
small-t power series and the large-t asymptotic series of ive, so no truncation of
the s-range enters the result.

This module is test infrastructure: only tests, the smoke check and the CPU
baseline of the benchmark may import it.
"""
from __future__ import annotations

import math
import numpy as np
import mpmath
from scipy.special import ive as _scipy_ive
from scipy.special import gammaln

# quadrature parameters (s = log t)
S_LO = -16.0
S_HI = 40.0
DS = 0.125
_X_SCIPY_MAX = 2.0e8     # scipy's ive is used for x <= this, the asymptotic series above
_ASYM_TERMS = 16
_SERIES_DEG = 40         # degree of the small-t power series used for the low tail
_LOW_TAIL_ORDER = 12     # low-tail series only matters for i + j below this


# --------------------------------------------------------------------------
# 1D coefficients: closed form (Gamma functions), evaluated in 40-digit mpmath
# --------------------------------------------------------------------------
def riesz_coeffs(alpha: float, n: int) -> np.ndarray:
    """a_k^(alpha), k = 0..n-1, from the printed closed form
    (-1)^k Gamma(alpha+1) / (Gamma(alpha/2 - k + 1) Gamma(alpha/2 + k + 1))."""
    with mpmath.workdps(40):
        al = mpmath.mpf(alpha)
        g = mpmath.gamma(al + 1)
        out = np.empty(n)
        for k in range(n):
            # 1/Gamma(z) is entire: rgamma handles the poles at non-positive integers
            v = (-1) ** k * g * mpmath.rgamma(al / 2 - k + 1) * mpmath.rgamma(al / 2 + k + 1)
            out[k] = float(v)
    return out


# --------------------------------------------------------------------------
# exponentially scaled modified Bessel functions ive(k, x) = e^-x I_k(x)
# --------------------------------------------------------------------------
def _ive_asym(k: np.ndarray, x: float) -> np.ndarray:
    """Large-x asymptotic series of e^-x I_k(x) (Hankel): accurate when x >> k^2."""
    mu = 4.0 * np.asarray(k, dtype=np.float64) ** 2
    term = np.ones_like(mu)
    acc = np.ones_like(mu)
    for m in range(1, _ASYM_TERMS + 1):
        term = term * (-(mu - (2 * m - 1) ** 2) / (m * 8.0 * x))
        acc = acc + term
    return acc / math.sqrt(2.0 * math.pi * x)


def ive(k, x: float) -> np.ndarray:
    k = np.asarray(k)
    if x <= _X_SCIPY_MAX:
        return _scipy_ive(k, x)
    return _ive_asym(k, x)


def _check_asym_range(kmax: int) -> None:
    # the asymptotic branch is only used where (k^2 / 2x) is small
    assert kmax ** 2 / (2 * _X_SCIPY_MAX) < 0.2, "orders too large for the asymptotic branch"


# --------------------------------------------------------------------------
# closed-form sums over the nodes outside [S_LO, S_HI]
# --------------------------------------------------------------------------
def _geom_tail(rate: float, s_edge: float, direction: int) -> float:
    """sum_{q>=1} DS * exp(rate * (s_edge + direction*q*DS)) for the decaying direction."""
    x = -direction * rate * DS          # > 0 for the decaying direction
    assert x > 0.0
    # r / (1 - r) with r = e^-x, written without cancellation
    return DS * math.exp(rate * s_edge) / math.expm1(x)


def _series_coeffs_exp_i(k: int, deg: int) -> np.ndarray:
    """Power-series coefficients (in t) of I_k(2t) up to t^deg (exact rationals in fp64)."""
    c = np.zeros(deg + 1)
    m = 0
    while 2 * m + k <= deg:
        c[2 * m + k] = math.exp(-gammaln(m + 1) - gammaln(m + k + 1))
        m += 1
    return c


def _series_coeffs_exp(a: float, deg: int) -> np.ndarray:
    """Power-series coefficients of exp(-a t)."""
    return np.array([(-a) ** p / math.factorial(p) for p in range(deg + 1)])


def _low_tail_2d(i: int, j: int, beta: float) -> float:
    """Trapezoid sum over nodes s < S_LO of ive(i,2t) ive(j,2t) t^-beta (t = e^s)."""
    deg = _SERIES_DEG
    f = np.convolve(np.convolve(_series_coeffs_exp(4.0, deg), _series_coeffs_exp_i(i, deg))[: deg + 1],
                    _series_coeffs_exp_i(j, deg))[: deg + 1]
    tot = 0.0
    for n in range(deg + 1):
        if f[n] != 0.0:
            tot += f[n] * _geom_tail(n - beta, S_LO, -1)
    return tot


def _low_tail_origin_2d(beta: float) -> float:
    """Trapezoid sum over nodes s < S_LO of (1 - ive(0,2t)^2) t^-beta."""
    deg = _SERIES_DEG
    f = np.convolve(np.convolve(_series_coeffs_exp(4.0, deg), _series_coeffs_exp_i(0, deg))[: deg + 1],
                    _series_coeffs_exp_i(0, deg))[: deg + 1]
    g = -f
    g[0] = 0.0             # 1 - e^{-4t} I0(2t)^2: the constant terms cancel exactly
    tot = 0.0
    for n in range(1, deg + 1):
        if g[n] != 0.0:
            tot += g[n] * _geom_tail(n - beta, S_LO, -1)
    return tot


def _low_tail_1d(k: int, beta: float, origin: bool) -> float:
    deg = _SERIES_DEG
    f = np.convolve(_series_coeffs_exp(2.0, deg), _series_coeffs_exp_i(k, deg))[: deg + 1]
    if origin:
        f = -f
        f[0] = 0.0
    tot = 0.0
    for n in range(deg + 1):
        if f[n] != 0.0 and n - beta > 0:
            tot += f[n] * _geom_tail(n - beta, S_LO, -1)
    return tot


def _asym_coeffs(k: np.ndarray, nterms: int, x_scale: float) -> np.ndarray:
    """Rows m = 0..nterms-1 of the Hankel series of ive(k, x_scale*t) in powers of 1/t,
    without the (2 pi x_scale t)^-1/2 prefactor."""
    mu = 4.0 * np.asarray(k, dtype=np.float64) ** 2
    out = np.empty((nterms, mu.size))
    term = np.ones_like(mu)
    out[0] = term
    for m in range(1, nterms):
        term = term * (-(mu - (2 * m - 1) ** 2) / (m * 8.0 * x_scale))
        out[m] = term
    return out


# --------------------------------------------------------------------------
# origin terms 1 - e^{-2t} I0(2t) and 1 - e^{-4t} I0(2t)^2 without cancellation
# --------------------------------------------------------------------------
def _i0m1_series(t: float) -> float:
    """I_0(2t) - 1 = sum_{m>=1} t^(2m) / (m!)^2, summed directly (t < 1)."""
    term = 1.0
    acc = 0.0
    m = 0
    while True:
        m += 1
        term *= t * t / (m * m)
        acc += term
        if term < 1e-18 * acc:
            return acc


def _one_minus_ive0_pow(t: float, power: int) -> float:
    """1 - (e^{-2t} I_0(2t))^power for power in {1, 2}."""
    if t < 1.0:
        return -math.expm1(power * (math.log1p(_i0m1_series(t)) - 2.0 * t))
    return -math.expm1(power * math.log(float(ive(0, 2.0 * t))))


# --------------------------------------------------------------------------
# 1D coefficients through the same quadrature (used only to pin the quadrature)
# --------------------------------------------------------------------------
def riesz_coeffs_quadrature(alpha: float, n: int) -> np.ndarray:
    """a_k, k = 0..n-1, from beta/Gamma(1-beta) int (delta_k0 - ive(k,2t)) t^(-1-beta) dt."""
    beta = alpha / 2.0
    cb = beta / math.gamma(1.0 - beta)
    k = np.arange(n)
    _check_asym_range(n)
    s_nodes = np.arange(S_LO, S_HI + 0.5 * DS, DS)
    acc = np.zeros(n)
    acc0 = 0.0
    for s in s_nodes:
        t = math.exp(s)
        w = DS * math.exp(-beta * s)
        acc += w * ive(k, 2.0 * t)
        acc0 += w * _one_minus_ive0_pow(t, 1)
    # nodes below S_LO: small-t power series
    for kk in range(min(n, _LOW_TAIL_ORDER)):
        acc[kk] += _low_tail_1d(kk, beta, origin=False)
    acc0 += _low_tail_1d(0, beta, origin=True)
    # nodes above S_HI: ive(k,2t) = (4 pi t)^-1/2 sum_m A_m(k) t^-m, times t^-beta
    A = _asym_coeffs(k, _ASYM_TERMS, 2.0)
    hi = np.zeros(n)
    for m in range(_ASYM_TERMS):
        hi += A[m] * _geom_tail(-(0.5 + beta + m), S_HI, +1)
    hi /= math.sqrt(4.0 * math.pi)
    acc += hi
    acc0 += _geom_tail(-beta, S_HI, +1) - hi[0]
    out = -cb * acc
    out[0] = cb * acc0
    return out


# --------------------------------------------------------------------------
# 2D coefficients a_ij, 0 <= i, j < n
# --------------------------------------------------------------------------
def laplacian_coeffs(alpha: float, n: int) -> np.ndarray:
    """a_ij^(alpha) for 0 <= i, j < n as an (n, n) array indexed [i, j] (symmetric)."""
    beta = alpha / 2.0
    cb = beta / math.gamma(1.0 - beta)
    _check_asym_range(n)
    k = np.arange(n)
    s_nodes = np.arange(S_LO, S_HI + 0.5 * DS, DS)
    # node matrix: row q = sqrt(weight_q) * ive(k, 2 t_q); the sum over nodes is Bm^T Bm
    Bm = np.empty((s_nodes.size, n))
    acc0 = 0.0
    for q, s in enumerate(s_nodes):
        t = math.exp(s)
        w = DS * math.exp(-beta * s)
        Bm[q] = math.sqrt(w) * ive(k, 2.0 * t)
        acc0 += w * _one_minus_ive0_pow(t, 2)
    acc = Bm.T @ Bm
    # nodes above S_HI: product of the two Hankel series, (4 pi t)^-1 prefactor
    A = _asym_coeffs(k, _ASYM_TERMS, 2.0)
    W = np.zeros((_ASYM_TERMS, _ASYM_TERMS))
    for p in range(_ASYM_TERMS):
        for r in range(_ASYM_TERMS - p):
            W[p, r] = _geom_tail(-(1.0 + beta + p + r), S_HI, +1) / (4.0 * math.pi)
    hi = A.T @ W @ A
    acc += hi
    acc0 += _geom_tail(-beta, S_HI, +1) - hi[0, 0]
    # nodes below S_LO: only orders with small i + j contribute
    m = min(n, _LOW_TAIL_ORDER)
    for i in range(m):
        for j in range(i, m - i):
            if i + j == 0:
                continue
            v = _low_tail_2d(i, j, beta)
            acc[i, j] += v
            if i != j:
                acc[j, i] += v
    acc0 += _low_tail_origin_2d(beta)
    out = -cb * acc
    out[0, 0] = cb * acc0
    return out
