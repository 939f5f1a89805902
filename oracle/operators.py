"""Oracle: the discrete operators of the S-ADI scheme in plain FP64 (test infrastructure).

Notation follows the paper (sections "Construction of S-ADI scheme" and "Fast
implementation based on GS formula"): grid functions are N x N arrays U with
U[i, j] = u(x_i, y_j), i the x index, j the y index.  D = h^-alpha T(a_0..a_{N-1})
is the matrix of the 1D fractional centred difference, so delta_x U = D U and
delta_y U = U D; L_h is the discrete fractional Laplacian (a BTTB operator).
The zero exterior condition means every operator is simply truncated to the grid.

Two routes for L_h U:
  * lh_apply_dense: the defining double sum, as an explicit N^2 x N^2 matrix
    (small N only);
  * lh_apply_fft: the BCCB embedding of the kernel a_{|i|,|j|} in a P x P
    circulant (P >= 2N-1) and a library 2D real FFT (scipy.fft).

Line solves use a Cholesky factorisation of H = I + (kappa tau^2 / 2) D (scipy).
This module is test infrastructure: only tests, the smoke check and the CPU
baseline of the benchmark may import it.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import scipy.fft
import scipy.linalg


def grid(a: float, b: float, n: int) -> tuple[float, np.ndarray]:
    """h = (b-a)/(N+1) and the interior nodes x_i = a + i h, i = 1..N."""
    h = (b - a) / (n + 1)
    return h, a + h * np.arange(1, n + 1)


def riesz_matrix(a1: np.ndarray, n: int, h: float, alpha: float) -> np.ndarray:
    """D = h^-alpha [a_{|i-j|}]_{i,j<N} (symmetric Toeplitz)."""
    return h ** (-alpha) * scipy.linalg.toeplitz(a1[:n])


def bttb_matrix(a2: np.ndarray, n: int, h: float, alpha: float) -> np.ndarray:
    """Explicit matrix of L_h on vec(U) with vec index i + N j (column stacking):
    entry ((i,j),(k,l)) = h^-alpha a_{|i-k|,|j-l|}."""
    idx = np.arange(n)
    di = np.abs(idx[:, None] - idx[None, :])           # |i-k|
    # L[(i + N j), (k + N l)] = a[|i-k|, |j-l|]
    L = a2[di[None, :, None, :], di[:, None, :, None]]  # axes (j, i, l, k)
    return h ** (-alpha) * L.reshape(n * n, n * n)


def lh_apply_dense(L: np.ndarray, U: np.ndarray) -> np.ndarray:
    n = U.shape[0]
    v = U.reshape(-1, order="F")                       # column stacking: i fastest
    return (L @ v).reshape(n, n, order="F")


def lh_apply_loops(a2: np.ndarray, U: np.ndarray, h: float, alpha: float) -> np.ndarray:
    """(L_h U)_ij = h^-alpha sum_{k,l} a_{|i-k|,|j-l|} U_kl, as written (tiny N only)."""
    n = U.shape[0]
    out = np.zeros_like(U)
    for i in range(n):
        for j in range(n):
            s = 0.0
            for k in range(n):
                for l in range(n):
                    s += a2[abs(i - k), abs(j - l)] * U[k, l]
            out[i, j] = s
    return h ** (-alpha) * out


class BCCBSymbol:
    """Eigenvalues of the P x P block-circulant embedding of L_h (h^-alpha excluded).

    Any P >= 2N - 1 embeds the BTTB matrix exactly (section "Fast implementation based on
    GS formula"); P = 2N unless given.  Two sizes give the same product in exact arithmetic
    and differ only in rounding, which measures the float64 floor of L_h u."""

    def __init__(self, a2: np.ndarray, n: int, p: Optional[int] = None):
        p = 2 * n if p is None else int(p)
        if p < 2 * n - 1:
            raise ValueError("embedding size must be >= 2N - 1")
        e = np.zeros((p, p))
        q = a2[:n, :n]
        e[:n, :n] = q
        e[p - n + 1:, :n] = q[1:][::-1, :]
        e[:n, p - n + 1:] = q[:, 1:][:, ::-1]
        e[p - n + 1:, p - n + 1:] = q[1:, 1:][::-1, ::-1]
        self.p = p
        self.n = n
        self.lam = scipy.fft.rfft2(e)                  # real up to rounding (even kernel)

    def apply(self, U: np.ndarray, workers: int = -1) -> np.ndarray:
        n, p = self.n, self.p
        pad = np.zeros((p, p))
        pad[:n, :n] = U
        out = scipy.fft.irfft2(scipy.fft.rfft2(pad, workers=workers) * self.lam, s=(p, p), workers=workers)
        return out[:n, :n]


def lh_apply_fft(sym: BCCBSymbol, U: np.ndarray, h: float, alpha: float, workers: int = -1) -> np.ndarray:
    return h ** (-alpha) * sym.apply(U, workers=workers)


def h_matrix(D: np.ndarray, kappa: float, tau: float) -> np.ndarray:
    """H = I + (kappa tau^2 / 2) D: the SPD Toeplitz line matrix of the ADI factors."""
    n = D.shape[0]
    return np.eye(n) + 0.5 * kappa * tau * tau * D
