"""Oracle: the S-ADI time stepping, in plain FP64 (test infrastructure).

Two independent renderings of the scheme of the paper:

* the literal forms, equation (ADI scheme) for n >= 1 and equation (ADI scheme
  initial) for n = 0, with the explicit remainder R = L_h - delta_x - delta_y,
  multiplied through by tau^2 (resp. tau^2/2) and with the implicit part factored
  as (1 + kappa tau^2/2 delta_x)(1 + kappa tau^2/2 delta_y), i.e. H U H;
* the delta form of section "Fast implementation based on GS formula"
  (equation (ADI scheme equivalent)): H Uhat H = B with the full L_h applied
  explicitly, then u^{n+1} = 2u^n - u^{n-1} + Uhat (n >= 1), u^1 = u^0 + Uhat (n = 0).

Both solve H X H = Y as H^-1 Y H^-1 with a Cholesky factor of H (scipy); no
Gohberg-Semencul formula and no fast Toeplitz solver appear here.

Also here: the discrete energy H_n of the stability proof (section "Stability";
exactly conserved when g = 0) and the Error_1 / Error_2 estimators of section
"Numerical experiments".

This module is test infrastructure: only tests, the smoke check and the CPU
baseline of the benchmark may import it.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np
import scipy.linalg
from threadpoolctl import threadpool_limits

from . import coeffs, operators

# nonlinearity g(u) of the equation; the paper's examples use -sin u and -u^3
G_FUNCS: dict[str, Callable[[np.ndarray, float], np.ndarray]] = {
    "zero": lambda u, m: np.zeros_like(u),
    "neg_sin": lambda u, m: -np.sin(u),
    "neg_cube": lambda u, m: -(u ** 3),
    "neg_linear": lambda u, m: -m * u,
}


@dataclasses.dataclass
class Problem:
    alpha: float
    kappa: float
    n: int
    tau: float
    domain: tuple[float, float] = (-1.0, 1.0)
    g: str = "neg_sin"
    g_param: float = 0.0
    dense: Optional[bool] = None          # None: dense L_h matrix for N <= 48
    a1: Optional[np.ndarray] = None       # injected 1D coefficients (length >= N)
    a2: Optional[np.ndarray] = None       # injected 2D coefficients (N x N)
    embed: Optional[int] = None           # size P of the BCCB embedding of L_h (None: 2N)

    def __post_init__(self):
        n = self.n
        self.h, self.x = operators.grid(self.domain[0], self.domain[1], n)
        if self.a1 is None:
            self.a1 = coeffs.riesz_coeffs(self.alpha, n)
        if self.a2 is None:
            self.a2 = coeffs.laplacian_coeffs(self.alpha, n)
        self.D = operators.riesz_matrix(self.a1, n, self.h, self.alpha)
        self.H = operators.h_matrix(self.D, self.kappa, self.tau)
        self.cho = scipy.linalg.cho_factor(self.H, lower=True)
        if self.dense is None:
            self.dense = n <= 48
        if self.dense:
            self.L = operators.bttb_matrix(self.a2, n, self.h, self.alpha)
        else:
            self.sym = operators.BCCBSymbol(self.a2, n, self.embed)
        self._hinv = None

    # --- operators -------------------------------------------------------
    def g_of(self, U: np.ndarray) -> np.ndarray:
        return G_FUNCS[self.g](U, self.g_param)

    def lh(self, U: np.ndarray) -> np.ndarray:
        if self.dense:
            return operators.lh_apply_dense(self.L, U)
        return operators.lh_apply_fft(self.sym, U, self.h, self.alpha)

    def dx(self, U):
        return self.D @ U

    def dy(self, U):
        return U @ self.D

    def remainder(self, U):
        """R U = (L_h - delta_x - delta_y) U, the explicitly treated part."""
        return self.lh(U) - self.dx(U) - self.dy(U)

    def solve_hh(self, Y: np.ndarray) -> np.ndarray:
        """X with H X H = Y: both line sweeps by Cholesky solves."""
        X = scipy.linalg.cho_solve(self.cho, Y)            # H^-1 Y (x-lines)
        return scipy.linalg.cho_solve(self.cho, X.T).T     # (.) H^-1 (y-lines)

    def solve_hh_inverse(self, Y: np.ndarray) -> np.ndarray:
        """Same as solve_hh through an explicit H^-1 (two GEMMs; faster for large N)."""
        if self._hinv is None:
            self._hinv = scipy.linalg.cho_solve(self.cho, np.eye(self.n))
        return self._hinv @ Y @ self._hinv

    # --- literal forms ---------------------------------------------------
    def first_step_literal(self, U0: np.ndarray, Phi2: np.ndarray) -> np.ndarray:
        k, t = self.kappa, self.tau
        rhs = (U0 + t * Phi2 + (k * k * t ** 4 / 4.0) * self.dy(self.dx(U0))
               - (k * t * t / 2.0) * self.remainder(U0) + (t * t / 2.0) * self.g_of(U0))
        return self.solve_hh(rhs)

    def step_literal(self, Uprev: np.ndarray, Ucur: np.ndarray) -> np.ndarray:
        k, t = self.kappa, self.tau
        rhs = (2.0 * Ucur - Uprev
               - (k * t * t / 2.0) * (self.dx(Uprev) + self.dy(Uprev))
               + (k * k * t ** 4 / 4.0) * self.dy(self.dx(2.0 * Ucur - Uprev))
               - k * t * t * self.remainder(Ucur) + t * t * self.g_of(Ucur))
        return self.solve_hh(rhs)

    # --- delta form ------------------------------------------------------
    def rhs_delta(self, Ucur: np.ndarray, Phi2: Optional[np.ndarray] = None) -> np.ndarray:
        k, t = self.kappa, self.tau
        if Phi2 is None:
            return -t * t * k * self.lh(Ucur) + t * t * self.g_of(Ucur)
        return t * Phi2 - (t * t / 2.0) * k * self.lh(Ucur) + (t * t / 2.0) * self.g_of(Ucur)

    def increment(self, Ucur: np.ndarray, Phi2: Optional[np.ndarray] = None, gemm: bool = False) -> np.ndarray:
        B = self.rhs_delta(Ucur, Phi2)
        return self.solve_hh_inverse(B) if gemm else self.solve_hh(B)

    def first_step_delta(self, U0, Phi2, gemm: bool = False):
        return U0 + self.increment(U0, Phi2, gemm)

    def step_delta(self, Uprev, Ucur, gemm: bool = False):
        return 2.0 * Ucur - Uprev + self.increment(Ucur, None, gemm)

    # --- single calls (what the device entry points compute) -------------
    def line_solve(self, V: np.ndarray) -> np.ndarray:
        """H^-1 v for every row v of V (shape (nlines, N))."""
        with self.blas_limits():
            return scipy.linalg.cho_solve(self.cho, V.T).T

    def first_step(self, U0, Phi2):
        with self.blas_limits():
            return self.first_step_delta(U0, Phi2, gemm=self.n >= 256)

    def step(self, Uprev, Ucur):
        with self.blas_limits():
            return self.step_delta(Uprev, Ucur, gemm=self.n >= 256)

    def lh_apply(self, U):
        with self.blas_limits():
            return self.lh(U)

    # --- whole runs ------------------------------------------------------
    def blas_limits(self):
        """Single-threaded BLAS for small grids (thread start-up dominates there)."""
        return threadpool_limits(limits=1 if self.n < 256 else None)

    def run(self, U0, Phi2, nsteps: int, form: str = "delta", gemm: bool = False,
            callback=None):
        """u^0 .. u^nsteps; returns (u^{nsteps-1}, u^{nsteps}).  nsteps >= 1."""
        with self.blas_limits():
            return self._run(U0, Phi2, nsteps, form, gemm, callback)

    def _run(self, U0, Phi2, nsteps, form, gemm, callback):
        if form == "literal":
            first, step = self.first_step_literal, self.step_literal
            U1 = first(U0, Phi2)
        else:
            U1 = self.first_step_delta(U0, Phi2, gemm)
            step = lambda a, b: self.step_delta(a, b, gemm)
        prev, cur = U0, U1
        if callback:
            callback(1, prev, cur)
        for n in range(1, nsteps):
            prev, cur = cur, step(prev, cur)
            if callback:
                callback(n + 1, prev, cur)
        return prev, cur

    # --- diagnostics -----------------------------------------------------
    def inner(self, V, W):
        return self.h * self.h * float(np.sum(V * W))

    def energy(self, Uprev, Ucur) -> float:
        """H_n of the stability proof with w^n = Uprev, w^{n+1} = Ucur (g = 0 case)."""
        k, t = self.kappa, self.tau
        dt = (Ucur - Uprev) / t
        nrm = self.inner(dt, dt)
        at = self.inner(self.dx(dt) + self.dy(dt), dt)
        a = self.inner(self.lh(dt), dt)
        b = self.inner(self.dy(self.dx(dt)), dt)
        e2 = (nrm + (t * t * k / 2.0) * (at - a)
              + (k / 2.0) * (self.inner(self.lh(Ucur), Ucur) + self.inner(self.lh(Uprev), Uprev))
              + (k * k * t ** 4 / 4.0) * b)
        return math.sqrt(e2)


def error1(u_tau: np.ndarray, u_tau_half: np.ndarray, h: float) -> float:
    """Error_1(tau,h) = sqrt(h^2 sum |u^M(tau,h) - u^{2M}(tau/2,h)|^2)."""
    return math.sqrt(h * h * float(np.sum((u_tau - u_tau_half) ** 2)))


def error2(u_h: np.ndarray, u_h_half: np.ndarray, h: float) -> float:
    """Error_2(tau,h) = sqrt(h^2 sum |u^M_ij(tau,h) - u^M_{2i,2j}(tau,h/2)|^2); the fine grid
    has 2N+1 interior nodes and its node 2i (1-based) is x_i."""
    n = u_h.shape[0]
    assert u_h_half.shape[0] == 2 * n + 1
    fine = u_h_half[1::2, 1::2]                        # 1-based 2i -> 0-based 2i-1
    return math.sqrt(h * h * float(np.sum((u_h - fine) ** 2)))
