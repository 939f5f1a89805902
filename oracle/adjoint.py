"""Oracle: gradients through the S-ADI time loop (test infrastructure).

The paper has no adjoint; this is the chain rule applied to the delta form of the scheme
(section "Fast implementation based on GS formula"), written on a stored trajectory with
dense operators:

    u^1     = u^0 + Uh^0,   Uh^0 = H^-1 B^0 H^-1,  B^0 = tau phi2 - tau^2/2 kappa L u^0 + tau^2/2 g(u^0)
    u^{n+1} = 2 u^n - u^{n-1} + Uh^n,               B^n = -tau^2 kappa L u^n + tau^2 g(u^n)

with H = I + kappa tau^2/2 D.  For a scalar J(u^K) and a^n = dJ/du^n (totals), walking
back from a^K = dJ/du^K:

    a^n = 2 a^{n+1} - a^{n+2} + Jac_n^T a^{n+1}    (n >= 1; a^0 uses 1 instead of 2)
    Jac_n^T w = -c kappa L (H^-1 w H^-1) + c g'(u^n) * (H^-1 w H^-1),  c = tau^2 (tau^2/2 at n=0)

and dJ/dkappa = sum_n < a^{n+1}, dUh^n/dkappa >, where the kappa-derivative of Uh^n at
fixed u^n is H^-1 (dB/dkappa) H^-1 - H^-1 dH Uh^n - Uh^n dH H^-1, dH = tau^2/2 D.

Only tests, the smoke check and the benchmark's CPU leg may import this module.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .scheme import Problem

G_PRIME = {
    "zero": lambda u, m: np.zeros_like(u),
    "neg_sin": lambda u, m: -np.cos(u),
    "neg_cube": lambda u, m: -3.0 * u * u,
    "neg_linear": lambda u, m: -m * np.ones_like(u),
}


def trajectory(P: Problem, phi1: np.ndarray, phi2: np.ndarray, nsteps: int) -> list:
    """u^0 .. u^nsteps of the delta form."""
    U = [phi1, P.first_step_delta(phi1, phi2)]
    for _ in range(1, nsteps):
        U.append(P.step_delta(U[-2], U[-1]))
    return U


def loss(P: Problem, phi1, phi2, nsteps: int, u_obs) -> float:
    return float(np.sum((trajectory(P, phi1, phi2, nsteps)[-1] - u_obs) ** 2))


def gradients(P: Problem, phi1, phi2, nsteps: int, u_obs):
    """J = sum((u^K - u_obs)^2) and its gradients with respect to phi1 and kappa."""
    U = trajectory(P, phi1, phi2, nsteps)
    K = nsteps
    hinv = scipy.linalg.cho_solve(P.cho, np.eye(P.n))
    dH = (P.tau ** 2 / 2.0) * P.D
    gp = G_PRIME[P.g]
    a_next = 2.0 * (U[K] - u_obs)         # a^K
    a_next2 = np.zeros_like(a_next)       # a^{K+1}
    dkappa = 0.0
    for n in range(K - 1, -1, -1):
        c = P.tau ** 2 if n >= 1 else P.tau ** 2 / 2.0
        w = a_next                         # a^{n+1}
        z = hinv @ w @ hinv
        jt = -c * P.kappa * P.lh(z) + c * gp(U[n], P.g_param) * z
        B = P.rhs_delta(U[n], phi2 if n == 0 else None)
        uh = hinv @ B @ hinv
        dB = -c * P.lh(U[n])
        dU = hinv @ dB @ hinv - hinv @ dH @ uh - uh @ dH @ hinv
        dkappa += float(np.sum(w * dU))
        a_n = (2.0 if n >= 1 else 1.0) * w - a_next2 + jt
        a_next2, a_next = a_next, a_n
    return float(np.sum((U[K] - u_obs) ** 2)), a_next, dkappa
