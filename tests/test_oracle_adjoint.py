"""Pins of the oracle's reverse-mode gradients: central finite differences of the
oracle's own forward loss (no adjoint algebra involved)."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as A
from oracle import scheme as S

N, ALPHA, KAPPA, TAU, K = 15, 1.6, 1.3, 0.05, 12


def problem(kappa=KAPPA, g="neg_sin"):
    return S.Problem(alpha=ALPHA, kappa=kappa, n=N, tau=TAU, g=g)


def data():
    phi1 = 3.0 * W.asymmetric_field(N, seed=41)
    phi2 = 0.5 * W.asymmetric_field(N, seed=42)
    u_obs = W.asymmetric_field(N, seed=43)
    return phi1, phi2, u_obs


@pytest.mark.parametrize("g", ["neg_sin", "neg_cube", "zero"])
def test_kappa_gradient_matches_central_difference(g):
    phi1, phi2, u_obs = data()
    _, _, dk = A.gradients(problem(g=g), phi1, phi2, K, u_obs)
    eps = 1e-5
    jp = A.loss(problem(KAPPA + eps, g), phi1, phi2, K, u_obs)
    jm = A.loss(problem(KAPPA - eps, g), phi1, phi2, K, u_obs)
    fd = (jp - jm) / (2 * eps)
    assert abs(dk - fd) <= 1e-7 * abs(fd)


@pytest.mark.parametrize("g", ["neg_sin", "neg_cube"])
def test_phi1_gradient_matches_directional_differences(g):
    phi1, phi2, u_obs = data()
    P = problem(g=g)
    _, grad, _ = A.gradients(P, phi1, phi2, K, u_obs)
    rng = np.random.default_rng(7)
    for _ in range(3):
        v = rng.standard_normal(phi1.shape)
        eps = 1e-6
        fd = (A.loss(P, phi1 + eps * v, phi2, K, u_obs) - A.loss(P, phi1 - eps * v, phi2, K, u_obs)) / (2 * eps)
        assert abs(float(np.sum(grad * v)) - fd) <= 1e-6 * abs(fd)


def test_gradient_of_a_single_step_is_exact_for_the_linear_case():
    """g = 0: J is quadratic in phi1, so the central difference is exact up to rounding
    for any step, and the gradient must match it to near machine precision."""
    phi1, phi2, u_obs = data()
    P = problem(g="zero")
    _, grad, _ = A.gradients(P, phi1, phi2, 3, u_obs)
    e = np.zeros_like(phi1)
    e[4, 9] = 1.0
    fd = (A.loss(P, phi1 + 0.5 * e, phi2, 3, u_obs) - A.loss(P, phi1 - 0.5 * e, phi2, 3, u_obs)) / 1.0
    assert abs(grad[4, 9] - fd) <= 1e-10 * max(1.0, abs(fd))
