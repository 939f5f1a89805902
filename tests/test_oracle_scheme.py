"""Pins for the oracle's operators and time stepping (CPU only)."""
import math

import numpy as np
import pytest
import scipy.fft

import workloads as W
from oracle import coeffs as C
from oracle import operators as O
from oracle import scheme as S


# ----------------------------------------------------------------- operators
def test_bttb_matrix_is_the_double_sum():
    alpha, n = 1.5, 5
    a2 = C.laplacian_coeffs(alpha, n)
    h, _ = O.grid(-1.0, 1.0, n)
    U = W.asymmetric_field(n, seed=3)
    L = O.bttb_matrix(a2, n, h, alpha)
    np.testing.assert_allclose(O.lh_apply_dense(L, U), O.lh_apply_loops(a2, U, h, alpha), rtol=0, atol=1e-13)


@pytest.mark.parametrize("n", [17, 31, 48])
def test_bccb_fft_matches_dense(n):
    alpha = 1.3
    a2 = C.laplacian_coeffs(alpha, n)
    h, _ = O.grid(-1.0, 1.0, n)
    U = W.asymmetric_field(n, seed=n)
    ref = O.lh_apply_dense(O.bttb_matrix(a2, n, h, alpha), U)
    got = O.lh_apply_fft(O.BCCBSymbol(a2, n), U, h, alpha)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("alpha", [1.1, 1.5, 1.9])
def test_operator_positivity_lemmas(alpha):
    """delta_x + delta_y, delta_x delta_y and L_h are SPD; L_h - delta_x - delta_y is NSD
    (the lemmas of section "Stability")."""
    n = 8
    h, _ = O.grid(-1.0, 1.0, n)
    a1 = C.riesz_coeffs(alpha, n)
    a2 = C.laplacian_coeffs(alpha, n)
    D = O.riesz_matrix(a1, n, h, alpha)
    I = np.eye(n)
    # on vec(U) (i fastest): delta_x = I (x) D, delta_y = D (x) I
    dxdy = np.kron(I, D) + np.kron(D, I)
    L = O.bttb_matrix(a2, n, h, alpha)
    for M in (dxdy, np.kron(D, D), L):
        assert np.allclose(M, M.T, atol=1e-12)
        assert np.linalg.eigvalsh(M).min() > 0
    assert np.linalg.eigvalsh(L - dxdy).max() < 0


# ----------------------------------------------------------------- scheme
def _problem(n, alpha=1.5, g="neg_sin", tau=1 / 16, **kw):
    return S.Problem(alpha=alpha, kappa=kw.pop("kappa", 1.0), n=n, tau=tau, g=g, **kw)


@pytest.mark.parametrize("n,dense", [(15, True), (33, False), (63, False)])
def test_literal_and_delta_forms_agree(n, dense):
    P = _problem(n, alpha=1.7, kappa=1.3, dense=dense)
    U0 = W.asymmetric_field(n, seed=1)
    Phi2 = 0.5 * W.asymmetric_field(n, seed=2)
    a = P.run(U0, Phi2, 40, form="literal")[1]
    b = P.run(U0, Phi2, 40, form="delta")[1]
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    # first step alone (start-up scheme)
    a1 = P.first_step_literal(U0, Phi2)
    b1 = P.first_step_delta(U0, Phi2)
    assert np.abs(a1 - b1).max() <= 1e-13 * np.abs(a1).max()


@pytest.mark.parametrize("alpha", [1.2, 1.8])
def test_energy_conserved_without_nonlinearity(alpha):
    """With g = 0 the discrete energy H_n of the stability proof is constant for n >= 0."""
    P = _problem(19, alpha=alpha, g="zero", tau=0.05)
    E = []
    P.run(W.asymmetric_field(19, seed=4), 0.3 * W.asymmetric_field(19, seed=5), 64,
          callback=lambda k, a, b: E.append(P.energy(a, b)))
    E = np.array(E)
    assert np.abs(E - E[0]).max() <= 1e-13 * E[0]


def test_energy_not_conserved_with_nonlinearity():
    P = _problem(19, alpha=1.5, g="neg_sin", tau=0.05)
    E = []
    P.run(3.0 * W.asymmetric_field(19, seed=4), np.zeros((19, 19)), 32,
          callback=lambda k, a, b: E.append(P.energy(a, b)))
    assert np.abs(np.array(E) - E[0]).max() > 1e-6 * E[0]


@pytest.mark.parametrize("form", ["delta", "literal"])
def test_alpha2_modal_closed_form(form):
    """alpha = 2 with injected 3-point / 5-point coefficients: every operator is diagonal in
    the DST-I basis, and each mode (k,l) follows c^{n+1} = (2-rho) c^n - c^{n-1}, solved in
    closed form as A cos(n theta) + B sin(n theta), cos theta = 1 - rho/2."""
    n, tau, kappa, m, steps = 21, 0.03, 0.8, 0.7, 50
    a1 = np.zeros(n)
    a1[:2] = [2.0, -1.0]
    a2 = np.zeros((n, n))
    a2[0, 0], a2[1, 0], a2[0, 1] = 4.0, -1.0, -1.0
    P = S.Problem(alpha=2.0, kappa=kappa, n=n, tau=tau, g="neg_linear", g_param=m, a1=a1, a2=a2)
    U0 = W.asymmetric_field(n, seed=7)
    Phi2 = W.asymmetric_field(n, seed=8)
    got = P.run(U0, Phi2, steps, form=form)[1]

    h = P.h
    k = np.arange(1, n + 1)
    mu = 4.0 * np.sin(k * np.pi / (2 * (n + 1))) ** 2
    beta = kappa * tau * tau / (2 * h * h)
    lam = (mu[:, None] + mu[None, :]) / (h * h)
    den = (1 + beta * mu[:, None]) * (1 + beta * mu[None, :])
    dst = lambda X: scipy.fft.dstn(X, type=1, norm="ortho")
    c0, p2 = dst(U0), dst(Phi2)
    c1 = c0 + (tau * p2 - 0.5 * tau * tau * (kappa * lam + m) * c0) / den
    rho = tau * tau * (kappa * lam + m) / den
    theta = np.arccos(1.0 - rho / 2.0)
    A = c0
    B = (c1 - c0 * np.cos(theta)) / np.sin(theta)
    ref = dst(A * np.cos(steps * theta) + B * np.sin(steps * theta))
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_second_order_in_time():
    """Order_1 = log2(Error_1(tau)/Error_1(tau/2)) -> 2 (Theorem + Remark of section 6)."""
    n, T = 31, 0.5
    P = {}
    sols = {}
    for M in (8, 16, 32, 64):
        P[M] = _problem(n, alpha=1.5, tau=T / M)
        sols[M] = P[M].run(W.config1_phi1(n), np.zeros((n, n)), M)[1]
    h = P[8].h
    e = [S.error1(sols[M], sols[2 * M], h) for M in (8, 16, 32)]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert all(1.9 < o < 2.1 for o in orders), orders


# ----------------------------------------------------------------- the paper's tables
@pytest.mark.parametrize("row", range(3))
def test_table2_sine_gordon_space_errors(golden, row):
    t = golden["table2_sine_gordon_space"]
    alpha, ref = t["rows"][row]["alpha"], t["rows"][row]["error2"]
    M = round(t["T"] / t["tau"])
    sol = {}
    for n in (19, 39):
        P = S.Problem(alpha=alpha, kappa=1.0, n=n, tau=t["tau"], domain=(-10.0, 10.0), g="neg_sin")
        phi1, phi2 = W.sine_gordon_data(n)
        sol[n] = P.run(phi1, phi2, M)[1]
    e = S.error2(sol[19], sol[39], 20.0 / 20)
    # the paper prints 5 significant digits
    assert abs(e / ref - 1.0) < 1.5e-5, (e, ref)


@pytest.mark.parametrize("row", range(3))
def test_table4_klein_gordon_space_errors(golden, row):
    t = golden["table4_klein_gordon_space"]
    alpha, ref = t["rows"][row]["alpha"], t["rows"][row]["error2"]
    M = round(t["T"] / t["tau"])
    sol = {}
    for n in (49, 99):
        P = S.Problem(alpha=alpha, kappa=1.0, n=n, tau=t["tau"], domain=(-10.0, 10.0), g="neg_cube")
        phi1, phi2 = W.klein_gordon_data(n)
        sol[n] = P.run(phi1, phi2, M)[1]
    e = S.error2(sol[49], sol[99], 0.4)
    assert abs(e / ref - 1.0) < 1.5e-5, (e, ref)


def test_table1_sine_gordon_time_error(golden):
    t = golden["table1_sine_gordon_time"]
    alpha, ref = t["rows"][0]["alpha"], t["rows"][0]["error1"]
    n = round(20.0 / t["h"]) - 1
    sol = {}
    for tau in (t["tau"], t["tau"] / 2):
        P = S.Problem(alpha=alpha, kappa=1.0, n=n, tau=tau, domain=(-10.0, 10.0), g="neg_sin")
        phi1, phi2 = W.sine_gordon_data(n)
        sol[tau] = P.run(phi1, phi2, round(t["T"] / tau), gemm=True)[1]
    e = S.error1(sol[t["tau"]], sol[t["tau"] / 2], t["h"])
    assert abs(e / ref - 1.0) < 1.5e-5, (e, ref)
