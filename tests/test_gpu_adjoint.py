"""Gradients through the S-ADI time loop on the GPU (sadi_adjoint_step behind a torch
autograd function) against the oracle's reverse-mode gradients and against central
finite differences of the GPU forward run."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as A
from oracle import scheme as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(G):
    return torch.from_numpy(np.ascontiguousarray(G.T)).to(_dev())


def from_dev(t):
    return t.detach().cpu().numpy().T.copy()


def grads_gpu(phi1, phi2, u_obs, alpha, kappa, n, tau, steps, checkpoint):
    from paper_2312_06206_amd.adjoint import sadi_loop
    x = to_dev(phi1).requires_grad_(True)
    k = torch.tensor(kappa, dtype=torch.float64, requires_grad=True)
    uK = sadi_loop(x, k, alpha, n, tau, steps, phi2=to_dev(phi2), checkpoint=checkpoint)
    J = ((uK - to_dev(u_obs)) ** 2).sum()
    J.backward()
    return float(J.item()), from_dev(x.grad), float(k.grad.item())


@pytest.mark.parametrize("n,steps,checkpoint,g", [(15, 12, 5, "neg_sin"), (31, 20, 50, "neg_sin"),
                                                  (63, 9, 4, "neg_sin")])
def test_adjoint_matches_oracle_gradients(n, steps, checkpoint, g):
    _say(f"adjoint vs oracle n={n} steps={steps} C={checkpoint}")
    alpha, kappa, tau = 1.6, 1.3, 0.05
    phi1 = 3.0 * W.asymmetric_field(n, seed=41)
    phi2 = 0.5 * W.asymmetric_field(n, seed=42)
    u_obs = W.asymmetric_field(n, seed=43)
    P = S.Problem(alpha=alpha, kappa=kappa, n=n, tau=tau, g=g)
    J_ref, g_ref, k_ref = A.gradients(P, phi1, phi2, steps, u_obs)
    J, gphi, gk = grads_gpu(phi1, phi2, u_obs, alpha, kappa, n, tau, steps, checkpoint)
    assert abs(J - J_ref) <= 1e-11 * abs(J_ref)
    assert np.abs(gphi - g_ref).max() <= 1e-10 * np.abs(g_ref).max()
    assert abs(gk - k_ref) <= 1e-10 * abs(k_ref)


def test_checkpoint_interval_does_not_change_the_gradient():
    _say("adjoint checkpoint invariance")
    n, alpha, kappa, tau, steps = 63, 1.6, 1.0, 0.02, 23
    phi1 = W.asymmetric_field(n, seed=51)
    u_obs = W.asymmetric_field(n, seed=52)
    out = [grads_gpu(phi1, np.zeros_like(phi1), u_obs, alpha, kappa, n, tau, steps, c) for c in (1, 5, 23, 100)]
    # runs alternate the grid orientation from their first step, so segments of different
    # lengths round differently: the gradients agree to rounding, not bit for bit
    for J, gphi, gk in out[1:]:
        assert abs(J - out[0][0]) <= 1e-13 * abs(out[0][0])
        assert np.abs(gphi - out[0][1]).max() <= 1e-12 * np.abs(out[0][1]).max()
        assert abs(gk - out[0][2]) <= 1e-12 * abs(out[0][2])
    # the same checkpoint interval twice: bitwise identical
    again = grads_gpu(phi1, np.zeros_like(phi1), u_obs, alpha, kappa, n, tau, steps, 5)
    assert again[0] == out[1][0] and np.array_equal(again[1], out[1][1]) and again[2] == out[1][2]


def test_adjoint_vs_central_differences_n511():
    """N = 511, alpha = 1.6, 500 steps, tau = 1e-3; u_obs from kappa = 1.3 and a seeded
    bump; gradient at kappa = 1 and another seeded bump, checkpoint every 50 steps."""
    from paper_2312_06206_amd import Solver
    _say("adjoint vs finite differences N=511")
    n, alpha, tau, steps = 511, 1.6, 1e-3, 500
    dev = _dev()
    obs_phi1 = W.seeded_bump(n, seed=0)
    with Solver(alpha, 1.3, n, tau) as s:
        a = to_dev(obs_phi1)
        b = s.first_step(a, torch.zeros_like(a))
        s.run(a, b, steps - 1)
        u_obs = from_dev(b)
    phi1 = W.seeded_bump(n, seed=1)
    J, gphi, gk = grads_gpu(phi1, np.zeros_like(phi1), u_obs, alpha, 1.0, n, tau, steps, 50)

    def loss(kappa, p1):
        with Solver(alpha, kappa, n, tau) as s:
            a = to_dev(p1)
            b = s.first_step(a, torch.zeros_like(a))
            s.run(a, b, steps - 1)
            return float(((b - to_dev(u_obs)) ** 2).sum().item())

    eps = 1e-4
    fd_k = (loss(1.0 + eps, phi1) - loss(1.0 - eps, phi1)) / (2 * eps)
    assert abs(gk - fd_k) <= 1e-6 * abs(fd_k)
    v = W.asymmetric_field(n, seed=3)
    e = 1e-4
    fd_v = (loss(1.0, phi1 + e * v) - loss(1.0, phi1 - e * v)) / (2 * e)
    assert abs(float(np.sum(gphi * v)) - fd_v) <= 1e-6 * abs(fd_v)
    assert torch.device(dev).type == "cuda"
