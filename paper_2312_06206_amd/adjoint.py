"""Differentiable S-ADI time loop: u^K as a torch function of phi1 and kappa.

The forward pass runs the library's FP64 steps and keeps the state pair every
`checkpoint` steps; the backward pass recomputes each segment from its checkpoint and
walks it back with sadi_adjoint_step (include/sadi.h), which gives dJ/du^n and the
kappa-derivative of every step.  All arithmetic runs in the library's kernels; this
module only schedules the calls and holds the tensors.
"""
from __future__ import annotations

from typing import Sequence

import torch

from .binding import Solver


class _Loop(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi1, kappa, phi2, alpha, n, tau, steps, domain, checkpoint):
        solver = Solver(alpha, float(kappa.item()), n, tau, domain)
        u0 = phi1.detach().contiguous().clone()
        p2 = phi2.detach().contiguous()
        prev, cur = u0.clone(), solver.first_step(u0, p2)
        pairs = {}                                  # k -> (u^{kC-1}, u^{kC}) for 1 <= k, kC < K
        done = 1
        k = 1
        while k * checkpoint < steps:               # backward restarts only from kC < K
            solver.run(prev, cur, k * checkpoint - done)
            done = k * checkpoint
            pairs[k] = (prev.clone(), cur.clone())
            k += 1
        if done < steps:
            solver.run(prev, cur, steps - done)
        ctx.solver, ctx.pairs, ctx.u0, ctx.p2 = solver, pairs, u0, p2
        ctx.steps, ctx.checkpoint = steps, checkpoint
        return cur.clone()

    @staticmethod
    def backward(ctx, grad_out):
        s, C, K = ctx.solver, ctx.checkpoint, ctx.steps
        a_next = grad_out.detach().contiguous().clone()       # a^K
        a_next2 = None                                        # a^{K+1} = 0
        dk = torch.zeros(1, dtype=torch.float64, device=a_next.device)
        nseg = (K - 1) // C                                   # segments k = nseg .. 0 cover n = kC .. kC + C - 1
        for k in range(nseg, -1, -1):
            lo, hi = k * C, min(k * C + C, K)                 # adjoint steps n = hi-1 .. lo need u^{lo-1} .. u^{hi}
            if k == 0:
                states = {0: ctx.u0, 1: s.first_step(ctx.u0, ctx.p2)}
                first = 1
            else:
                a, b = ctx.pairs[k]
                states = {lo - 1: a.clone(), lo: b.clone()}
                first = lo
            for m in range(first, hi):
                nxt = states[m - 1].clone()
                s.step(nxt, states[m])
                states[m + 1] = nxt
            for n in range(hi - 1, lo - 1, -1):
                a_cur = torch.empty_like(a_next)
                s.adjoint_step(0 if n >= 1 else 1, states.get(n - 1), states[n], states[n + 1], a_next, a_next2,
                               a_cur, dk)
                a_next2, a_next = a_next, a_cur
        grad_phi1 = a_next                                    # a^0 = dJ/dphi1
        grad_kappa = dk.reshape(()).cpu()
        # the solver stays open while the autograd context holds it (a second backward with
        # retain_graph=True reuses it); Solver.__del__ frees it with the context
        return grad_phi1, grad_kappa, None, None, None, None, None, None, None


def sadi_loop(phi1: torch.Tensor, kappa: torch.Tensor, alpha: float, n: int, tau: float, steps: int,
              phi2: torch.Tensor | None = None, domain: Sequence[float] = (-1.0, 1.0),
              checkpoint: int = 50) -> torch.Tensor:
    """u^steps of the S-ADI scheme from (phi1, phi2) with parameter kappa (a 0-d CPU
    float64 tensor).  Differentiable with respect to phi1 and kappa."""
    if steps < 1 or checkpoint < 1:
        raise ValueError("steps and checkpoint must be >= 1")
    if phi2 is None:
        phi2 = torch.zeros_like(phi1)
    return _Loop.apply(phi1, kappa, phi2, float(alpha), int(n), float(tau), int(steps),
                       (float(domain[0]), float(domain[1])), int(checkpoint))
