"""Steps captured in a HIP graph (through torch.cuda.graph) replay to the eager results.  Needs a GPU.

The step entry points enqueue only kernels on the bound stream (no memset or host wait), so a
caller may capture them.  Each replay is checked against the same calls made eagerly on a
second solver, with eager work and synchronisations between the replays.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


# N = 799: the general-N correction runs as matrix-core products inside the captured step
@pytest.mark.parametrize("n,call,count", [(255, "step", 2), (1023, "step", 2), (255, "run", 3), (511, "run", 4),
                                          (799, "step", 2), (799, "run", 3), (4095, "step", 2), (4095, "run", 3)])
def test_graph_replay_matches_eager(n, call, count):
    from paper_2312_06206_amd import Solver
    dev = _dev()
    _say(f"graph replay n={n} call={call} count={count}")
    alpha, tau = 1.5, 2.0 / 64
    phi1 = W.asymmetric_field(n, seed=n)
    phi2 = 0.3 * W.seeded_bump(n, seed=n + 1)
    g_s = Solver(alpha, 1.0, n, tau)
    e_s = Solver(alpha, 1.0, n, tau)
    u0 = torch.from_numpy(np.ascontiguousarray(phi1.T)).to(dev)
    v0 = torch.from_numpy(np.ascontiguousarray(phi2.T)).to(dev)
    u1 = g_s.first_step(u0, v0)
    ga, gb = u0.clone(), u1.clone()      # graph state (u_prev, u_cur)
    ea, eb = u0.clone(), u1.clone()      # eager state
    torch.cuda.synchronize()

    def body(s, a, b):
        if call == "step":
            for k in range(count):        # u_prev <- next, roles alternate
                if k % 2 == 0:
                    s.step(a, b)
                else:
                    s.step(b, a)
        else:
            s.run(a, b, count)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):        # one eager call on the capture stream first
        body(g_s, ga, gb)
    torch.cuda.current_stream().wait_stream(side)
    body(e_s, ea, eb)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        body(g_s, ga, gb)
    torch.cuda.synchronize()
    for rep in range(3):
        graph.replay()
        body(e_s, ea, eb)
        scratch = torch.randn(n, n, dtype=torch.float64, device=dev).sum()   # unrelated eager work
        torch.cuda.synchronize()
        assert torch.isfinite(scratch)
        for g, e in ((ga, ea), (gb, eb)):
            assert _rel(g, e) <= 1e-13, (rep, _rel(g, e))
    _say(f"  ok after 3 replays, |u| = {float(gb.abs().max()):.3e}")
    g_s.close()
    e_s.close()
