"""Batched S-ADI (instances of different N, alpha, kappa in one set of launches) against
the CPU oracle, for both line-sweep paths, with and without HIP graph replay."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import scheme as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TAU = 5e-3


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


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


_ref = {}


def members():
    return W.batch_members(7, seed=11, n_choices=(15, 31, 63, 127))


def reference(mb, nsteps):
    """Oracle (u^{nsteps-1}, u^nsteps) from phi1 and phi2 = 0.3 phi1-shaped field."""
    key = (mb, nsteps)
    if key not in _ref:
        P = S.Problem(alpha=mb.alpha, kappa=mb.kappa, n=mb.n, tau=TAU, g="neg_sin")
        phi1 = mb.phi1()
        phi2 = 0.3 * W.asymmetric_field(mb.n, seed=mb.n)
        _ref[key] = P.run(phi1, phi2, nsteps)
    return _ref[key]


def make_batch(path=None, graph=False, schedule="work_lists"):
    """path: one path for every group, or a dict N -> path."""
    from paper_2312_06206_amd import Batch
    _dev()
    ms = members()
    b = Batch([m.n for m in ms], [m.alpha for m in ms], [m.kappa for m in ms], TAU, dense_max_n=127)
    if path is not None:
        for n in sorted({m.n for m in ms}):
            b.set_path(n, path[n] if isinstance(path, dict) else path)
    b.set_graph(graph)
    b.set_schedule(schedule)
    u0 = [to_dev(m.phi1()) for m in ms]
    u1 = [torch.zeros_like(t) for t in u0]
    p2 = [to_dev(0.3 * W.asymmetric_field(m.n, seed=m.n)) for m in ms]
    b.bind(u0, u1, p2)
    return b, ms, u0, u1


MIXED = {15: "dense", 31: "fft_gs", 63: "dense_mixed", 127: "fft_gs"}


@pytest.mark.parametrize("path,graph,schedule", [("fft_gs", False, "work_lists"), ("fft_gs", True, "work_lists"),
                                                 ("fft_gs", False, "groups"), ("fft_gs", True, "groups"),
                                                 ("dense", False, "work_lists"), ("dense", True, "groups"),
                                                 ("dense_mixed", False, "groups"), ("dense_mixed", True, "work_lists"),
                                                 ("mixed", False, "work_lists"), ("mixed", True, "work_lists")])
def test_batch_run_matches_oracle(path, graph, schedule):
    """The three line-sweep paths (and a mix of them across groups), both launch schedules
    (the FFT groups in shared work-list launches, or every group on its own), with and
    without graph replay.  The FP32 dense path with its FP64 refinement keeps the FP64
    bar."""
    _say(f"batch path={path} graph={graph} schedule={schedule}")
    b, ms, u0, u1 = make_batch(MIXED if path == "mixed" else path, graph, schedule)
    with b:
        b.first_step()
        b.run(6)                      # steps 2..7
        for k, m in enumerate(ms):
            ref_prev, ref_cur = reference(m, 7)
            assert rel(from_dev(u1[k]), ref_cur) < 1e-11, (k, m)
            assert rel(from_dev(u0[k]), ref_prev) < 1e-11, (k, m)


def test_batch_members_match_single_contexts():
    """A batch builds its members' line tables (Levinson recursion, Algorithm 1 tables) for
    all members in one launch; single contexts build their own.  Both run the same kernel
    bodies, so each member's run matches the same problem solved on its own context to
    rounding (the single contexts' tables are pinned to the host's extended-precision
    tables elsewhere)."""
    from paper_2312_06206_amd import Solver
    _say("batch members vs single contexts")
    b, ms, u0, u1 = make_batch("fft_gs", False, "groups")
    with b:
        b.first_step()
        b.run(9)
        torch.cuda.synchronize()
        worst = 0.0
        for k, m in enumerate(ms):
            with Solver(m.alpha, m.kappa, m.n, TAU) as s:
                a = to_dev(m.phi1())
                c = s.first_step(a, to_dev(0.3 * W.asymmetric_field(m.n, seed=m.n)))
                s.run(a, c, 9)
                e = max(rel(from_dev(u1[k]), from_dev(c)), rel(from_dev(u0[k]), from_dev(a)))
            worst = max(worst, e)
            assert e < 1e-13, (k, m, e)
        _say(f"  worst relative difference {worst:.2e}")


@pytest.mark.parametrize("counts", [(0, 1, 2), (3, 5), (4, 4)])
def test_batch_run_lengths_and_graph_replays(counts):
    """Several runs in a row (graph replays with eager work and synchronisation between
    them); every run is checked against the oracle."""
    _say(f"batch run lengths {counts}")
    b, ms, u0, u1 = make_batch("fft_gs", True)
    with b:
        b.first_step()
        done = 1
        for c in counts:
            b.run(c)
            done += c
            torch.cuda.synchronize()
            for k, m in enumerate(ms):
                ref_prev, ref_cur = reference(m, done)
                assert rel(from_dev(u1[k]), ref_cur) < 1e-11, (c, k, m)
                assert rel(from_dev(u0[k]), ref_prev) < 1e-11, (c, k, m)


def test_batch_tune_keeps_state():
    _say("batch tune")
    b, ms, u0, u1 = make_batch()
    with b:
        b.first_step()
        before = [t.clone() for t in u0 + u1]
        groups = b.tune(steps=3)
        after = u0 + u1
        assert all(torch.equal(x, y) for x, y in zip(before, after))
        assert sorted(g["n"] for g in groups) == sorted({m.n for m in ms})
        for g in groups:
            times = {"fft_gs": g["ms_fft_gs"], "dense": g["ms_dense"], "dense_mixed": g["ms_dense_mixed"]}
            assert all(t > 0 for t in times.values())
            assert g["path"] == min(times, key=lambda p: (times[p], p != "fft_gs"))
            assert g["dense_tile"] in (32, 64)
        sched, ms_groups, ms_lists = b.schedule()
        assert ms_groups > 0 and ms_lists > 0
        assert sched == ("work_lists" if ms_lists <= ms_groups else "groups")
        b.run(3)
        for k, m in enumerate(ms):
            assert rel(from_dev(u1[k]), reference(m, 4)[1]) < 1e-11


@pytest.mark.parametrize("schedule", ["work_lists", "groups"])
def test_batch_at_the_benchmark_sizes(schedule):
    """Members drawn from the batched workload's sizes (N in {255, 511, 1023}, alpha and
    kappa from its distributions): the line-sweep path with graph replay, the start-up
    step and four steps against the oracle's runs."""
    from paper_2312_06206_amd import Batch
    _dev()
    ms = W.batch_members(4, seed=0, n_choices=(255, 511, 1023))   # N = 1023, 511, 1023, 255
    _say(f"batch at benchmark sizes: {[m.n for m in ms]} schedule={schedule}")
    b = Batch([m.n for m in ms], [m.alpha for m in ms], [m.kappa for m in ms], TAU)
    for n in sorted({m.n for m in ms}):
        b.set_path(n, "fft_gs")
    b.set_graph(True)
    b.set_schedule(schedule)
    u0 = [to_dev(m.phi1()) for m in ms]
    u1 = [torch.zeros_like(t) for t in u0]
    p2 = [to_dev(0.3 * W.asymmetric_field(m.n, seed=m.n)) for m in ms]
    b.bind(u0, u1, p2)
    with b:
        b.first_step()
        b.run(4)
        for k, m in enumerate(ms):
            ref_prev, ref_cur = reference(m, 5)
            assert rel(from_dev(u1[k]), ref_cur) < 1e-11, (k, m.n)
            assert rel(from_dev(u0[k]), ref_prev) < 1e-11, (k, m.n)


@pytest.mark.parametrize("path", ["fft_gs", "dense"])
def test_batch_general_n(path):
    """Members whose N + 1 is not a power of two (the line solves' rank-(M - N) correction,
    ranks 2, 12 and 28 here, applied per line inside the batched kernels), on both paths,
    under graph replay, against the oracle after 7 steps."""
    from paper_2312_06206_amd import Batch
    _dev()
    ms = W.batch_members(6, seed=5, n_choices=(20, 62, 100))
    _say(f"batch general N: {[m.n for m in ms]} path={path}")
    b = Batch([m.n for m in ms], [m.alpha for m in ms], [m.kappa for m in ms], TAU, dense_max_n=127)
    for n in sorted({m.n for m in ms}):
        b.set_path(n, path)
    b.set_graph(True)
    u0 = [to_dev(m.phi1()) for m in ms]
    u1 = [torch.zeros_like(t) for t in u0]
    p2 = [to_dev(0.3 * W.asymmetric_field(m.n, seed=m.n)) for m in ms]
    b.bind(u0, u1, p2)
    with b:
        b.first_step()
        b.run(6)
        for k, m in enumerate(ms):
            ref_prev, ref_cur = reference(m, 7)
            assert rel(from_dev(u1[k]), ref_cur) < 1e-11, (k, m.n)
            assert rel(from_dev(u0[k]), ref_prev) < 1e-11, (k, m.n)
