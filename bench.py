#!/usr/bin/env python3
"""Benchmark: S-ADI grid-point-steps/s on one MI355X.

Workload (one GPU): Omega = (-1,1)^2, N = 4095 interior nodes per direction, alpha = 1.5,
kappa = 1, g(u) = -sin u, phi1 a centred Gaussian bump whose width is drawn U[0.05, 0.3]
from the seed, phi2 = 0, tau = 1e-3.  A "step" is one whole S-ADI step (BTTB product,
right-hand side, x-line and y-line Gohberg-Semencul solves, leapfrog update).  The
state is resident in HBM before the timed region; setup is timed separately.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line.  `value` comes from one timed region of exactly K steps; `repeats`
holds further K-step runs (on a copy of the state) and their median.  `roofline` covers
the kernel with the largest share of the step: algorithmic bytes per launch over its
mean launch time, from HIP events on the library's stream in a separate run of the same
launches (events inside the timed region would cost device time), beside the
counter-measured bytes when the committed counters match the kernel sources.
`cpu_baseline` times the FP64 CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
FP64_VALU_PEAK_TFLOPS = 78.6     # MI355X FP64 vector: 256 CUs x 4 SIMDs x 16 lanes x 2 (fma) x 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4.0   # wave64 VALU instructions per second (4 cycles each per SIMD)
METRIC = "S-ADI grid-point-steps/s at N=4095 (FP64 vs FP32+refine), % HBM roofline"


def algorithmic_bytes(n: int) -> dict:
    """Compulsory HBM bytes per launch of each kernel in a run of steps (float64 state,
    complex128 half spectrum of N rows x (M+1) columns, (M+1)^2 BCCB eigenvalues).  A run
    has three kernels per step: the y-sweep kernel also forms u^{n+1} and the next step's
    row transform (on the transposed grid); the row transform of its own is launched once
    per run."""
    m = n + 1
    pts = n * n
    spec = n * (m + 1) * 16
    return {
        "rows_fwd": pts * 8 + spec,                          # once per run: read u, write spectrum
        "cols_conv": 2 * spec + (m + 1) * (m + 1) * 8,      # read+write spectrum, eigenvalues
        "rows_rhs_gs": spec + pts * 8 + pts * 8,            # read spectrum, u; write X
        # read X, u^n, u^{n-1}; write u^{n+1} and the next spectrum
        "cols_gs_fwd": 4 * pts * 8 + spec,
    }


STEP_KERNELS = ("cols_conv", "rows_rhs_gs", "cols_gs_fwd")


def alu_view(kernel: str, avg_ms: float):
    """FP64 vector-ALU view of a step kernel from committed rocprofv3 VALU counts (None if
    they were not taken on the current kernel sources)."""
    try:
        from paper_2312_06206_amd import profiling
        v = profiling.valu_for(kernel)
    except Exception:
        v = None
    if not v:
        return None
    t = avg_ms * 1e-3
    return {"bound": "alu", "kernel": kernel, "fp64_flops_per_launch": v["fp64_flops"],
            "achieved": v["fp64_flops"] / t / 1e12, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": v["fp64_flops"] / t / 1e12 / FP64_VALU_PEAK_TFLOPS,
            "valu_insts_per_launch": v["SQ_INSTS_VALU"],
            "valu_issue_frac": v["SQ_INSTS_VALU"] / t / VALU_ISSUE_PEAK,
            "source": "profiles/valu_counters_N4095.json (rocprofv3 SQ_INSTS_VALU*)"}


def traffic_record(kernel: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were taken on the
    current kernel sources (else None)."""
    try:
        from paper_2312_06206_amd import profiling
        return profiling.traffic_for(kernel)
    except Exception:
        return None


def cpu_baseline(wl, sample_steps: int) -> dict:
    import numpy as np
    import scipy.fft
    from threadpoolctl import threadpool_limits, threadpool_info

    from oracle import scheme as S

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    with threadpool_limits(limits=threads), scipy.fft.set_workers(threads):
        P = S.Problem(alpha=wl.alpha, kappa=wl.kappa, n=wl.n, tau=wl.tau, g=wl.g, domain=wl.domain)
        u0 = wl.phi1()
        u1 = P.first_step(u0, wl.phi2())       # untimed: also builds the explicit H^-1
        prev, cur = u0, u1
        t0 = time.perf_counter()
        for _ in range(sample_steps):
            prev, cur = cur, P.step_delta(prev, cur, gemm=True)
        dt = time.perf_counter() - t0
        blas = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    pts = wl.n * wl.n * sample_steps
    # one thread: two further steps of the same sample
    with threadpool_limits(limits=1), scipy.fft.set_workers(1):
        t1 = time.perf_counter()
        for _ in range(2):
            prev, cur = cur, P.step_delta(prev, cur, gemm=True)
        dt1 = time.perf_counter() - t1
    return {"value": pts / dt, "unit": "grid-point-steps/s", "cores": int(max(blas, threads)), "kind": "oracle",
            "sample": f"{sample_steps} steps n>=1 of the same N={wl.n} workload after the start-up step "
                      f"(setup and explicit H^-1 excluded), {dt:.1f} s wall, numpy/scipy FP64 with "
                      f"{threads} FFT workers and BLAS threads",
            "single_thread_value": wl.n * wl.n * 2 / dt1,
            "single_thread_sample": f"2 further steps, 1 FFT worker and 1 BLAS thread, {dt1:.1f} s wall"}


def stored_oracle_run(n: int, alpha: float, seed: int):
    """The oracle's own 1000-step run of this workload, if one is stored (written by
    tests/golden/make_long_runs.py from the oracle alone), else None."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "long_runs", f"N{n}_a{alpha}.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        ref = {k: z[k] for k in z.files}
    if int(ref["meta"][4]) != seed:
        return None
    return ref


def oracle_run_errors(s, wl, ref, precisions) -> dict:
    """Each precision's u^999 and u^1000 (start-up step + 999 steps through sadi_run) against
    the oracle's stored run: max error over the stored sample nodes relative to max |u| of
    the oracle's whole grid."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    out = {}
    for prec in precisions:
        s.set_options(wl.g, 0.0, prec)
        a = torch.from_numpy(np.ascontiguousarray(wl.phi1().T)).to(dev)
        b = s.first_step(a, torch.zeros_like(a))
        s.run(a, b, 999)
        errs = []
        for k, t in enumerate((a, b)):
            g = t.cpu().numpy().T.ravel()
            errs.append(float(np.abs(g[ref["idx"]] - ref["prev" if k == 0 else "cur"]).max() / ref["full_max"][k]))
        out[prec] = max(errs)
    s.set_options(wl.g, 0.0, "fp64")
    return out


def attainable_copy_rate() -> dict:
    """Attainable HBM rate of a plain streaming copy: torch's device copy over six rotating
    256 MiB buffer pairs (3 GiB in all, so the 256 MB Infinity Cache cannot serve the
    reads), bytes read + written over the elapsed time of 24 copies."""
    import torch
    n = (256 << 20) // 8
    src = [torch.ones(n, dtype=torch.float64, device="cuda:0") for _ in range(6)]
    dst = [torch.empty_like(a) for a in src]
    for k in range(6):
        dst[k].copy_(src[k])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 24
    for k in range(reps):
        dst[k % 6].copy_(src[(k + 3) % 6])
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3
    gbs = 2.0 * n * 8 * reps / sec / 1e9
    del src, dst
    return {"copy_GBps": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS,
            "method": "torch copy_ of 256 MiB float64 buffers, 6 rotating pairs, 24 copies, read + write bytes"}


def batched_leg(seed: int, count: int, steps: int, unbatched_sample: int) -> dict:
    """Uneven batch: `count` problems with N uniform over {127, 255, 511, 1023}, alpha ~
    U(1.1, 1.9), kappa ~ U(0.5, 2), seeded Gaussian phi1, phi2 = 0, tau = 1e-3; autotuned
    line-sweep path per N, `steps` steps replayed from a HIP graph.  Compared with the same
    problems run one by one through the single-instance FP64 path."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2312_06206_amd import Batch, Solver

    dev = torch.device("cuda:0")
    ms = W.batch_members(count, seed)
    tau = 1e-3
    t0 = time.perf_counter()
    b = Batch([m.n for m in ms], [m.alpha for m in ms], [m.kappa for m in ms], tau, dense_max_n=1023)
    setup_s = time.perf_counter() - t0
    u0 = [torch.from_numpy(np.ascontiguousarray(m.phi1().T)).to(dev) for m in ms]
    u1 = [torch.zeros_like(t) for t in u0]
    p2 = [torch.zeros_like(t) for t in u0]
    b.bind(u0, u1, p2)
    t0 = time.perf_counter()
    groups = b.tune(steps=5)
    tune_s = time.perf_counter() - t0
    schedule, ms_groups, ms_lists = b.schedule()
    b.set_graph(True)
    b.first_step()
    b.run(4)                                   # warm-up (captures the graph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    finite = all(bool(torch.isfinite(t).all().item()) for t in u1)
    pts = sum(m.n * m.n for m in ms)
    b.close()

    # the same problems one at a time (sampled steps per instance, extrapolated)
    one_ms = 0.0
    for m in ms:
        s = Solver(m.alpha, m.kappa, m.n, tau)
        a = torch.from_numpy(np.ascontiguousarray(m.phi1().T)).to(dev)
        c = s.first_step(a, torch.zeros_like(a))
        s.run(a, c, 2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.run(a, c, unbatched_sample)
        torch.cuda.synchronize()
        one_ms += 1e3 * (time.perf_counter() - t1) / unbatched_sample
        s.close()
    batch_ms = 1e3 * dt / steps
    # compulsory bytes of a step of every instance on the Gohberg-Semencul path (the three
    # kernels of a run step); dense-path groups move more (two N^3 products re-read H^-1)
    alg = sum(sum(algorithmic_bytes(m.n)[k] for k in STEP_KERNELS) for m in ms)
    alg_gbs = alg / (batch_ms * 1e-3) / 1e9
    return {"workload": f"{count} instances, N uniform over {{127,255,511,1023}}, alpha~U(1.1,1.9), "
                        f"kappa~U(0.5,2), seeded Gaussian phi1, phi2=0, tau=1e-3, seed {seed}",
            "steps": steps, "ms_per_step": batch_ms, "value": pts * steps / dt, "unit": "grid-point-steps/s",
            "one_by_one_ms_per_step": one_ms, "speedup_vs_one_by_one": one_ms / batch_ms,
            "groups": groups, "schedule": schedule,
            "tuned_ms_per_step": {"groups": ms_groups, "work_lists": ms_lists},
            "roofline": {"bound": "hbm", "algorithmic_bytes_per_step": alg, "achieved": alg_gbs,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": alg_gbs / HBM_PEAK_GBS},
            "setup_s": setup_s, "tune_s": tune_s, "graph": True, "finite": finite,
            "one_by_one_sample_steps": unbatched_sample}


def adjoint_leg(seed: int) -> dict:
    """Gradient of J = ||u(T) - u_obs||^2 with respect to phi1 and kappa: N = 511,
    alpha = 1.6, 500 steps, tau = 1e-3, u_obs from kappa = 1.3 and a seeded bump, the
    gradient at kappa = 1 and another seeded bump; checkpoints every 50 steps."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2312_06206_amd import Solver
    from paper_2312_06206_amd.adjoint import sadi_loop

    dev = torch.device("cuda:0")
    n, alpha, tau, steps = 511, 1.6, 1e-3, 500
    to_dev = lambda G: torch.from_numpy(np.ascontiguousarray(G.T)).to(dev)
    with Solver(alpha, 1.3, n, tau) as s:
        a = to_dev(W.seeded_bump(n, seed))
        u_obs = s.first_step(a, torch.zeros_like(a))
        s.run(a, u_obs, steps - 1)
    for _ in range(2):   # the first pass warms up; the second is timed (solver set-up included)
        x = to_dev(W.seeded_bump(n, seed + 1)).requires_grad_(True)
        k = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        uK = sadi_loop(x, k, alpha, n, tau, steps, checkpoint=50)
        J = ((uK - u_obs) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
    return {"workload": "N=511, alpha=1.6, 500 steps, tau=1e-3, loss ||u(T)-u_obs||^2, u_obs from kappa=1.3, "
                        "gradient w.r.t. kappa and phi1 at kappa=1, checkpoint every 50 steps",
            "forward_s": t1 - t0, "backward_s": t2 - t1, "backward_over_forward": (t2 - t1) / (t1 - t0),
            "loss": float(J.item()), "dJ_dkappa": float(k.grad.item()),
            "grad_phi1_norm": float(x.grad.norm().item())}


def config_sweep(seed: int, steps: int) -> list:
    """The plain FP64 configuration over N in {1023, 2047, 4095} and alpha in {1.2, 1.5, 1.8}
    (kappa = 1, g = -sin u, seeded Gaussian phi1, phi2 = 0, tau = 1e-3): ms/step of a run
    after a warm-up run, and the step's algorithmic HBM rate."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2312_06206_amd import Solver

    dev = torch.device("cuda:0")
    out = []
    for n in (1023, 2047, 4095):
        alg = algorithmic_bytes(n)
        step_bytes = sum(alg[k] for k in STEP_KERNELS)
        for alpha in (1.2, 1.5, 1.8):
            wl = W.config2(n, alpha, seed=seed, steps=steps)
            with Solver(wl.alpha, wl.kappa, wl.n, wl.tau, wl.domain, g=wl.g) as s:
                u0 = torch.from_numpy(np.ascontiguousarray(wl.phi1().T)).to(dev)
                u1 = s.first_step(u0, torch.zeros_like(u0))
                s.run(u0, u1, 10)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.run(u0, u1, steps)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                out.append({"N": n, "alpha": alpha, "steps": steps, "ms_per_step": 1e3 * dt / steps,
                            "value": n * n * steps / dt, "step_alg_GBps": step_bytes * steps / dt / 1e9,
                            "step_alg_frac": step_bytes * steps / dt / 1e9 / HBM_PEAK_GBS,
                            "finite": bool(torch.isfinite(u1).all().item())})
    return out


# the paper's own CPU timings (seconds, S-ADI column) and printed errors for two of its
# workloads: Table 1 (sine-Gordon, h = 1/40, N = 799) and Table 3 (Klein-Gordon, h = 1/50,
# N = 999), alpha = 1.5, Omega = (-10, 10)^2
PAPER_ROWS = [
    {"table": "Table 1", "g": "neg_sin", "n": 799, "T": 5.0, "tau": 1.0 / 80, "paper_cpu_s": 223.1865,
     "paper_error1": 1.4136e-4},
    {"table": "Table 3", "g": "neg_cube", "n": 999, "T": 8.0, "tau": 1.0 / 50, "paper_cpu_s": 430.4121,
     "paper_error1": 6.7184e-3},
]


def paper_leg() -> list:
    """Two of the paper's own experiments run as printed (kappa = 1): the GPU time of the
    run the paper timed, and Error_1 against the run with tau/2."""
    import math

    import numpy as np
    import torch

    import workloads as W
    from paper_2312_06206_amd import Solver

    dev = torch.device("cuda:0")
    out = []
    for row in PAPER_ROWS:
        n, alpha = row["n"], 1.5
        data = W.sine_gordon_data if row["g"] == "neg_sin" else W.klein_gordon_data
        phi1, phi2 = data(n)
        finals, secs = {}, {}
        for tau in (row["tau"], row["tau"] / 2):
            steps = round(row["T"] / tau)
            with Solver(alpha, 1.0, n, tau, (-10.0, 10.0), g=row["g"]) as s:
                a = torch.from_numpy(np.ascontiguousarray(phi1.T)).to(dev)
                p2 = torch.from_numpy(np.ascontiguousarray(phi2.T)).to(dev)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                b = s.first_step(a, p2)
                s.run(a, b, steps - 1)
                torch.cuda.synchronize()
                secs[tau] = time.perf_counter() - t0
                finals[tau] = b.cpu().numpy()
        h = 20.0 / (n + 1)
        err = math.sqrt(h * h * float(np.sum((finals[row["tau"]] - finals[row["tau"] / 2]) ** 2)))
        steps = round(row["T"] / row["tau"])
        out.append({"workload": f"{row['table']}: g={row['g']}, alpha=1.5, N={n}, tau={row['tau']:.6g}, "
                                f"{steps} steps, Omega=(-10,10)^2",
                    "gpu_s": secs[row["tau"]], "paper_cpu_s": row["paper_cpu_s"],
                    "ratio_paper_over_gpu": row["paper_cpu_s"] / secs[row["tau"]],
                    "error1": err, "paper_error1": row["paper_error1"],
                    "note": "the paper names no hardware for its timings: context only"})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=4095)
    ap.add_argument("--alpha", type=float, default=1.5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=20)
    ap.add_argument("--no-variants", action="store_true", help="skip the FP32 / FP32+refine runs")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched (uneven N) leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the gradient (adjoint) leg")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper's own workloads")
    ap.add_argument("--no-sweep", action="store_true", help="skip the N x alpha sweep of the FP64 configuration")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the 1000-step runs compared with the oracle's stored run")
    ap.add_argument("--repeats", type=int, default=5,
                    help="further timed runs of K steps, reported with their median beside value")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain device copies of 1 GiB (calibrates the HBM byte counters)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(4):
            torch.mul(a, 1.0, out=b)      # plain elementwise kernel: reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8, "copies": 4}))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the slab decomposition across GPUs is designed but not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2312_06206_amd import Solver

    dev = torch.device("cuda:0")
    wl = W.config2(args.n, args.alpha, seed=args.seed, steps=args.steps)

    t0 = time.perf_counter()
    s = Solver(wl.alpha, wl.kappa, wl.n, wl.tau, wl.domain, g=wl.g)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0     # the first context of the process: includes one-time init
    t0 = time.perf_counter()
    Solver(wl.alpha, wl.kappa, wl.n, wl.tau, wl.domain, g=wl.g).close()
    torch.cuda.synchronize()
    setup_warm_s = time.perf_counter() - t0

    u0 = torch.from_numpy(np.ascontiguousarray(wl.phi1().T)).to(dev)
    phi2 = torch.zeros_like(u0)
    u1 = s.first_step(u0, phi2)
    steps = args.steps   # exactly K: an odd count ends the run with a swap instead of a transpose
    if args.warmup:
        s.run(u0, u1, args.warmup)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    s.run(u0, u1, steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    finite = bool(torch.isfinite(u1).all().item())
    # further runs of the same K steps on a copy of the state (u0, u1 stay at step K for the
    # precision variants' comparison below): their median beside the single timed region
    repeat_ms = []
    if args.repeats:
        ra, rb = u0.clone(), u1.clone()
        for _ in range(args.repeats):
            t0r = time.perf_counter()
            s.run(ra, rb, steps)
            torch.cuda.synchronize()
            repeat_ms.append(1e3 * (time.perf_counter() - t0r) / steps)
        finite = finite and bool(torch.isfinite(rb).all().item())
        del ra, rb
    # per-kernel device times from a separate run bracketed by events (each event costs a
    # few microseconds of device time, so the timed run above records none)
    state = (u0.clone(), u1.clone())
    s.set_kernel_timing(True)
    s.run(state[0], state[1], min(steps, 200))
    ktimes = s.kernel_times()
    s.set_kernel_timing(False)
    del state
    ktimes["cols_gs_fwd"] = ktimes.pop("cols_gs")   # slot 3 of a run: y-sweep + next row transform

    # precision variants on the same workload: speed, and the final state's difference from
    # the FP64 path; below, every precision against the oracle's stored 1000-step run
    variants = {}
    if not args.no_variants:
        ref_final = u1.clone()
        for prec in ("fp32_refine", "fp32"):
            s.set_options(wl.g, 0.0, prec)
            v0 = torch.from_numpy(np.ascontiguousarray(wl.phi1().T)).to(dev)
            v1 = s.first_step(v0, phi2)
            if args.warmup:
                s.run(v0, v1, args.warmup)
            torch.cuda.synchronize()
            t0v = time.perf_counter()
            s.run(v0, v1, steps)
            torch.cuda.synchronize()
            dtv = time.perf_counter() - t0v
            err = float((v1 - ref_final).abs().max() / ref_final.abs().max())
            variants[prec] = {"ms_per_step": 1e3 * dtv / steps, "value": wl.n * wl.n * steps / dtv,
                              "speedup_vs_fp64": dt / dtv, "rel_err_vs_fp64_path": err,
                              "steps": steps + args.warmup + 1}
        s.set_options(wl.g, 0.0, "fp64")
    # every precision against the oracle's own 1000-step run of this workload
    ref = None if args.no_accuracy else stored_oracle_run(wl.n, wl.alpha, args.seed)
    oracle_errs = None
    if ref is not None:
        oracle_errs = oracle_run_errors(s, wl, ref, ["fp64"] + list(variants))
        for prec, e in oracle_errs.items():
            if prec in variants:
                variants[prec]["rel_err_vs_oracle_run_1000"] = e

    copy = attainable_copy_rate()

    n = wl.n
    value = n * n * steps / dt
    ms_per_step = 1e3 * dt / steps
    alg = algorithmic_bytes(n)
    dom = max(STEP_KERNELS, key=lambda k: ktimes[k][0])
    avg_ms = ktimes[dom][0] / max(ktimes[dom][1], 1)
    achieved = alg[dom] / (avg_ms * 1e-3) / 1e9
    total_alg = sum(alg[k] for k in STEP_KERNELS)   # the run's one row transform excluded
    step_gbs = total_alg / (ms_per_step * 1e-3) / 1e9
    dom_traffic = traffic_record(dom)
    step_tr = [traffic_record(k) for k in STEP_KERNELS]
    step_traffic = sum(step_tr) if all(step_tr) else None

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"S-ADI FP64 single instance, Omega=(-1,1)^2, N={n}, alpha={wl.alpha}, kappa=1, "
                               f"g=-sin u, seeded Gaussian phi1 (width {W.seeded_width(args.seed):.4f}), phi2=0, "
                               f"tau=1e-3",
                   "N": n, "alpha": wl.alpha, "tau": wl.tau, "precision": "fp64", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": dom_traffic,
                     # the measured (counter) bytes over the same launch time
                     "traffic_GBps": dom_traffic / (avg_ms * 1e-3) / 1e9 if dom_traffic else None,
                     # the same against what a plain streaming copy attains on this machine
                     "attainable_GBps": copy["copy_GBps"], "frac_of_attainable": achieved / copy["copy_GBps"]},
        "attainable_copy": copy,
        "step_roofline": {"algorithmic_bytes_per_step": total_alg, "achieved_GBps": step_gbs,
                          "frac": step_gbs / HBM_PEAK_GBS, "frac_of_attainable": step_gbs / copy["copy_GBps"],
                          "counter_bytes_per_step": step_traffic,
                          "counter_GBps": step_traffic / (ms_per_step * 1e-3) / 1e9 if step_traffic else None},
        "alu_view": alu_view(dom, avg_ms),
        "kernels_ms_avg": {k: v[0] / max(v[1], 1) for k, v in ktimes.items() if k in STEP_KERNELS},
        "repeats": {"ms_per_step": repeat_ms,
                    "median_ms_per_step": float(np.median(repeat_ms)) if repeat_ms else None},
        "setup_s": setup_s,
        "setup_warm_s": setup_warm_s,
        "finite": finite,
        "precision_variants": variants,
        "rel_err_vs_oracle_run_1000": None if oracle_errs is None else oracle_errs["fp64"],
    }
    s.close()
    if not args.no_batched:
        out["batched"] = batched_leg(args.seed, args.batch_count, args.batch_steps, 20)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(args.seed)
    if not args.no_paper:
        out["paper_workloads"] = paper_leg()
    if not args.no_sweep:
        out["config_sweep"] = config_sweep(args.seed, 300)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
