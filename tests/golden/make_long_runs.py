"""Write the oracle's 1000-step runs of the large single-instance workloads as sampled
expected values (tests/golden/long_runs/N<n>_a<alpha>.npz).

Workload (one file per grid N and order alpha): Omega = (-1,1)^2, kappa = 1,
g = -sin u, tau = 1e-3, phi1 = the seeded Gaussian bump of workloads.config2 (seed 0),
phi2 = 0; the start-up step of the scheme and 999 steps after it, i.e. u^999 and
u^1000.  The run is the oracle's delta form with explicit-inverse line sweeps
(oracle.scheme.Problem.run(..., gemm=True)); nothing here calls the device library.

Stored per file (plain float64 / int64 arrays, loadable with allow_pickle=False):
  idx        flat indices i * N + j into the oracle's G[i, j] grid (i the x index): the
             centre x-line and y-line, a strided sub-grid and seeded random nodes
  prev, cur  u^999 and u^1000 at idx
  full_max   max |u| over the whole grid for (u^999, u^1000)
  full_l2    sqrt(sum u^2) over the whole grid for (u^999, u^1000)
  meta       (n, alpha, tau, steps, seed)

    python tests/golden/make_long_runs.py [N alpha] ...     # default: all nine

Floor runs (N<n>_a<alpha>_p<P>.npz, same contents): the same workload with the BCCB
embedding of L_h at size P instead of 2N.  Every P >= 2N - 1 gives the same scheme in exact
arithmetic, so the distance between the two oracle runs is the float64 rounding floor of
the 1000-step run itself (L_h u of the smooth solution loses about eps ||L_h|| / lambda_min,
and the leapfrog turns that into a phase error of the slow modes).

    python tests/golden/make_long_runs.py --embed P N alpha
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import scheme as S  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "long_runs")
STEPS = 1000
SEED = 0
ALL = [(4095, 1.5), (1023, 1.2), (1023, 1.5), (1023, 1.8), (2047, 1.5), (2047, 1.2), (2047, 1.8),
       (4095, 1.2), (4095, 1.8)]


def sample_indices(n: int) -> np.ndarray:
    """Centre lines, a sub-grid of about 32 x 32 nodes and 1024 seeded random nodes."""
    c = n // 2
    s = max(1, (n + 1) // 32)
    sub = np.arange(s // 2, n, s)
    rows = [c * n + np.arange(n),                                   # x index c, all y
            np.arange(n) * n + c,                                   # all x, y index c
            (sub[:, None] * n + sub[None, :]).ravel(),
            np.random.default_rng(12345).integers(0, n * n, 1024)]
    return np.unique(np.concatenate(rows)).astype(np.int64)


def path_for(n: int, alpha: float, embed: int | None = None) -> str:
    return os.path.join(OUT, f"N{n}_a{alpha}" + ("" if embed is None else f"_p{embed}") + ".npz")


def make(n: int, alpha: float, embed: int | None = None) -> None:
    wl = W.config2(n, alpha, seed=SEED, steps=STEPS)
    t0 = time.time()
    P = S.Problem(alpha=wl.alpha, kappa=wl.kappa, n=n, tau=wl.tau, embed=embed)
    phi1 = wl.phi1()
    phi2 = np.zeros_like(phi1)

    def progress(k, prev, cur):
        if k % 100 == 0:
            print(f"  N={n} alpha={alpha}: step {k} ({time.time() - t0:.0f} s)", flush=True)

    prev, cur = P.run(phi1, phi2, STEPS, gemm=True, callback=progress)
    idx = sample_indices(n)
    os.makedirs(OUT, exist_ok=True)
    out = path_for(n, alpha, embed)
    tmp = out + ".tmp.npz"
    np.savez(tmp, idx=idx, prev=prev.ravel()[idx], cur=cur.ravel()[idx],
             full_max=np.array([np.abs(prev).max(), np.abs(cur).max()]),
             full_l2=np.array([np.sqrt(np.sum(prev * prev)), np.sqrt(np.sum(cur * cur))]),
             meta=np.array([n, alpha, wl.tau, STEPS, SEED], dtype=np.float64))
    os.replace(tmp, out)
    print(f"N={n} alpha={alpha} embed={embed}: done in {time.time() - t0:.0f} s, {idx.size} samples", flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    embed = None
    if args[:1] == ["--embed"]:
        embed, args = int(args[1]), args[2:]
    jobs = [(int(args[i]), float(args[i + 1])) for i in range(0, len(args), 2)] if args else ALL
    for n, a in jobs:
        make(n, a, embed)
