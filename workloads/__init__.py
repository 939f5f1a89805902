"""Seeded synthetic inputs for the S-ADI solver: initial data, lines, parameters.

This module only samples input functions on the grid and draws seeded random
numbers; it holds none of the scheme's arithmetic.  Both the device path's tests
and benchmark and the CPU oracle's tests take their inputs from here.

Conventions: the interior grid of Omega = (a,b)^2 has N nodes per direction,
x_i = a + i h with h = (b-a)/(N+1), i = 1..N (the paper's grid, section
"Construction of S-ADI scheme").  Grid functions are returned as float64 arrays
G[i, j] = f(x_i, y_j) (i the x index).  The device library stores the same grid
function with x fastest in memory, i.e. as G.T (row j holds the x-line y = y_j).
"""
from __future__ import annotations

import dataclasses

import numpy as np


def nodes(a: float, b: float, n: int) -> np.ndarray:
    h = (b - a) / (n + 1)
    return a + h * np.arange(1, n + 1)


def mesh(a: float, b: float, n: int):
    x = nodes(a, b, n)
    return np.meshgrid(x, x, indexing="ij")


def gaussian_bump(n: int, domain=(-1.0, 1.0), width: float = 0.2, center=(0.0, 0.0),
                  amplitude: float = 1.0) -> np.ndarray:
    """amplitude * exp(-((x-cx)^2 + (y-cy)^2) / (2 width^2))."""
    X, Y = mesh(domain[0], domain[1], n)
    return amplitude * np.exp(-((X - center[0]) ** 2 + (Y - center[1]) ** 2) / (2.0 * width * width))


def config1_phi1(n: int = 63, domain=(-1.0, 1.0)) -> np.ndarray:
    """exp(-10 (x^2 + y^2)): the small single-instance workload's initial displacement."""
    X, Y = mesh(domain[0], domain[1], n)
    return np.exp(-10.0 * (X ** 2 + Y ** 2))


def seeded_width(seed: int) -> float:
    """Gaussian width drawn U[0.05, 0.3] from the seed."""
    return float(np.random.default_rng(seed).uniform(0.05, 0.3))


def seeded_bump(n: int, seed: int, domain=(-1.0, 1.0)) -> np.ndarray:
    """Centred Gaussian bump with a seeded width (large single-instance workloads)."""
    return gaussian_bump(n, domain, width=seeded_width(seed))


def asymmetric_field(n: int, seed: int, domain=(-1.0, 1.0)) -> np.ndarray:
    """Sum of three off-centre anisotropic bumps with seeded centres/widths/signs:
    not symmetric under x <-> y or reflections, so layout mistakes show up."""
    rng = np.random.default_rng(seed)
    X, Y = mesh(domain[0], domain[1], n)
    L = domain[1] - domain[0]
    out = np.zeros_like(X)
    for _ in range(3):
        cx, cy = domain[0] + L * rng.uniform(0.25, 0.75, size=2)
        wx, wy = L * rng.uniform(0.04, 0.15, size=2)
        amp = rng.uniform(0.3, 1.0) * rng.choice([-1.0, 1.0])
        out += amp * np.exp(-((X - cx) ** 2) / (2 * wx * wx) - ((Y - cy) ** 2) / (2 * wy * wy))
    return out


def random_lines(nlines: int, n: int, seed: int) -> np.ndarray:
    """(nlines, n) standard-normal right-hand sides for line solves."""
    return np.random.default_rng(seed).standard_normal((nlines, n))


def sech(x):
    return 1.0 / np.cosh(np.minimum(np.abs(x), 700.0))


def sine_gordon_data(n: int, domain=(-10.0, 10.0)):
    """First example of the paper: phi1 = 0, phi2 = sech(sqrt(x^2 + y^2))."""
    X, Y = mesh(domain[0], domain[1], n)
    return np.zeros_like(X), sech(np.sqrt(X ** 2 + Y ** 2))


def klein_gordon_data(n: int, domain=(-10.0, 10.0), amplitude: float = 2.0):
    """Second example of the paper: phi1 = A sech(cosh(x^2 + y^2)), phi2 = 0.
    The printed formula has A = 1; A = 2 is the reading that reproduces the
    paper's tabulated errors."""
    X, Y = mesh(domain[0], domain[1], n)
    return amplitude * sech(np.cosh(np.minimum(X ** 2 + Y ** 2, 700.0))), np.zeros_like(X)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int
    alpha: float
    kappa: float
    tau: float
    steps: int
    domain: tuple = (-1.0, 1.0)
    g: str = "neg_sin"
    seed: int = 0

    def phi1(self) -> np.ndarray:
        if self.name == "config1":
            return config1_phi1(self.n, self.domain)
        return seeded_bump(self.n, self.seed, self.domain)

    def phi2(self) -> np.ndarray:
        return np.zeros((self.n, self.n))


# the single-instance workloads (Omega = (-1,1)^2, kappa = 1, g = -sin u, phi2 = 0)
CONFIG1 = Workload("config1", n=63, alpha=1.5, kappa=1.0, tau=1.0 / 64, steps=64)


def config2(n: int = 4095, alpha: float = 1.5, seed: int = 0, steps: int = 1000) -> Workload:
    assert n in (1023, 2047, 4095)
    return Workload(f"sadi_N{n}_a{alpha}", n=n, alpha=alpha, kappa=1.0, tau=1e-3, steps=steps, seed=seed)


@dataclasses.dataclass(frozen=True)
class BatchMember:
    """One problem of a batch: Omega = (-1,1)^2, g = -sin u, phi2 = 0 unless given, a
    Gaussian bump with seeded width and centre as phi1."""
    n: int
    alpha: float
    kappa: float
    width: float
    center: tuple

    def phi1(self, domain=(-1.0, 1.0)) -> np.ndarray:
        return gaussian_bump(self.n, domain, width=self.width, center=self.center)


def batch_members(count: int, seed: int, n_choices=(127, 255, 511, 1023)) -> list:
    """Seeded batch of uneven problems: N uniform over n_choices, alpha ~ U(1.1, 1.9),
    kappa ~ U(0.5, 2), bump width ~ U(0.05, 0.3), centre ~ U(-0.3, 0.3)^2."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(n_choices))
        out.append(BatchMember(n=n, alpha=float(rng.uniform(1.1, 1.9)), kappa=float(rng.uniform(0.5, 2.0)),
                               width=float(rng.uniform(0.05, 0.3)),
                               center=(float(rng.uniform(-0.3, 0.3)), float(rng.uniform(-0.3, 0.3)))))
    return out
