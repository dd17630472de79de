"""Seeded synthetic inputs for the 2-D curved-space Dirac solves.

This module only draws parameters and builds initial spinors (Gaussian
packets); it holds none of the time-stepping arithmetic.  Both the HIP path
(through ``bench.py`` and the tests) and the CPU oracle consume what it
returns, so the two sides always see identical inputs.

Spinor arrays are complex128 of shape ``(n2, n1, 2)``: axis 0 is y, axis 1 is
x, axis 2 the spinor component (the host layout of the C ABI).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

METRIC_FLAT = 0
METRIC_GAUSS_BUMP = 1
METRIC_PAPER_EXP3 = 2
METRIC_FIELDS = 3
SPIN_NONE = 0
SPIN_PAPER = 1
SPIN_2P1 = 2


@dataclass
class SolveSpec:
    """One solve: grid, physics, metric model, absorbing layer and initial packet."""
    n1: int
    n2: int
    a1: float = 20.0
    a2: float = 20.0
    dt: float = 0.01
    c: float = 1.0
    m: float = 1.0
    metric: int = METRIC_FLAT
    spin: int = SPIN_NONE
    bump_A: float = 0.0
    bump_s: float = 1.0
    pml_width: int = 0
    pml_type: int = 1
    pml_sigma0: float = 1.0
    pml_theta: float = 0.0
    x0: tuple = (0.0, 0.0)
    k0: tuple = (1.0, 0.0)
    width: float = 4.0
    comp: tuple = (1.0, 0.0)
    steps: int = 100
    seed: int | None = None
    extra: dict = field(default_factory=dict)

    def as_dict(self):
        return asdict(self)


def gaussian_packet(n1: int, n2: int, a1: float, a2: float, x0=(0.0, 0.0), k0=(1.0, 0.0),
                    width: float = 4.0, comp=(1.0, 0.0)) -> np.ndarray:
    """exp(-|x - x0|^2 / (2 width^2)) exp(i k0 . x) times the constant spinor comp,
    sampled at x_i = -a1 + i h1, y_j = -a2 + j h2."""
    x = -a1 + (2.0 * a1 / n1) * np.arange(n1)
    y = -a2 + (2.0 * a2 / n2) * np.arange(n2)
    X, Y = np.meshgrid(x, y)
    env = np.exp(-((X - x0[0]) ** 2 + (Y - x0[1]) ** 2) / (2.0 * width * width))
    ph = np.exp(1j * (k0[0] * X + k0[1] * Y))
    f = env * ph
    out = np.empty((n2, n1, 2), dtype=np.complex128)
    out[..., 0] = comp[0] * f
    out[..., 1] = comp[1] * f
    return out


def gaussian_packet3(n1: int, n2: int, n3: int, a1: float, a2: float, a3: float, x0=(0.0, 0.0, 0.0),
                     k0=(1.0, 0.0, 0.0), width: float = 2.0, comp=(1.0, 0.0, 0.0, 0.0)) -> np.ndarray:
    """3-D packet exp(-|x - x0|^2 / (2 width^2)) exp(i k0 . x) times a constant
    4-spinor, shape (n3, n2, n1, 4), x fastest."""
    ax = [-a + (2.0 * a / n) * np.arange(n) for n, a in ((n1, a1), (n2, a2), (n3, a3))]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    f = (np.exp(-((X - x0[0]) ** 2 + (Y - x0[1]) ** 2 + (Z - x0[2]) ** 2) / (2.0 * width * width))
         * np.exp(1j * (k0[0] * X + k0[1] * Y + k0[2] * Z)))
    return np.stack([c * f for c in comp], axis=-1)


def initial_spinor(s: SolveSpec) -> np.ndarray:
    return gaussian_packet(s.n1, s.n2, s.a1, s.a2, s.x0, s.k0, s.width, s.comp)


def random_spinor(n1: int, n2: int, seed: int) -> np.ndarray:
    """Smooth-free random data (normal re/im parts) for stage-parity checks."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n2, n1, 2)) + 1j * rng.standard_normal((n2, n1, 2))


# --- the flat 64^2 packet solve --------------------------------------------------

def flat_small(n: int = 64, steps: int = 100) -> SolveSpec:
    """Flat space, n x n periodic grid on [-20,20)^2, c = 1, m = 1, packet of width 4
    at x0 = 0 with k0 = (1, 0) in component 0, dt = 0.01, no absorbing layer."""
    return SolveSpec(n1=n, n2=n, a1=20.0, a2=20.0, dt=0.01, c=1.0, m=1.0, metric=METRIC_FLAT,
                     spin=SPIN_NONE, x0=(0.0, 0.0), k0=(1.0, 0.0), width=4.0, comp=(1.0, 0.0),
                     steps=steps)


# --- the strained-graphene-shaped curved solve ------------------------------------

def bump_draw(seed: int):
    """Bump amplitude A ~ U[0.5, 2], width s ~ U[2, 6], packet momentum |k0| ~ U[1, 4]
    at a uniform angle, packet start x0 = -8 k0/|k0| so that it crosses the bump."""
    rng = np.random.default_rng(seed)
    A = float(rng.uniform(0.5, 2.0))
    s = float(rng.uniform(2.0, 6.0))
    kmag = float(rng.uniform(1.0, 4.0))
    ang = float(rng.uniform(0.0, 2.0 * math.pi))
    k0 = (kmag * math.cos(ang), kmag * math.sin(ang))
    x0 = (-8.0 * math.cos(ang), -8.0 * math.sin(ang))
    return A, s, k0, x0


def curved_bump(n: int = 512, seed: int = 1909, steps: int = 2000, m: float = 0.0,
                pml_width: int | None = None) -> SolveSpec:
    """Gaussian out-of-plane bump h = A exp(-r^2/s^2) on [-20,20)^2 (static sheet
    metric, conformal spin connection), absorbing layer of n/16 points per side
    (32 at n = 512; type I, sigma0 = 1, theta = 0), packet of width 2, c = 1,
    dt = 0.01."""
    A, s, k0, x0 = bump_draw(seed)
    return SolveSpec(n1=n, n2=n, a1=20.0, a2=20.0, dt=0.01, c=1.0, m=m, metric=METRIC_GAUSS_BUMP,
                     spin=SPIN_2P1, bump_A=A, bump_s=s,
                     pml_width=(n // 16 if pml_width is None else pml_width), pml_type=1,
                     pml_sigma0=1.0, pml_theta=0.0, x0=x0, k0=k0, width=2.0, comp=(1.0, 0.0),
                     steps=steps, seed=seed)


def paper_exp3(n: int = 512, steps: int = 400) -> SolveSpec:
    """Numerical Experiment 3 of the paper: [-5,5]^2, Phi = exp(-0.01|x|^2),
    Psi = exp(-0.005|x|^2), packet exp(-|x|^2/2 + i k0.x), k0 = (5, 5), dt = 1.14e-4,
    spin connection from Phi; mass not stated by the paper (m = 1 taken)."""
    return SolveSpec(n1=n, n2=n, a1=5.0, a2=5.0, dt=1.14e-4, c=1.0, m=1.0, metric=METRIC_PAPER_EXP3,
                     spin=SPIN_PAPER, x0=(0.0, 0.0), k0=(5.0, 5.0), width=1.0, comp=(1.0, 0.0),
                     steps=steps)


def batch_mix(count: int = 256, seed0: int = 4000, sizes=(128, 256, 512), steps: int = 1000):
    """Independent bump solves, seeds seed0 + i; grid size drawn uniformly from sizes
    (same physical domain, absorbing layer n/16 points)."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        out.append(curved_bump(n=n, seed=seed0 + i, steps=steps))
    return out


def serving_arrivals(count: int, rate_per_s: float, seed: int = 5000,
                     sizes=(64, 128, 256, 512, 1024), steps_range=(200, 5000)):
    """Poisson arrival process: exponential inter-arrival gaps at the given rate;
    each request is a bump solve with n uniform over sizes and a step count uniform
    in steps_range (inclusive)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate_per_s))
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        st = int(rng.integers(steps_range[0], steps_range[1] + 1))
        reqs.append((t, curved_bump(n=n, seed=seed + 1 + i, steps=st)))
    return reqs
