"""Seeded synthetic workloads (problem parameters, initial-data descriptors, noise).

This module draws random numbers and describes inputs; it holds none of the
method's arithmetic (no basis, projection, operator or time stepping), which is
why both the HIP path and the CPU oracle may use it.

Initial data of species s of an instance is described as

    U_s = sum_t amp_t * Proj[prod_m g_{t,m}] * (1 + mult_t)  +  add_s

where Proj is the L2 projection onto the sparse space (each side computes its
own), mult_t / add_s are per-coefficient arrays (or None) in the canonical DOF
order, and a 1D factor g is  ("cos", f, phi) = cos(2 pi f x + phi)  or
("box", a, b) = indicator of [a, b).

Reaction polynomials are arrays c[s, a, b] (species x 4 x 4):
f_s(u, v) = sum_{a,b} c[s, a, b] u^a v^b.

Workloads (d-dimensional periodic unit cube, sigma = 20, nq = k+1):

  heat_linear_d2   d=2 N=5 k=1,  u_t = Lap u - u,  sin(2 pi x) sin(2 pi y),
                   dt=0.01, 10 steps, M=20
  schnakenberg_d2  d=2 N=7 k=2,  u_t = 0.01 Lap u + a - u + u^2 v,
                   v_t = Lap v + b - u^2 v, a=0.1, b=0.9; IC (a+b, b/(a+b)^2)
                   plus U[-0.01, 0.01] noise per coefficient; dt=0.05,
                   200 steps, M=30
  allen_cahn_d3    d=3 N=7 k=1,  u_t = div(K grad u) + u - u^3,
                   K_ii = 1 + 0.5 sin(2 pi x_i); IC: 8 Fourier modes,
                   |freq| <= 3, amplitudes N(0, 0.1^2); dt=0.01, 100 steps, M=30
  gray_scott_batch 64 instances d=2, n = 5 + (i mod 4), k = 1 + (i//4 mod 2),
                   u_t = D_u Lap u - u v^2 + F (1-u), v_t = D_v Lap v + u v^2 - (F+kappa) v,
                   F ~ U[0.02,0.06], kappa ~ U[0.05,0.065], D_u = 2e-5/6.25,
                   D_v = 1e-5/6.25 (the [0,2.5]^2 domain mapped to [0,1]^2);
                   IC u = 1, v = 0 outside the centred square of side 0.25,
                   inside u = 0.5(1+0.01 xi), v = 0.25(1+0.01 eta); dt=1, 500 steps, M=25
  quadratic_d4     d=4 N=6 k=1,  u_t = Lap u - u^2, 0.5 prod sin(2 pi x_i),
                   dt=0.005, 100 steps, M=40; batch variant: 16 right-hand sides
                   with amplitudes U[0.1, 1]

  example2 / example3  Examples 2 and 3 of Sec. 4 (periodic with forcing;
                   zero Dirichlet with u^2 and forcing), analytic data, no seed

Seeds: numpy default_rng(1810_11111 + index), index = 1..5 in the order above.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 1810_11111

SIN = ("cos", 1.0, -math.pi / 2.0)  # sin(2 pi x)
COS = ("cos", 1.0, 0.0)
ONE = ("cos", 0.0, 0.0)


def rx_zeros(species: int):
    return np.zeros((species, 4, 4), dtype=np.float64)


def rx_linear(c: float):
    r = rx_zeros(1)
    r[0, 1, 0] = c
    return r


def rx_schnakenberg(a: float, b: float, kappa: float = 1.0):
    r = rx_zeros(2)
    r[0, 0, 0], r[0, 1, 0], r[0, 2, 1] = kappa * a, -kappa, kappa
    r[1, 0, 0], r[1, 2, 1] = kappa * b, -kappa
    return r


def rx_gray_scott(F: float, kappa: float):
    r = rx_zeros(2)
    r[0, 0, 0], r[0, 1, 0], r[0, 1, 2] = F, -F, -1.0
    r[1, 1, 2], r[1, 0, 1] = 1.0, -(F + kappa)
    return r


def rx_allen_cahn():
    r = rx_zeros(1)
    r[0, 1, 0], r[0, 3, 0] = 1.0, -1.0
    return r


def rx_quadratic(c: float = -1.0):
    r = rx_zeros(1)
    r[0, 2, 0] = c
    return r


def rx_stiff_linear_system(b: float, c: float):
    """u_t = D Lap u - b u + v,  v_t = D Lap v - c v."""
    r = rx_zeros(2)
    r[0, 1, 0], r[0, 0, 1] = -b, 1.0
    r[1, 0, 1] = -c
    return r


def fourier_mode_terms(amp: float, freqs, phase: float):
    """amp*cos(2 pi freqs.x + phase) as 2^d separable terms.

    cos(phase + sum_m t_m) = sum over subsets S of the axes of
    cos(phase + |S| pi/2) * prod_{m in S} sin(t_m) * prod_{m not in S} cos(t_m).
    """
    d = len(freqs)
    terms = []
    for mask in range(2 ** d):
        nsin = bin(mask).count("1")
        coef = amp * math.cos(phase + nsin * math.pi / 2.0)
        factors = []
        for m in range(d):
            ph = -math.pi / 2.0 if (mask >> m) & 1 else 0.0
            factors.append(("cos", float(freqs[m]), ph))
        terms.append((coef, factors))
    return terms


class Instance:
    """One independent problem: grid, species, reaction, diffusion, kappa."""

    def __init__(self, d, N, k, D, rx, kdiag=None, bc=0):
        self.d, self.N, self.k = int(d), int(N), int(k)
        self.D = [float(x) for x in D]
        self.rx = np.asarray(rx, dtype=np.float64)
        self.kdiag = kdiag  # None or (a0, a1, f): k_ii(x) = a0 + a1 sin(2 pi f x), every axis
        self.bc = int(bc)  # 0: periodic, 1: zero Dirichlet on every face

    @property
    def species(self):
        return len(self.D)


class Workload:
    def __init__(self, name, instances, dt, steps, M, prec, ics, sources=None):
        self.name = name
        self.instances = instances
        self.dt, self.steps, self.M = float(dt), int(steps), int(M)
        self.prec = prec
        self._ics = ics  # callable(inst_index, ndof) -> list over species of (terms, mult, add)
        # forcing of species 0: list of (amp, [factor per axis], rate), meaning
        # sum amp * exp(-rate t) * prod_m g_m(x_m); each side projects it itself
        self.sources = sources or []

    def initial_condition(self, inst: int, ndof: int):
        return self._ics(inst, ndof)


def heat_linear_d2():
    inst = Instance(2, 5, 1, [1.0], rx_linear(-1.0))
    return Workload("heat_linear_d2", [inst], 0.01, 10, 20, "fp64",
                    lambda i, n: [([(1.0, [SIN, SIN])], [None], None)])


def schnakenberg_d2(N=7, k=2, steps=200):
    a, b = 0.1, 0.9
    inst = Instance(2, N, k, [0.01, 1.0], rx_schnakenberg(a, b))

    def ics(i, n):
        rng = np.random.default_rng(SEED_BASE + 2)
        nu = rng.uniform(-0.01, 0.01, size=n)
        nv = rng.uniform(-0.01, 0.01, size=n)
        return [([(a + b, [ONE, ONE])], [None], nu),
                ([(b / (a + b) ** 2, [ONE, ONE])], [None], nv)]

    return Workload("schnakenberg_d2", [inst], 0.05, steps, 30, "fp64", ics)


def allen_cahn_d3(N=7, steps=100):
    inst = Instance(3, N, 1, [1.0], rx_allen_cahn(), kdiag=(1.0, 0.5, 1.0))
    rng = np.random.default_rng(SEED_BASE + 3)
    modes = []
    while len(modes) < 8:
        f = rng.integers(-3, 4, size=3)
        if np.any(f != 0):
            modes.append(f)
    amps = rng.normal(0.0, 0.1, size=8)
    phases = rng.uniform(0.0, 2.0 * math.pi, size=8)
    terms = []
    for f, am, ph in zip(modes, amps, phases):
        terms += fourier_mode_terms(float(am), f, float(ph))
    return Workload("allen_cahn_d3", [inst], 0.01, steps, 30, "bf16",
                    lambda i, n: [(terms, [None] * len(terms), None)])


def gray_scott_batch(ninst=64, steps=500):
    rng = np.random.default_rng(SEED_BASE + 4)
    Fs = rng.uniform(0.02, 0.06, size=ninst)
    ks = rng.uniform(0.05, 0.065, size=ninst)
    Du, Dv = 2e-5 / 6.25, 1e-5 / 6.25
    insts = [Instance(2, 5 + (i % 4), 1 + ((i // 4) % 2), [Du, Dv], rx_gray_scott(Fs[i], ks[i]))
             for i in range(ninst)]
    box = ("box", 0.375, 0.625)

    def ics(i, n):
        r = np.random.default_rng([SEED_BASE + 4, i])
        xi = r.uniform(-1.0, 1.0, size=n)
        eta = r.uniform(-1.0, 1.0, size=n)
        return [([(1.0, [ONE, ONE]), (-0.5, [box, box])], [None, 0.01 * xi], None),
                ([(0.25, [box, box])], [0.01 * eta], None)]

    return Workload("gray_scott_batch", insts, 1.0, steps, 25, "fp32", ics)


def quadratic_d4(N=6, nrhs=1, steps=100):
    rng = np.random.default_rng(SEED_BASE + 5)
    amps = [0.5] if nrhs == 1 else list(rng.uniform(0.1, 1.0, size=nrhs))
    insts = [Instance(4, N, 1, [1.0], rx_quadratic(-1.0)) for _ in amps]
    return Workload("quadratic_d4", insts, 0.005, steps, 40, "fp64",
                    lambda i, n: [([(float(amps[i]), [SIN] * 4)], [None], None)])


def _sin2_terms(d: int, amp: float):
    """amp * prod_m sin^2(2 pi x_m) = amp * prod_m (1 - cos(4 pi x_m)) / 2 as 2^d separable terms."""
    terms = []
    for mask in range(2 ** d):
        coef = amp * (-1.0) ** bin(mask).count("1") / 2.0 ** d
        terms.append((coef, [("cos", 2.0, 0.0) if (mask >> m) & 1 else ONE for m in range(d)]))
    return terms


def example2(d=2, N=5, k=1):
    """Sec. 4, Example 2: u_t = kap Lap u + u - exp(-t) prod sin(2 pi x_i), periodic,
    u(x, 0) = prod sin(2 pi x_i), exact exp(-t) prod sin(2 pi x_i); kap = 1/(8 pi^2)
    (2D) or 1/(12 pi^2) (3D); dt = h_N, T = 1 (2D) or 0.4 (3D), M = 25."""
    kap = 1.0 / (8.0 * math.pi ** 2) if d == 2 else 1.0 / (12.0 * math.pi ** 2)
    inst = Instance(d, N, k, [kap], rx_linear(1.0))
    dt = 2.0 ** -N
    T = 1.0 if d == 2 else 0.4
    return Workload(f"example2_d{d}", [inst], dt, int(round(T / dt)), 25, "fp64",
                    lambda i, n: [([(1.0, [SIN] * d)], [None], None)], sources=[(-1.0, [SIN] * d, 1.0)])


def example3(d=2, N=5, k=1):
    """Sec. 4, Example 3: u_t = kap Lap u + u^2 - exp(-2t) prod sin^2(2 pi x_i), zero
    Dirichlet boundary, u(x, 0) = prod sin(2 pi x_i), exact exp(-t) prod sin(2 pi x_i);
    kap as Example 2; dt = h_N, T = 1 (2D) or 0.2 (3D), M = 25."""
    kap = 1.0 / (8.0 * math.pi ** 2) if d == 2 else 1.0 / (12.0 * math.pi ** 2)
    inst = Instance(d, N, k, [kap], rx_quadratic(1.0), bc=1)
    dt = 2.0 ** -N
    T = 1.0 if d == 2 else 0.2
    src = [(a, f, 2.0) for a, f in _sin2_terms(d, -1.0)]
    return Workload(f"example3_d{d}", [inst], dt, int(round(T / dt)), 25, "fp64",
                    lambda i, n: [([(1.0, [SIN] * d)], [None], None)], sources=src)


def smooth_random(n: int, seed: int, nrhs: int = 1):
    """Seeded random vectors for operator tests (uniform in [-1, 1])."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(nrhs, n))
