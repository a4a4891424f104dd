"""Seeded synthetic workloads (problem statements only; no solver arithmetic).

The paper's experiments take their data from formulas (x(1-x), sin 2 pi x, a
cos^2 bump, a randomly perturbed time grid), not from a dataset.  The workloads
here are seeded sine series of the same smoothness class, drawn with
``numpy.random.default_rng([config, stream])``:

* stream 0: amplitudes of u_0, stream 1: amplitudes of v_0 (wave) or of the
  perturbation Delta (adjoint), stream 2: the time-grid jitter, stream 3: batch
  sizes and diffusivities.
* Amplitudes are N(0, sigma^2) over sine modes 1..J, sigma = 0.1 unless stated.

A workload is returned as plain numbers (sizes, step, diffusivity, sine-mode
amplitudes, optional step list); both the GPU library and the oracle turn the
amplitudes into initial data themselves.  This module is shared by the two
sides and must never hold any of the method's arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

HEAT = 0
BD2 = 1


@dataclass
class Workload:
    name: str
    scheme: int
    n: int
    ell: int
    tau: float
    kappa: float
    modes: np.ndarray                     # int32 sine-mode numbers of u_0
    amps: np.ndarray                      # float64 amplitudes of u_0
    v_modes: Optional[np.ndarray] = None  # wave initial velocity
    v_amps: Optional[np.ndarray] = None
    restart: int = 30
    tol: float = 1e-8
    maxit: int = 300
    extra: dict = field(default_factory=dict)


def sine_amps(seed, J, sigma=0.1):
    rng = np.random.default_rng(seed)
    return np.arange(1, J + 1, dtype=np.int32), rng.normal(0.0, sigma, size=J)


def perturbed_steps(ell, delta, seed):
    """Step sizes tau_j = t_j - t_{j-1} of the jittered grid
    t_0 = 0, t_j = (j + delta (U_j - 1/2)) / ell (1 <= j < ell), t_ell = 1,
    with U_j uniform on [0,1) (the paper's perturbed grid, read with 1/ell)."""
    rng = np.random.default_rng(seed)
    u = rng.random(ell - 1)
    t = np.empty(ell + 1)
    t[0] = 0.0
    t[1:ell] = (np.arange(1, ell) + delta * (u - 0.5)) / ell
    t[ell] = 1.0
    return np.diff(t)


def paper_initial_data(name, n):
    """Nodal values at x_i = i/(n+1), i = 1..n, of the paper's initial functions
    (Sec. 4): "x(1-x)" (u_0^{s1}), "sin2pix" (u_0^{s2}) and "bump", the non-smooth
    u_0^{ns} = cos^2(4 pi (x - 1/2)) on (3/8, 5/8) and 0 elsewhere."""
    x = np.arange(1, n + 1) / (n + 1)
    if name == "x(1-x)":
        return x * (1 - x)
    if name == "sin2pix":
        return np.sin(2 * np.pi * x)
    if name == "bump":
        return np.where((x > 3 / 8) & (x < 5 / 8), np.cos(4 * np.pi * (x - 0.5)) ** 2, 0.0)
    raise ValueError(name)


def heat_small(n=63, ell=64):
    """Heat, n = 63, ell = 64, tau = 1/64: sin(pi x) plus a 10-mode N(0, 0.1^2)
    series; GMRES(50), tol 1e-10."""
    modes, amps = sine_amps([1, 0], 10)
    amps = amps.copy()
    amps[0] += 1.0
    return Workload("heat_n63_l64", HEAT, n, ell, 1.0 / ell, 1.0, modes, amps,
                    restart=50, tol=1e-10)


def heat_large(n=4095, ell=4096):
    """Heat, n = 4095, ell = 4096 (16.8 M unknowns), tau = 1/ell, 50-mode series;
    GMRES(30) at 1e-8."""
    modes, amps = sine_amps([2, 0], 50)
    return Workload(f"heat_n{n}_l{ell}", HEAT, n, ell, 1.0 / ell, 1.0, modes, amps,
                    restart=30, tol=1e-8)


def heat_large_steps(ell, delta):
    """Jittered step list for the Neumann sweep of the large heat case."""
    return perturbed_steps(ell, delta, [2, 2])


def wave_bd2(n=2047, ell=8192):
    """Wave BD2, n = 2047, ell = 8192, tau = 1/ell, 30-mode u_0 and v_0;
    GMRES(30) at 1e-8."""
    modes, amps = sine_amps([3, 0], 30)
    vm, va = sine_amps([3, 1], 30)
    return Workload(f"wave_bd2_n{n}_l{ell}", BD2, n, ell, 1.0 / ell, 1.0, modes, amps,
                    v_modes=vm, v_amps=va, restart=30, tol=1e-8, maxit=600)


def heat_batch(count=64):
    """64 heat problems: n_p uniform on {255..4095}, ell_p uniform on {256..2048},
    kappa_p uniform on [0.5, 2], 20-mode u_0 each; GMRES(30) at 1e-8."""
    rng = np.random.default_rng([4, 3])
    ns = rng.integers(255, 4096, size=count)
    ells = rng.integers(256, 2049, size=count)
    kappas = rng.uniform(0.5, 2.0, size=count)
    out: List[Workload] = []
    for p in range(count):
        modes, amps = sine_amps([4, 0, p], 20)
        ell = int(ells[p])
        out.append(Workload(f"batch{p}", HEAT, int(ns[p]), ell, 1.0 / ell, float(kappas[p]),
                            modes, amps, restart=30, tol=1e-8))
    return out


def heat_adjoint(n=2047, ell=2048):
    """Adjoint heat, n = 2047, ell = 2048: the target trajectory comes from a
    20-mode u_0 at kappa = 1; the gradient is taken at u_0 + Delta (20 modes,
    N(0, 0.05^2)) and kappa = 1.25."""
    modes, amps = sine_amps([5, 0], 20)
    dm, da = sine_amps([5, 1], 20, sigma=0.05)
    w = Workload(f"heat_adjoint_n{n}_l{ell}", HEAT, n, ell, 1.0 / ell, 1.25, modes,
                 amps + da, restart=30, tol=1e-10)
    w.extra = dict(target_amps=amps, target_kappa=1.0)
    return w


@dataclass
class SquareWorkload:
    name: str
    scheme: int
    nx: int
    ny: int
    ell: int
    tau: float
    kappa: float
    u0: np.ndarray                        # (ny, nx) nodal values, x fastest
    restart: int = 30
    tol: float = 1e-8
    maxit: int = 300


def square_heat(nx=511, ny=511, ell=64):
    """Heat on the unit square, nx x ny interior nodes (511 x 511, 16.7 M unknowns with
    64 steps: the unknown count of the 1D n = 4095, ell = 4096 case), tau = 1/ell,
    kappa = 1; u_0 the nodal values of sin(pi x) sin(pi y) plus an 8 x 8 series of sine
    products with N(0, 0.1^2) amplitudes; GMRES(30) at 1e-8."""
    rng = np.random.default_rng([6, 0])
    a = rng.normal(0.0, 0.1, size=(8, 8))
    a[0, 0] += 1.0
    x = np.arange(1, nx + 1) / (nx + 1)
    y = np.arange(1, ny + 1) / (ny + 1)
    m = np.arange(1, 9)
    sx = np.sin(np.pi * np.outer(m, x))       # (8, nx)
    sy = np.sin(np.pi * np.outer(m, y))       # (8, ny)
    u0 = sy.T @ a @ sx                        # a[q, p] sin(q pi y) sin(p pi x)
    return SquareWorkload(f"square_heat_{nx}x{ny}_l{ell}", HEAT, nx, ny, ell, 1.0 / ell, 1.0,
                          np.ascontiguousarray(u0))
