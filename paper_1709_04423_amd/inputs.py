"""Seeded synthetic inputs for the SSCN Gross-Pitaevskii workloads.

This module only draws and lays out inputs; it holds none of the time-stepping
arithmetic, and both the GPU path's tests/benchmark and the FP64 CPU oracle take
their inputs from it.  The paper's own sample inputs are not available, so every
workload is synthetic: harmonic traps, Gaussian starting states (the g = 0
ground state of each trap, optionally with seeded complex noise) and seeded
parameter draws, with the grid sizes, spacings, time steps and nonlinearities
of the five workloads below.

Arrays are complex128 (or complex64), C-contiguous, shape (Nz, Ny, Nx) /
(Ny, Nx) / (Nx,) with x fastest; grid sizes and spacings are given x first.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 1709


def seed_for(index: int, base: int = BASE_SEED) -> np.random.SeedSequence:
    """Child seed number ``index`` of the base seed (one per workload)."""
    return np.random.SeedSequence(base).spawn(index + 1)[index]


def axis_coords(n: int, dx: float) -> np.ndarray:
    """Sample points of the half-open box [-n dx/2, n dx/2), from its left edge."""
    return (np.arange(n, dtype=np.float64) - 0.5 * n) * dx


def gaussian(n, dx, omega, dtype=np.complex128) -> np.ndarray:
    """Product of 1D harmonic-oscillator ground states (w/pi)^(1/4) exp(-w x^2/2)."""
    n = list(n)
    dx = list(np.broadcast_to(np.asarray(dx, dtype=np.float64), (len(n),)))
    omega = list(np.broadcast_to(np.asarray(omega, dtype=np.float64), (len(n),)))
    psi = np.ones((), dtype=np.float64)
    for a in range(len(n)):  # x first; outer product places x last (fastest)
        x = axis_coords(n[a], dx[a])
        f = (omega[a] / np.pi) ** 0.25 * np.exp(-0.5 * omega[a] * x * x)
        psi = np.multiply.outer(f, psi) if a > 0 else f
    return np.ascontiguousarray(psi, dtype=dtype)


def noisy_gaussian(n, dx, omega, seed, amp=1e-3, dtype=np.complex128) -> np.ndarray:
    """Gaussian plus amp * (U[-1,1) + i U[-1,1)) per point, scaled to unit norm."""
    psi = gaussian(n, dx, omega, np.complex128)
    rng = np.random.default_rng(seed)
    noise = rng.uniform(-1.0, 1.0, size=psi.shape) + 1j * rng.uniform(-1.0, 1.0, size=psi.shape)
    psi = psi + amp * noise
    dv = float(np.prod(np.broadcast_to(np.asarray(dx, dtype=np.float64), (len(list(n)),))))
    psi /= np.sqrt(dv * np.sum(np.abs(psi) ** 2))
    return np.ascontiguousarray(psi, dtype=dtype)


def random_field(shape, seed, dtype=np.complex128) -> np.ndarray:
    """Seeded complex field with N(0,1) real and imaginary parts."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return np.ascontiguousarray(a, dtype=dtype)


@dataclass
class Workload:
    """One SSCN run: grid (x first), spacing, time step, trap, g, step count."""
    name: str
    n: tuple
    dx: float
    dt: float
    omega: tuple
    g: float
    steps: int
    mode: str = "imag"
    extra: dict = field(default_factory=dict)

    @property
    def ndim(self) -> int:
        return len(self.n)

    @property
    def points(self) -> int:
        return int(np.prod(self.n))

    @property
    def shape(self) -> tuple:
        return tuple(self.n[::-1])


# 1D imaginary time, N = 512 on [-12.8, 12.8), V = x^2/2, g in {0, 62.74}.
ONE_D = Workload("1d_imag_512", (512,), 0.05, 5e-4, (1.0,), 62.74, 10_000, "imag",
                 {"g_values": (0.0, 62.74)})
# 3D real time, 128^3, dx = 0.1, V = (x^2 + y^2 + 16 z^2)/2, g = 100, quench w_x 1 -> 0.5.
QUENCH_3D = Workload("3d_real_128_quench", (128, 128, 128), 0.1, 1e-3, (0.5, 1.0, 4.0), 100.0,
                     1_000, "real", {"omega_before": (1.0, 1.0, 4.0)})
# 3D 256^3, dx = 0.05, V = (x^2 + 4 y^2 + 9 z^2)/2, g = 1000, dt = 2e-4, 2000 steps per mode.
HEADLINE_3D = Workload("3d_256_imag_real", (256, 256, 256), 0.05, 2e-4, (1.0, 2.0, 3.0), 1000.0,
                       2_000, "imag+real", {"noise": 1e-3})
# 2D real-time adjoint, 256^2, dx = 0.05, V = (gamma(t)^2 x^2 + y^2)/2, g = 200, T = 2000.
ADJOINT_2D = Workload("2d_adjoint_256", (256, 256), 0.05, 1e-3, (1.0, 1.0), 200.0, 2_000, "real",
                      {"gamma_range": (0.8, 1.2), "gamma_target": 1.5})

WORKLOADS = {w.name: w for w in (ONE_D, QUENCH_3D, HEADLINE_3D, ADJOINT_2D)}
SEED_INDEX = {"1d_imag_512": 0, "3d_real_128_quench": 1, "3d_256_imag_real": 2, "2d_batch_64": 3,
              "2d_adjoint_256": 4}


def headline_initial(n=HEADLINE_3D.n, dtype=np.complex128, seed_index=SEED_INDEX["3d_256_imag_real"]):
    """Noisy Gaussian start of the 256^3 run (or the same recipe on another grid)."""
    w = HEADLINE_3D
    return noisy_gaussian(n, w.dx, w.omega, seed_for(seed_index), w.extra["noise"], dtype)


def batch_problems(count=64, sides=(128, 192, 256, 384, 512), seed_index=SEED_INDEX["2d_batch_64"]):
    """Independent 2D real-time problems: sides drawn per axis from ``sides``,
    dx = 0.05, g ~ U[10, 500], trap ratio nu ~ U[0.5, 2] on y, dt = 1e-3."""
    rng = np.random.default_rng(seed_for(seed_index))
    probs = []
    for k in range(count):
        nx = int(rng.choice(sides))
        ny = int(rng.choice(sides))
        g = float(rng.uniform(10.0, 500.0))
        nu = float(rng.uniform(0.5, 2.0))
        probs.append(Workload(f"batch_{k}", (nx, ny), 0.05, 1e-3, (1.0, nu), g, 1_000, "real"))
    return probs


def gamma_schedule(T=ADJOINT_2D.steps, lo=0.8, hi=1.2, seed_index=SEED_INDEX["2d_adjoint_256"]):
    """Trap-control values gamma_n ~ U[lo, hi], one per real-time step."""
    rng = np.random.default_rng(seed_for(seed_index))
    return rng.uniform(lo, hi, size=T)
