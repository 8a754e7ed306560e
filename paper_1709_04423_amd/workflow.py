"""Stationary -> dynamic workflow of the paper's real-time programs.

"Summary of revisions" describes it: solve the stationary problem by
imaginary-time propagation, store the wavefunction, read it into a real-time
run (the NSTP = 0 hand-over, which needs the same space mesh and
nonlinearity), introduce a perturbation and follow the rms sizes as the
dynamics evolves; the dimensionless nonlinearity comes from physical inputs.
This module only orchestrates: every step, observable and series record runs
in the library's kernels through ``binding``; states are stored as plain .npy
arrays (no pickles) with a JSON description of the mesh.
"""
from __future__ import annotations

import dataclasses
import json
from typing import Optional, Sequence

import numpy as np

from . import binding


@dataclasses.dataclass(frozen=True)
class Problem:
    """Grid (x first), spacings, trap frequencies, nonlinearity, geometry, precision."""
    n: tuple
    dx: tuple
    omega: tuple
    g: float
    geometry: int = binding.GP_CARTESIAN
    prec: int = binding.GP_C128

    @classmethod
    def from_physics(cls, n, dx, omega, natoms: float, a_bohr: float, l_micron: float, confine: float = 1.0,
                     geometry: int = binding.GP_CARTESIAN, prec: int = binding.GP_C128) -> "Problem":
        """g from the number of atoms, the scattering length (Bohr radii) and the oscillator
        length (micrometres); 3D-like geometries use the 3D form, 2D and 1D Cartesian grids
        the reduced forms with confinement ratio `confine` (lambda or nu)."""
        ndim = 3 if geometry in (binding.GP_SPHERICAL, binding.GP_AXIAL) else (
            2 if geometry == binding.GP_CIRCULAR else len(n))
        return cls(tuple(n), tuple(dx), tuple(omega), binding.nonlinearity(ndim, natoms, a_bohr, l_micron, confine),
                   geometry, prec)

    def plan(self, dt: float, mode: int, sched=None, sched_axis: int = 0) -> binding.Plan:
        return binding.Plan(self.n, self.dx, dt, mode, self.omega, self.g, self.prec, sched=sched,
                            sched_axis=sched_axis, geometry=self.geometry)

    @property
    def shape(self) -> tuple:
        return tuple(self.n[::-1])


def gaussian_start(p: Problem, device: str = "cuda"):
    """Product of the trap's g = 0 oscillator ground states on the plan's grid (a
    starting guess for imaginary time)."""
    import torch
    axes = []
    for a, (n, dx, w) in enumerate(zip(p.n, p.dx, p.omega)):
        radial = p.geometry != binding.GP_CARTESIAN and a == 0
        x = (np.arange(n) + 0.5) * dx if radial else (np.arange(n) - 0.5 * n) * dx
        axes.append(np.exp(-0.5 * w * x * x))
    psi = axes[0]
    for f in axes[1:]:
        psi = np.multiply.outer(f, psi)
    dtype = torch.complex128 if p.prec == binding.GP_C128 else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(psi, dtype=np.complex128)).to(device).to(dtype)


def ground_state(p: Problem, dt: float, psi=None, tol: float = 1e-12, block: int = 100,
                 max_steps: int = 1_000_000):
    """Imaginary-time propagation until the chemical potential changes by less than
    tol over `block` steps.  Returns (psi, steps taken, observables)."""
    plan = p.plan(dt, binding.GP_IMAG)
    psi = gaussian_start(p) if psi is None else psi
    prev, steps = None, 0
    while steps < max_steps:
        plan.step(psi, block)
        steps += block
        obs = plan.observables(psi)
        if prev is not None and abs(obs["mu"] - prev) < tol:
            return psi, steps, obs
        prev = obs["mu"]
    raise RuntimeError(f"imaginary time did not converge to {tol} in {max_steps} steps")


def save_state(path: str, psi, p: Problem) -> None:
    """Write psi to <path>.npy and the mesh and nonlinearity to <path>.json."""
    np.save(path + ".npy", psi.detach().cpu().numpy(), allow_pickle=False)
    with open(path + ".json", "w") as f:
        json.dump(dataclasses.asdict(p), f)


def load_state(path: str, p: Problem, device: str = "cuda"):
    """Read a stored wavefunction for problem p: the space mesh, geometry and
    nonlinearity must be the ones it was computed with (the hand-over condition);
    the trap may differ (that is a perturbation)."""
    import torch
    meta = json.load(open(path + ".json"))
    for key in ("n", "dx", "geometry", "g"):
        stored = meta[key]
        want = getattr(p, key)
        if (tuple(stored) if isinstance(stored, list) else stored) != want:
            raise ValueError(f"stored state has {key} = {stored}, the problem has {want}")
    a = np.load(path + ".npy", allow_pickle=False)
    if a.shape != p.shape:
        raise ValueError(f"stored array has shape {a.shape}, the problem has {p.shape}")
    dtype = torch.complex128 if p.prec == binding.GP_C128 else torch.complex64
    return torch.from_numpy(a).to(device).to(dtype)


def perturb(p: Problem, kind: str, factor: float, axis: int = 0) -> Problem:
    """Perturbation presets that start the dynamics: 'trap' scales the trap frequency
    of one axis (a quench: breathing and quadrupole modes), 'nonlinearity' scales g
    (a change of scattering length)."""
    if kind == "trap":
        om = list(p.omega)
        om[axis] *= factor
        return dataclasses.replace(p, omega=tuple(om))
    if kind == "nonlinearity":
        return dataclasses.replace(p, g=p.g * factor)
    raise ValueError(f"unknown perturbation {kind!r} (trap, nonlinearity)")


def dynamics(p: Problem, psi, dt: float, nsteps: int, every: int, sched: Optional[Sequence[float]] = None,
             sched_axis: int = 0):
    """Real-time propagation of psi (in place) under problem p, recording the
    observables every `every` steps (gp_step_series).  Returns a (records, 10)
    float64 array: step, norm, mu, energy, ekin, epot, eint, rms[0..2]."""
    plan = p.plan(dt, binding.GP_REAL, sched=sched, sched_axis=sched_axis)
    return plan.step_series(psi, nsteps, every).cpu().numpy()
