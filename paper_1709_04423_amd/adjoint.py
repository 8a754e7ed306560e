"""Differentiable real-time SSCN evolution (torch.autograd) over libgp's
hand-written adjoint kernels, with sqrt(T) checkpointing.

``evolve(psi0, sched, g, ...)`` runs T = len(sched) real-time steps whose
potential substep at step n uses omega[sched_axis] = sched[n], and returns the
final wavefunction.  Gradients flow to ``psi0`` (complex, PyTorch's convention
dL/dRe + i dL/dIm), ``sched`` and ``g``.

Forward keeps only every S-th state (S = ceil(sqrt(T))); backward walks the
segments in reverse, recomputes each segment's states from its checkpoint
with the forward kernels, and runs the adjoint kernels over the segment
(gp_step_adjoint), so memory is O(sqrt(T)) grids and the extra work one
forward pass.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import binding


def _prec(dtype) -> int:
    if dtype == torch.complex128:
        return binding.GP_C128
    if dtype == torch.complex64:
        return binding.GP_C64
    raise TypeError("psi0 must be complex128 or complex64")


class _SSCNEvolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi0, sched, g, n, dx, dt, omega, sched_axis, every):
        T = int(sched.numel())
        sched_np = sched.detach().to("cpu", torch.float64).numpy().copy()
        plan = binding.Plan(n, dx, dt, binding.GP_REAL, omega, float(g), _prec(psi0.dtype), sched=sched_np,
                            sched_axis=sched_axis)
        S = every or max(1, math.ceil(math.sqrt(T)))
        psi = psi0.detach().clone().contiguous()
        checkpoints = []
        for k0 in range(0, T, S):
            checkpoints.append(psi.clone())
            plan.step(psi, min(S, T - k0))
        ctx.plan = plan
        ctx.T, ctx.S = T, S
        ctx.save_for_backward(*checkpoints)
        ctx.sched_dtype = sched.dtype
        ctx.g_dtype = g.dtype if isinstance(g, torch.Tensor) else torch.float64
        return psi

    @staticmethod
    def backward(ctx, grad_out):
        plan, T, S = ctx.plan, ctx.T, ctx.S
        checkpoints = ctx.saved_tensors
        lam = grad_out.detach().to(checkpoints[0].dtype).clone().contiguous()
        dev = lam.device
        dsched = torch.zeros(T, dtype=torch.float64, device=dev)
        dg = torch.zeros(1, dtype=torch.float64, device=dev)
        states = torch.empty((S,) + tuple(lam.shape), dtype=lam.dtype, device=dev)
        for seg in range(len(checkpoints) - 1, -1, -1):
            k0 = seg * S
            m = min(S, T - k0)
            psi = checkpoints[seg].clone()
            plan.set_step(k0)
            plan.step_record(psi, m, states)  # recompute the segment, keeping every step's input
            plan.adjoint(states, lam, k0, m, dsched[k0:k0 + m], dg)
        return (lam, dsched.to(ctx.sched_dtype), dg.reshape(()).to(ctx.g_dtype), None, None, None, None, None,
                None)


def evolve(psi0: torch.Tensor, sched: torch.Tensor, g, n, dx, dt: float, omega, sched_axis: int = 0,
           checkpoint_every: int | None = None) -> torch.Tensor:
    """Differentiable T = len(sched) real-time SSCN steps from psi0 (see module doc).

    ``g`` may be a float or a 0-d float tensor (differentiable); grid sizes and
    spacings are given x first; psi0 is an (Nz, Ny, Nx)-shaped device tensor."""
    if not isinstance(g, torch.Tensor):
        g = torch.tensor(float(g), dtype=torch.float64)
    return _SSCNEvolve.apply(psi0, sched, g, tuple(n), dx, float(dt), omega, int(sched_axis), checkpoint_every)


def overlap_loss(psi_T: torch.Tensor, psi_target: torch.Tensor, dx) -> torch.Tensor:
    """1 - |<psi_target|psi_T>|^2 with the rectangle-rule inner product."""
    dv = float(np.prod(np.broadcast_to(np.asarray(dx, dtype=np.float64), (psi_T.dim(),))))
    c = dv * torch.sum(psi_target.conj() * psi_T)
    return 1.0 - (c.real ** 2 + c.imag ** 2)
