"""rho -> F as a differentiable torch operation.

The forward pass is one FDTD forward solve (eqs. (10a-c)) with the DFT gap
objective; the backward pass is the adjoint solve of eq. (20) with the
sensitivity sums of eq. (25) folded through eq. (27), i.e. dF/drho exactly as
the discrete forward scheme defines it.  Both run in the HIP library (through
``FDTD``); this module only moves tensors and orders calls.  With
``ckpt_every > 0`` on the solver the backward re-runs checkpointed forward
segments instead of reading a stored full history.

The solver context holds the state of its most recent forward solve.  If
another forward ran on it between this operation's forward and backward, the
backward first re-runs the forward on the saved density, so gradients always
belong to the density they were requested for.
"""
from __future__ import annotations

import torch

from .fdtd import FDTD


class Solver(FDTD):
    """An FDTD context on a torch stream of its own that counts its forward
    solves.  Every call first makes that stream wait for the caller's current
    stream and ends by making the caller's stream wait for it, so tensors
    flow between torch work and the library in order."""

    def __init__(self, w, ckpt_every=None, history_budget_bytes=0, device=None):
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        with torch.cuda.device(dev):
            self.tstream = torch.cuda.Stream(dev)
            super().__init__(w, stream=self.tstream.cuda_stream, history_budget_bytes=history_budget_bytes,
                             ckpt_every=ckpt_every)
        self.device = dev
        self.tdtype = torch.float32 if w["precision"] == 32 else torch.float64
        self.generation = 0

    def _enter(self, *tensors):
        self.tstream.wait_stream(torch.cuda.current_stream(self.device))
        for t in tensors:
            t.record_stream(self.tstream)

    def _leave(self):
        torch.cuda.current_stream(self.device).wait_stream(self.tstream)

    def solve(self, rho):
        """Forward solve on a device density; returns F (host float)."""
        self._enter(rho)
        self.set_density(rho)
        F = self.forward()
        self._leave()
        self.generation += 1
        return F

    def adjoint_gradient(self, out):
        """Adjoint solve and dF/drho into the device tensor `out`."""
        self._enter(out)
        self.adjoint()
        self.gradient(out=out)
        self._leave()
        return out


class _DensityToObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho, solver):
        r = rho.detach().contiguous()
        F = solver.solve(r)
        ctx.save_for_backward(r)
        ctx.solver = solver
        ctx.generation = solver.generation
        return torch.tensor(F, dtype=torch.float64, device=rho.device)

    @staticmethod
    def backward(ctx, gF):
        (r,) = ctx.saved_tensors
        s = ctx.solver
        if s.generation != ctx.generation:
            s.solve(r)
            ctx.generation = s.generation
        g = s.adjoint_gradient(torch.empty_like(r))
        return (gF.to(g.dtype) * g).reshape(r.shape), None


def objective(rho, solver):
    """F(rho) on `solver` (a :class:`Solver`); differentiable in rho.

    rho: CUDA tensor of the solver's dtype with one value per design cell,
    layout [z][y][x] (3D) / [y][x] (2D), values in [0, 1]."""
    if not (isinstance(rho, torch.Tensor) and rho.is_cuda):
        raise TypeError("rho must be a CUDA tensor")
    if rho.dtype != solver.tdtype or rho.numel() != solver.nd:
        raise ValueError(f"rho must be {solver.tdtype} with {solver.nd} values")
    return _DensityToObjective.apply(rho, solver)
