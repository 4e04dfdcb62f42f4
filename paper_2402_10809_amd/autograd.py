"""The sac objectives as differentiable functions of the porosity.

``region_objective(phi, solver, t_begin, t_end, T, kind=...)`` returns
J(phi) = time average over steps [t_begin, t_end) of a region mean, for a run
of T steps from rest with porosity phi:

* kind "ke": the region mean of rho |u|^2 / 2 (``sac_kinetic_energy``);
* kind "wss": the mean wall shear stress magnitude |tau| over the region's
  wall cells, the quantity the paper averages over the aneurysm wall
  (``sac_wall_shear_stress``).

When phi requires a gradient, the forward call runs ``lbm_adjoint``, which
returns J and dJ/dphi together (hand-written reverse steps over checkpointed
segments); the backward pass scales that gradient.  Otherwise only J is
computed.

phi is the dense box porosity (nz, ny, nx), FP32, on any device; it must keep
the solver's solid mask (0 on solid voxels, in (0, 1] on fluid, 1 on open
faces).  The solver is reset to the rest state by every evaluation.
fp64=True keeps the adjoint populations of the reverse sweep in FP64.
"""

from __future__ import annotations

from typing import Optional

import torch


class RegionObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi: torch.Tensor, solver, t_begin: int, t_end: int, T: int, ckpt: Optional[int], kind: str,
                fp64: bool = False):
        # device to device: the library reads phi in place (no host copy)
        solver.set_porosity(phi.detach().to(solver.device, torch.float32).contiguous())
        ctx.phi_device = phi.device
        if ctx.needs_input_grad[0]:
            J, g = solver.adjoint(t_begin, t_end, T, ckpt, kind=kind, fp64=fp64)
            ctx.save_for_backward(g)
        else:
            J = solver.objective(t_begin, t_end, T, kind=kind)
        return torch.tensor(J, dtype=torch.float64, device=phi.device)

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        gphi = (grad_out.to(g.device, torch.float64) * g.to(torch.float64)).to(torch.float32)
        return gphi.to(ctx.phi_device), None, None, None, None, None, None, None


def region_objective(phi: torch.Tensor, solver, t_begin: int, t_end: int, T: int,
                     ckpt: Optional[int] = None, kind: str = "ke", fp64: bool = False) -> torch.Tensor:
    """Differentiable J(phi); see the module docstring."""
    return RegionObjective.apply(phi, solver, int(t_begin), int(t_end), int(T), ckpt, kind, bool(fp64))


def sac_kinetic_energy(phi: torch.Tensor, solver, t_begin: int, t_end: int, T: int,
                       ckpt: Optional[int] = None, fp64: bool = False) -> torch.Tensor:
    """Differentiable time-averaged region kinetic energy."""
    return region_objective(phi, solver, t_begin, t_end, T, ckpt, "ke", fp64)


def sac_wall_shear_stress(phi: torch.Tensor, solver, t_begin: int, t_end: int, T: int,
                          ckpt: Optional[int] = None, fp64: bool = False) -> torch.Tensor:
    """Differentiable time-averaged WSS magnitude over the region's wall cells."""
    return region_objective(phi, solver, t_begin, t_end, T, ckpt, "wss", fp64)
