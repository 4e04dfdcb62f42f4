"""Pins of the oracle's porosity gradient of the sac objectives (kinetic
energy, and wall shear stress magnitude over the sac's wall cells).

Three independent routes must agree: central finite differences of the FP64
objective, forward-mode dual numbers through the whole run, and the
checkpointed reverse sweep with per-cell local Jacobians.
"""

import numpy as np
import pytest

import oracle
from synth import aniso_shape, fd_voxels, tiny_case


def _case(seed, lattice="open"):
    forch = lattice.endswith("_forch")
    aniso = lattice.endswith("_aniso")
    c = tiny_case(lattice.rsplit("_", 1)[0] if (forch or aniso) else lattice, seed=seed)
    if forch:
        c.porous = dict(c.porous, forchheimer=1)
    if aniso:
        c.porous = dict(c.porous, forchheimer=1, aniso=aniso_shape(), aniso_iters=6)
    c.wave = (0.04, 0.5, 20.0)
    c.rheology = dict(c.rheology, lam=200.0)  # shear-thinning active at these speeds
    return c


@pytest.mark.parametrize("kind", ["ke", "wss"])
@pytest.mark.parametrize("seed,lattice", [(0, "open"), (1, "open"), (0, "open_extrap"), (1, "open_extrap"),
                                          (0, "open_forch"), (1, "open_forch"), (0, "open_aniso")])
def test_reverse_sweep_matches_dual_and_fd(seed, lattice, kind):
    """Also with the extrapolation outflow, whose unknowns are state carried
    from step to step, with Forchheimer drag, and with the anisotropic
    permeability (six fixed-point iterates per cell and step)."""
    case = _case(seed, lattice)
    T, tb, te, ckpt = 24, 12, 24, 5
    o = oracle.Oracle(case)
    J, grad = o.grad_reverse(T, tb, te, ckpt, kind)
    assert J > 0
    vox = fd_voxels(case, 6, seed=16)
    Jd, gd = o.grad_dual(T, tb, te, vox, kind)
    # the same FP64 arithmetic in two instantiations (double and dual numbers):
    # the compiler may fuse multiply-adds differently in each
    assert abs(Jd - J) < 1e-14 * J
    gr = grad.reshape(-1)[vox]
    scale = np.abs(grad).max()
    assert np.abs(gr - gd).max() < 1e-11 * scale
    # the WSS magnitude of a wall cell bends sharply with its own porosity:
    # the central difference needs a smaller step there (its error ~ eps^2)
    eps = 1e-5 if kind == "ke" else 1e-6
    for k, b in enumerate(vox):
        p = case.phi.astype(np.float64).reshape(-1).copy()
        p[b] += eps
        Jp = oracle.Oracle(case, phi=p.reshape(case.phi.shape)).objective(T, tb, te, kind)
        p[b] -= 2 * eps
        Jm = oracle.Oracle(case, phi=p.reshape(case.phi.shape)).objective(T, tb, te, kind)
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - gd[k]) < 1e-6 * scale + 1e-7 * abs(gd[k])
    # the gradient vanishes off the fluid
    assert np.all(grad.reshape(-1)[case.solid.reshape(-1) == 1] == 0)


def test_objective_matches_stepping():
    case = _case(2)
    o = oracle.Oracle(case)
    f, om = o.init()
    ke = o.run(f, om, 0, 20, want_ke=True)
    assert abs(o.objective(20, 8, 20) - ke[8:20].mean()) < 1e-17 + 1e-14 * abs(ke[8:20].mean())
