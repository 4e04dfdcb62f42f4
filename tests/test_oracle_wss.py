"""Pins of the oracle's voxel wall shear stress (simulation section: WSS
tau = sigma n - (n . sigma n) n from the deviatoric stress sigma = (omega/2 - 1) Pi).

* Steady plane Poiseuille flow driven by a body force g between two halfway
  bounce-back walls H cells apart: the momentum balance of a slab fixes the
  shear stress at the first cell centre to rho g (H - 1) / 2 for any viscosity
  law, so this holds for the Newtonian and the Carreau-Yasuda fluid alike,
  with tau along the flow and the same for walls normal to y or to z.
* The wall normal of a flat wall is the axis, and of a 90-degree corner cell
  the diagonal.
* The sac WSS objective over a run equals the average of the stepped values.
"""

import numpy as np
import pytest

import oracle
from synth import tiny_case
from synth.cases import Case

CY = dict(nu0=0.1, nu_inf=0.01, lam=50.0, n=0.36, a=2.0)
NEWTONIAN = dict(nu0=0.1, nu_inf=0.1, lam=0.0, n=1.0, a=2.0)


def _slab(ny, wall_axis, g, rheology):
    if wall_axis == "y":
        solid = np.zeros((2, ny, 3), np.uint8)
        solid[:, 0, :] = 1
        solid[:, -1, :] = 1
        periodic = (True, False, True)
    else:
        solid = np.zeros((ny, 2, 3), np.uint8)
        solid[0] = 1
        solid[-1] = 1
        periodic = (True, True, False)
    nz, nyy, nx = solid.shape
    phi = np.where(solid == 0, 1.0, 0.0).astype(np.float32)
    return Case(name="slab", nx=nx, ny=nyy, nz=nz, periodic=periodic, solid=solid, phi=phi, sac=solid == 0,
                rheology=dict(rheology), porous=dict(nu_d=0.1, kc=180.0, d=2.0, forchheimer=0, g=(g, 0.0, 0.0)))


@pytest.mark.parametrize("wall_axis", ["y", "z"])
@pytest.mark.parametrize("law,g,steps", [("newtonian", 1e-5, 4000), ("carreau_yasuda", 1e-4, 20000)])
def test_plane_poiseuille_wall_shear(wall_axis, law, g, steps):
    ny = 10
    case = _slab(ny, wall_axis, g, NEWTONIAN if law == "newtonian" else CY)
    o = oracle.Oracle(case)
    f, om = o.init()
    o.run(f, om, 0, steps)
    m = o.moments(f, om, steps)
    tau = m["tau"]
    mag = np.sqrt((tau ** 2).sum(0))
    on_wall = mag > 0
    assert on_wall.sum() == 2 * 3 * 2  # both walls, 3 x 2 cells each
    expect = m["rho"][on_wall] * g * (ny - 2 - 1) / 2
    assert np.abs(mag[on_wall] - expect).max() < 1e-10 * expect.max()
    assert np.abs(tau[1:]).max() == 0.0  # along the flow only
    assert np.allclose(np.abs(tau[0][on_wall]), mag[on_wall], rtol=0, atol=0)


def test_wall_normals():
    # a closed box: face cells have the face normal, edge cells the diagonal
    n = 5
    solid = np.ones((n, n, n), np.uint8)
    solid[1:-1, 1:-1, 1:-1] = 0
    phi = np.where(solid == 0, 1.0, 0.0).astype(np.float32)
    case = Case(name="box", nx=n, ny=n, nz=n, periodic=(False, False, False), solid=solid, phi=phi,
                sac=solid == 0, porous=dict(nu_d=0.1, kc=180.0, d=2.0, forchheimer=0, g=(1e-4, 2e-4, 0.0)))
    o = oracle.Oracle(case)
    f, om = o.init()
    o.run(f, om, 0, 30)
    m = o.moments(f, om, 30)
    cells = o.cells()
    z, y, x = np.unravel_index(cells, solid.shape)
    tau = m["tau"]
    # the centre cell (2, 2, 2) touches no wall
    centre = np.flatnonzero((x == 2) & (y == 2) & (z == 2))[0]
    assert np.all(tau[:, centre] == 0)
    # a face cell of the x = 1 face: n = -e_x, so tau has no x component
    face = np.flatnonzero((x == 1) & (y == 2) & (z == 2))[0]
    assert tau[0, face] == 0 and np.abs(tau[1:, face]).max() > 0
    # an edge cell (x = 1, y = 1): n = -(e_x + e_y)/sqrt 2, so tau . n = 0
    edge = np.flatnonzero((x == 1) & (y == 1) & (z == 2))[0]
    assert abs(tau[0, edge] + tau[1, edge]) < 1e-18 and np.abs(tau[:, edge]).max() > 0


def test_wss_objective_matches_stepped_values():
    case = tiny_case("open", seed=2)
    o = oracle.Oracle(case)
    # wall cells of the sac: a wall link (neighbour code -1) and m != 0
    nb = o.neighbours()
    c = np.array([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
                  (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
                  (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)], np.float64)
    w = np.array([12.0] + [2.0] * 6 + [1.0] * 12)
    m = np.einsum("ix,ia->ax", (nb == -1) * w[:, None], c)
    wall = np.abs(m).sum(0) > 0
    on = case.sac.reshape(-1)[o.cells()] & wall
    assert on.sum() > 0
    f, om = o.init()
    vals = []
    for t in range(12):
        tau = o.moments(f, om, t)["tau"]
        vals.append(np.sqrt((tau ** 2).sum(0))[on].mean())
        o.run(f, om, t, 1)
    J = o.objective(12, 4, 12, "wss")
    assert J > 0
    assert abs(J - np.mean(vals[4:12])) < 1e-14 * J
