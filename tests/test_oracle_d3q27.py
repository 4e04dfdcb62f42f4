"""Pins of the oracle on the D3Q27 velocity set (the method section's
lattice), compiled from the same source with ORACLE_Q = 27.

* The set: 27 distinct velocities, weights summing to one, isotropy through
  the fourth moment, the canonical opposite-pair order (first 19 directions
  as in D3Q19), and the dense transcription's independently generated table.
* One cell: equilibrium moments, Guo-term moments, per-cell mass and momentum
  of the collision.
* Zou-He on 27 velocities: after the fill the cell carries the prescribed
  density and velocity (inflow) or density and zero tangential velocity
  (outflow), only the nine unknowns change, and the weight-proportional
  transverse correction reduces to the D3Q19 closure on the D3Q19 set.
* Plane Poiseuille flow is exact at the textbook relaxation time, as on D3Q19.
* Whole steps against the dense NumPy transcription: test_oracle_lattice.
"""

import numpy as np
import pytest

import oracle
from oracle import bruteforce
from synth import channel_case

RNG = np.random.default_rng(2727)


def _case(**kw):
    c = channel_case(4)
    c.lattice = 27
    c.porous = dict(c.porous, **{k: v for k, v in kw.items() if k in c.porous})
    return c


def _random_cell(phi, amp=0.05):
    c, w = oracle.lattice(27)
    rho = RNG.uniform(0.95, 1.05)
    u = RNG.uniform(-amp, amp, 3)
    cu = c @ u
    feq = w * phi * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * u @ u)
    f = feq * (1 + 0.05 * RNG.standard_normal(27))
    phit = np.where(RNG.random(27) < 0.7, RNG.uniform(0.55, 1.0, 27), phi)
    phit[0] = phi
    return f, phit


def test_lattice_is_d3q27_isotropic():
    c, w = oracle.lattice(27)
    assert len({tuple(v) for v in c}) == 27
    assert abs(w.sum() - 1) < 1e-15
    I = np.eye(3)
    assert np.abs(w @ c).max() < 1e-16
    assert np.abs(np.einsum("i,ia,ib->ab", w, c, c) - I / 3).max() < 1e-15
    assert np.abs(np.einsum("i,ia,ib,ic->abc", w, c, c, c)).max() < 1e-16
    M4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    iso = (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I) + np.einsum("ad,bc->abcd", I, I)) / 9
    assert np.abs(M4 - iso).max() < 1e-15
    for i in range(1, 27, 2):
        assert np.all(c[i] == -c[i + 1])
    c19, _ = oracle.lattice(19)
    assert np.all(c[:19] == c19)
    assert np.all(bruteforce.C27 == c) and np.allclose(bruteforce.W27, w, rtol=0, atol=1e-16)


@pytest.mark.parametrize("trial", range(4))
def test_cell_moments_and_collision(trial):
    case = _case(g=(2e-5, 1e-5, -3e-5), d=1.5, forchheimer=1)
    c, w = oracle.lattice(27)
    phi = RNG.uniform(0.6, 0.95)
    f, phit = _random_cell(phi)
    r = oracle.cell(case, f, 1.1, phi, phit)
    feq, rho, u, F, om = r["feq"], r["rho"], r["u"], r["F"], r["omega"]
    # equilibrium moments
    assert abs(feq.sum() - phi * rho) < 1e-14
    assert np.abs(feq @ c - phi * rho * u).max() < 1e-14
    M2 = np.einsum("i,ia,ib->ab", feq, c, c)
    assert np.abs(M2 - phi * rho * (np.eye(3) / 3 + np.outer(u, u))).max() < 1e-14
    # Guo term moments
    G = r["q"] - f + om * (f - feq) - w * rho * (phit - phi)
    assert abs(G.sum()) < 1e-15
    assert np.abs(G @ c - (1 - om / 2) * F).max() < 1e-15
    assert np.abs(np.einsum("i,ia,ib->ab", G, c, c) - (1 - om / 2) * (np.outer(u, F) + np.outer(F, u))).max() < 1e-15
    # collision mass and momentum
    jump = w * rho * (phit - phi)
    assert abs(r["q"].sum() - f.sum() - jump.sum()) < 1e-15
    assert np.abs(r["q"] @ c - (f @ c + F + jump @ c)).max() < 1e-15


@pytest.mark.parametrize("trial", range(5))
def test_zou_he_closures_d3q27(trial):
    c, w = oracle.lattice(27)
    f = w * (1 + 0.1 * RNG.standard_normal(27))
    u = np.array([RNG.uniform(0, 0.1), RNG.uniform(-0.02, 0.02), RNG.uniform(-0.02, 0.02)])
    g = oracle.zouhe_inlet(f, *u)
    assert np.abs(g @ c - g.sum() * u).max() < 1e-15
    assert np.all(g[c[:, 0] != 1] == f[c[:, 0] != 1])
    rho_out = RNG.uniform(0.98, 1.02)
    h = oracle.zouhe_outlet(f, rho_out)
    assert abs(h.sum() - rho_out) < 1e-15
    assert np.abs((h @ c)[1:]).max() < 1e-16
    assert np.all(h[c[:, 0] != -1] == f[c[:, 0] != -1])


@pytest.mark.parametrize("trial", range(3))
def test_weight_proportional_closure_is_the_d3q19_closure(trial):
    c, w = oracle.lattice(19)
    f = w * (1 + 0.1 * RNG.standard_normal(19))
    u = np.array([RNG.uniform(0, 0.1), RNG.uniform(-0.02, 0.02), RNG.uniform(-0.02, 0.02)])
    s0, sm = f[c[:, 0] == 0].sum(), f[c[:, 0] == -1].sum()
    rho = (s0 + 2 * sm) / (1 - u[0])
    N = (f[c[:, 0] == 0] @ c[c[:, 0] == 0])[1:] - 2 / 3 * rho * u[1:]
    g = f.copy()
    for i in np.flatnonzero(c[:, 0] == 1):
        o = np.flatnonzero((c == -c[i]).all(1))[0]
        g[i] = f[o] + 6 * w[i] * rho * (c[i] @ u) - 18 * w[i] * (c[i, 1] * N[0] + c[i, 2] * N[1])
    assert np.abs(g - oracle.zouhe_inlet(f, *u)).max() < 1e-16


def test_poiseuille_exact_at_magic_tau_d3q27():
    nu = np.sqrt(3) / 12
    H, g = 30, 1e-6
    c = channel_case(H + 2, nx=1, nz=1, g=g, rheology=dict(nu0=nu, nu_inf=nu, lam=0.0, n=1.0, a=2.0))
    c.lattice = 27
    o = oracle.Oracle(c)
    f, om = o.init()
    o.run(f, om, 0, 40000)
    m = o.moments(f, om, 40000)
    y = np.arange(1, H + 1)
    exact = g / (2 * nu) * (y - 0.5) * (H + 0.5 - y)
    assert np.abs(m["u"][0] - exact).max() / exact.max() < 1e-10
    assert np.abs(m["u"][1:]).max() < 1e-13
