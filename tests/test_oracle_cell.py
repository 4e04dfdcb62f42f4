"""Pins of the FP64 oracle's single-cell arithmetic.

Each check is a property the paper's definitions (method section) or textbook
lattice Boltzmann theory fix independently of how the oracle is written:
lattice isotropy, equilibrium and Guo-forcing moments, the implicit velocity
equation and the Remark's fixed-point iteration, momentum and mass of one
collision, the Zou-He closures, and the Carreau-Yasuda limits.
"""

import numpy as np
import pytest

import oracle
from oracle import bruteforce
from synth import channel_case

RNG = np.random.default_rng(1234)
PA = [0, 1, 2, 0, 0, 1]
PB = [0, 1, 2, 1, 2, 2]


def _case(**kw):
    c = channel_case(4)
    c.porous = dict(c.porous)
    c.rheology = dict(c.rheology)
    for k, v in kw.items():
        if k in c.porous:
            c.porous[k] = v
        elif k in c.rheology:
            c.rheology[k] = v
        else:
            raise KeyError(k)
    return c


def _random_cell(phi=None, amp=0.05):
    c, w = oracle.lattice()
    phi = RNG.uniform(0.55, 1.0) if phi is None else phi
    rho = RNG.uniform(0.95, 1.05)
    u = RNG.uniform(-amp, amp, 3)
    cu = c @ u
    feq = w * phi * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * u @ u)
    f = feq * (1 + 0.05 * RNG.standard_normal(19))
    phit = np.where(RNG.random(19) < 0.7, RNG.uniform(0.55, 1.0, 19), phi)
    phit[0] = phi
    return f, phi, phit


def test_lattice_is_d3q19_isotropic():
    c, w = oracle.lattice()
    assert len({tuple(v) for v in c}) == 19
    assert np.all((c ** 2).sum(1) <= 2)
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(w @ c).max() < 1e-16
    I = np.eye(3)
    M2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.abs(M2 - I / 3).max() < 1e-15
    M3 = np.einsum("i,ia,ib,ic->abc", w, c, c, c)
    assert np.abs(M3).max() < 1e-16
    M4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    iso = (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I) + np.einsum("ad,bc->abcd", I, I)) / 9
    assert np.abs(M4 - iso).max() < 1e-15
    # canonical order: each odd moving direction followed by its opposite
    for i in range(1, 19, 2):
        assert np.all(c[i] == -c[i + 1])
    # the brute-force transcription carries its own copy of the same table
    assert np.all(bruteforce.C == c) and np.allclose(bruteforce.W, w, rtol=0, atol=1e-16)


@pytest.mark.parametrize("trial", range(5))
def test_equilibrium_moments(trial):
    case = _case()
    f, phi, phit = _random_cell()
    r = oracle.cell(case, f, 1.2, phi, phit)
    c, _ = oracle.lattice()
    feq, rho, u = r["feq"], r["rho"], r["u"]
    assert abs(feq.sum() - phi * rho) < 1e-14
    assert np.abs(feq @ c - phi * rho * u).max() < 1e-14
    M2 = np.einsum("i,ia,ib->ab", feq, c, c)
    assert np.abs(M2 - phi * rho * (np.eye(3) / 3 + np.outer(u, u))).max() < 1e-14


@pytest.mark.parametrize("forch", [0, 1])
def test_velocity_solves_implicit_equation(forch):
    """u = (phi rho)^-1 (sum f c + rho f(u)/2) with f(u) the drag (+ body force)."""
    case = _case(forchheimer=forch, g=(3e-5, -2e-5, 1e-5), d=1.5)
    for _ in range(5):
        f, phi, phit = _random_cell(phi=RNG.uniform(0.6, 0.95))
        r = oracle.cell(case, f, 1.0, phi, phit)
        c, _ = oracle.lattice()
        m = f @ c
        rho, u = r["rho"], r["u"]
        k = phi ** 3 * 1.5 ** 2 / (180 * (1 - phi) ** 2)
        CF = 1.75 / np.sqrt(150 * phi ** 3) if forch else 0.0
        g = np.array(case.porous["g"])
        drag = -phi ** 2 * 0.1 / k * u - phi ** 3 * CF / np.sqrt(k) * np.linalg.norm(u) * u
        rhs = (m + 0.5 * rho * (g + drag)) / (phi * rho)
        assert np.abs(u - rhs).max() < 1e-15
        assert np.abs(r["F"] - rho * (g + drag)).max() < 1e-15


def test_velocity_matches_remark_fixed_point_iteration():
    """The Remark's iteration u_{m+1} = X_m^{-1} v, X_m = A + |u_m| B with K = kI
    converges to the closed-form velocity, and every iterate obeys |u_m| <= |v|."""
    case = _case(forchheimer=1, d=1.2, g=(0.0, 0.0, 0.0))
    c, _ = oracle.lattice()
    for _ in range(5):
        phi = RNG.uniform(0.6, 0.95)
        f, _, phit = _random_cell(phi=phi, amp=0.2)
        r = oracle.cell(case, f, 1.0, phi, phit)
        rho = f.sum() / phi
        v = (f @ c) / (phi * rho)
        k = phi ** 3 * 1.2 ** 2 / (180 * (1 - phi) ** 2)
        CF = 1.75 / np.sqrt(150 * phi ** 3)
        A = np.eye(3) * (1 + phi * 0.1 / (2 * k))
        B = np.eye(3) * (phi ** 2 * CF / 2 / np.sqrt(k))
        um = v.copy()
        for _ in range(200):
            um = np.linalg.solve(A + np.linalg.norm(um) * B, v)
            assert np.linalg.norm(um) <= np.linalg.norm(v) * (1 + 1e-15)
        assert np.abs(um - r["u"]).max() < 1e-15


def test_porosity_one_reduces_to_bgk_guo():
    """phi = 1: no medium (1/k = 0), u = (m + F/2)/rho, Omega^phi = 0 and the
    collision is the textbook BGK step with Guo forcing."""
    case = _case(g=(1e-4, 0, 0))
    c, w = oracle.lattice()
    f, _, _ = _random_cell(phi=1.0)
    r = oracle.cell(case, f, 1.3, 1.0, np.ones(19))
    rho = f.sum()
    u = (f @ c + 0.5 * rho * np.array([1e-4, 0, 0])) / rho
    assert np.abs(r["u"] - u).max() < 1e-16
    om = r["omega"]
    cu = c @ u
    feq = w * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * u @ u)
    F = rho * np.array([1e-4, 0, 0])
    guo = w * (1 - om / 2) * (3 * (c - u) @ F + 9 * cu * (c @ F))
    assert np.abs(r["q"] - (f - om * (f - feq) + guo)).max() < 1e-16


@pytest.mark.parametrize("trial", range(5))
def test_guo_term_moments(trial):
    """Extract the forcing term from one collision and check its moments:
    0, (1 - omega/2) F and (1 - omega/2)(u F + F u)."""
    case = _case(g=(2e-5, 1e-5, -3e-5), d=1.5, forchheimer=1)
    c, w = oracle.lattice()
    f, phi, phit = _random_cell(phi=RNG.uniform(0.6, 0.95))
    r = oracle.cell(case, f, 1.1, phi, phit)
    om, rho, u, F = r["omega"], r["rho"], r["u"], r["F"]
    G = r["q"] - f + om * (f - r["feq"]) - w * rho * (phit - phi)
    assert abs(G.sum()) < 1e-15
    assert np.abs(G @ c - (1 - om / 2) * F).max() < 1e-15
    M2 = np.einsum("i,ia,ib->ab", G, c, c)
    assert np.abs(M2 - (1 - om / 2) * (np.outer(u, F) + np.outer(F, u))).max() < 1e-15


@pytest.mark.parametrize("trial", range(5))
def test_collision_mass_and_momentum(trial):
    """Per cell: sum q = sum f + sum w rho (phi~ - phi) and
    sum q c = m + F + sum w rho (phi~ - phi) c."""
    case = _case(g=(2e-5, 1e-5, -3e-5), d=1.5, forchheimer=1)
    c, w = oracle.lattice()
    f, phi, phit = _random_cell(phi=RNG.uniform(0.6, 0.95))
    r = oracle.cell(case, f, 0.9, phi, phit)
    rho = r["rho"]
    jump = w * rho * (phit - phi)
    assert abs(r["q"].sum() - f.sum() - jump.sum()) < 1e-15
    assert np.abs(r["q"] @ c - (f @ c + r["F"] + jump @ c)).max() < 1e-15


def test_second_moment_and_shear_rate():
    """Pi is symmetric-stored as xx yy zz xy xz yz; the shear rate is
    omega_prev |Pi|_F / (c_s^2 rho) with the full Frobenius norm."""
    case = _case(g=(2e-5, 0, 0))
    c, _ = oracle.lattice()
    f, phi, phit = _random_cell(phi=1.0)
    om_prev = 1.37
    r = oracle.cell(case, f, om_prev, 1.0, np.ones(19))
    P = np.zeros((3, 3))
    for k in range(6):
        P[PA[k], PB[k]] = P[PB[k], PA[k]] = r["Pi"][k]
    neq = np.einsum("i,ia,ib->ab", f - r["feq"], c, c)
    F, u = r["F"], r["u"]
    assert np.abs(P - neq - 0.5 * (np.outer(F, u) + np.outer(u, F))).max() < 1e-16
    assert abs(r["shear"] - om_prev * np.linalg.norm(P) * 3 / r["rho"]) < 1e-14


def test_carreau_yasuda_limits():
    c, w = oracle.lattice()
    # rest: Pi = 0 -> shear 0 -> nu = nu0 -> textbook omega = 1/(3 nu0 + 1/2) at rho = 1
    case = _case(g=(0.0, 0.0, 0.0))
    feq = w * 1.0
    r = oracle.cell(case, feq, 1.0, 1.0, np.ones(19))
    assert r["shear"] < 1e-14 and abs(r["nu"] - 0.1) < 1e-15
    assert abs(r["omega"] - 1 / (3 * 0.1 + 0.5)) < 1e-15
    # n = 1 or lambda = 0: Newtonian with nu0 at any shear
    f, _, _ = _random_cell(phi=1.0, amp=0.1)
    for kw in (dict(n=1.0), dict(lam=0.0)):
        r = oracle.cell(_case(**kw), f, 1.2, 1.0, np.ones(19))
        assert r["shear"] > 0 and abs(r["nu"] - 0.1) < 1e-16
    # huge lambda: power-law asymptote nu ~ nu_inf + (nu0 - nu_inf)(lambda gamma)^(n-1)
    cs = _case(lam=1e9)
    r = oracle.cell(cs, f, 1.2, 1.0, np.ones(19))
    lg = 1e9 * r["shear"]
    assert abs(r["nu"] - (0.01 + 0.09 * lg ** (0.36 - 1))) < 1e-12
    # omega relation: omega = 2 rho c_s^2 / (2 nu + rho c_s^2) <=> nu = c_s^2 (1/omega - 1/2) at rho = 1 (textbook)
    for nu in (0.01, 0.05, 0.3):
        cc = _case(nu0=nu, nu_inf=nu, g=(0.0, 0.0, 0.0))
        r = oracle.cell(cc, w * 1.0, 1.0, 1.0, np.ones(19))
        assert abs((1 / r["omega"] - 0.5) / 3 - nu) < 1e-15


@pytest.mark.parametrize("trial", range(5))
def test_zou_he_inlet_closure(trial):
    c, w = oracle.lattice()
    f = w * (1 + 0.1 * RNG.standard_normal(19))
    u = np.array([RNG.uniform(0, 0.1), RNG.uniform(-0.02, 0.02), RNG.uniform(-0.02, 0.02)])
    g = oracle.zouhe_inlet(f, *u)
    rho = g.sum()
    assert np.abs(g @ c - rho * u).max() < 1e-15
    # only the five populations with c_x = +1 change
    assert np.all(g[c[:, 0] != 1] == f[c[:, 0] != 1])


@pytest.mark.parametrize("trial", range(5))
def test_zou_he_outlet_closure(trial):
    c, w = oracle.lattice()
    f = w * (1 + 0.1 * RNG.standard_normal(19))
    rho_out = RNG.uniform(0.98, 1.02)
    g = oracle.zouhe_outlet(f, rho_out)
    assert abs(g.sum() - rho_out) < 1e-15
    m = g @ c
    assert abs(m[1]) < 1e-16 and abs(m[2]) < 1e-16
    assert np.all(g[c[:, 0] != -1] == f[c[:, 0] != -1])
