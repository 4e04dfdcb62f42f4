"""Pins of the oracle's anisotropic permeability (the Remark of the method
section): K = k(phi) M with a symmetric positive definite shape M, and the
fixed-point iteration u_{m+1} = (A + |u_m| B)^-1 v from u_0 = v with
A = Id + (phi nu / 2) K^-1 and B = (phi^2 C_F / 2) K^-1/2.

* M = Id reduces to the isotropic closed form of u (and of the force).
* The converged u solves the implicit equation (A + |u| B) u = v, with K^-1/2
  taken from NumPy's eigen-decomposition (not the oracle's).
* Successive iterates contract at least at the Remark's rate
  q = ||(A + |v| B)^-1 |v| B||.
* Without the Forchheimer term one iteration is already exact (u = A^-1 v).
* The whole step agrees with the dense NumPy transcription (test_oracle_lattice).
"""

import numpy as np
import pytest

import oracle
from synth import channel_case

RNG = np.random.default_rng(77)


def _spd():
    Qm, _ = np.linalg.qr(RNG.standard_normal((3, 3)))
    M = Qm @ np.diag(RNG.uniform(0.3, 3.0, 3)) @ Qm.T
    return M, np.array([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]])


def _case(aniso=None, iters=8, forch=1):
    c = channel_case(4)
    c.porous = dict(c.porous, forchheimer=forch, nu_d=0.1, kc=180.0, d=2.0)
    if aniso is not None:
        c.porous["aniso"] = tuple(aniso)
        c.porous["aniso_iters"] = iters
    return c


def _cell_state(phi):
    c, w = oracle.lattice()
    u = RNG.uniform(-0.08, 0.08, 3)
    cu = c @ u
    f = w * phi * 1.01 * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * u @ u) * (1 + 0.03 * RNG.standard_normal(19))
    return f


def _v_and_tensors(case, f, phi, M):
    c, _ = oracle.lattice()
    po = case.porous
    rho = f.sum() / phi
    v = (f @ c) / (phi * rho) + np.asarray(po["g"]) / (2 * phi)
    invk = po["kc"] * (1 - phi) ** 2 / (po["d"] ** 2 * phi ** 3)
    cf = 1.75 / np.sqrt(150 * phi ** 3) if po["forchheimer"] else 0.0
    lam, V = np.linalg.eigh(M)
    Kinv = invk * np.linalg.inv(M)
    Khalf = np.sqrt(invk) * (V @ np.diag(lam ** -0.5) @ V.T)
    A = np.eye(3) + 0.5 * phi * po["nu_d"] * Kinv
    B = 0.5 * phi ** 2 * cf * Khalf
    return rho, v, A, B, Kinv, Khalf, cf


@pytest.mark.parametrize("phi", [0.55, 0.8, 0.97])
def test_identity_shape_is_the_isotropic_closed_form(phi):
    f = _cell_state(phi)
    phit = np.full(19, phi)
    iso = oracle.cell(_case(), f, 1.2, phi, phit)
    ani = oracle.cell(_case((1, 1, 1, 0, 0, 0), iters=60), f, 1.2, phi, phit)
    for k in ("u", "F", "q"):
        assert np.abs(ani[k] - iso[k]).max() < 1e-15 * max(1.0, np.abs(iso[k]).max()) * 10


@pytest.mark.parametrize("phi", [0.55, 0.8])
def test_converged_velocity_solves_the_implicit_equation(phi):
    M, m6 = _spd()
    case = _case(m6, iters=60)
    f = _cell_state(phi)
    r = oracle.cell(case, f, 1.2, phi, np.full(19, phi))
    rho, v, A, B, Kinv, Khalf, cf = _v_and_tensors(case, f, phi, M)
    u = r["u"]
    res = (A + np.linalg.norm(u) * B) @ u - v
    assert np.abs(res).max() < 1e-15
    # the force is the tensor drag of that velocity
    po = case.porous
    F = rho * (np.asarray(po["g"]) - phi ** 2 * po["nu_d"] * Kinv @ u - phi ** 3 * cf * np.linalg.norm(u) * Khalf @ u)
    assert np.abs(r["F"] - F).max() < 1e-15


def test_iteration_contracts_at_the_remark_rate():
    phi = 0.6
    M, m6 = _spd()
    f = _cell_state(phi)
    us = [oracle.cell(_case(m6, iters=n), f, 1.2, phi, np.full(19, phi))["u"] for n in range(1, 7)]
    rho, v, A, B, _, _, _ = _v_and_tensors(_case(m6), f, phi, M)
    vn = np.linalg.norm(v)
    q = np.linalg.norm(np.linalg.solve(A + vn * B, vn * B), 2)
    assert q < 1
    d = [np.linalg.norm(us[k + 1] - us[k]) for k in range(len(us) - 1)]
    for k in range(len(d) - 1):
        assert d[k + 1] <= q * d[k] * (1 + 1e-9) + 1e-18
    # and the first iterate is A + |v| B applied to v
    assert np.abs(us[0] - np.linalg.solve(A + vn * B, v)).max() < 1e-16


def test_darcy_only_is_exact_after_one_iteration():
    phi = 0.7
    M, m6 = _spd()
    f = _cell_state(phi)
    case1 = _case(m6, iters=1, forch=0)
    r1 = oracle.cell(case1, f, 1.2, phi, np.full(19, phi))
    r5 = oracle.cell(_case(m6, iters=5, forch=0), f, 1.2, phi, np.full(19, phi))
    rho, v, A, _, _, _, _ = _v_and_tensors(case1, f, phi, M)
    assert np.abs(r1["u"] - np.linalg.solve(A, v)).max() < 1e-16
    assert np.abs(r5["u"] - r1["u"]).max() < 1e-16


def test_six_iterations_reach_the_fixed_point():
    """The iteration count used in the tests and the benchmark (6) already gives
    the converged velocity at lattice speeds: 6 and 40 iterations agree to
    rounding over several steps of a porous lattice with the 3:1 shape."""
    from synth import aniso_shape, tiny_case

    runs = {}
    for it in (6, 40):
        case = tiny_case("periodic", seed=3)
        case.porous = dict(case.porous, forchheimer=1, aniso=aniso_shape(), aniso_iters=it, g=(5e-4, 2e-4, -1e-4))
        o = oracle.Oracle(case)
        f, om = o.init()
        o.run(f, om, 0, 20)
        runs[it] = o.moments(f, om, 20)["u"]
    assert np.abs(runs[6] - runs[40]).max() < 1e-15 * max(1.0, np.abs(runs[40]).max()) + 1e-17
    assert np.abs(runs[40]).max() > 1e-5
