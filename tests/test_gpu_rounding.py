"""Mass and momentum under the 16-bit storage roundings (evidence for the
choice of the default rounding).

Uniform flow: a 24^3 box periodic in every axis, porosity 1, body force g along
x, from rest.  In exact arithmetic the mass keeps its initial value M0 and the
momentum grows by g times the mass every step.  Every cell sees the same state,
so a deterministic rounding (to nearest, or conserving) makes the same error in
all N cells at every step and the total error grows with N; stochastic
rounding's errors are independent and of mean zero, so they add up like the
square root of N.

Porous flow: the same box with a Gaussian-random-field porosity (the
porosity-jump term moves mass between cells), against the FP64 oracle's mass
and momentum after the same number of steps; reported for every rounding."""

import numpy as np
import pytest

import oracle
from paper_2402_10809_amd import Solver
from synth import periodic_box_case

pytestmark = pytest.mark.gpu

ROUNDINGS = ("stochastic", "conserve", "nearest")


def say(msg):
    print(msg, flush=True)


def test_uniform_flow_mass_and_momentum():
    n, steps, g = 24, 2000, 1e-5
    case = periodic_box_case(nx=n, ny=n, nz=n, ell=3.0, g=g)
    case.phi = np.ones_like(case.phi)
    err = {}
    for storage in ("fp16", "bf16"):
        for rounding in ROUNDINGS:
            s = Solver.from_case(case, storage=storage, rounding=rounding)
            m0 = s.diagnostics()["mass"]
            s.step(steps)
            d = s.diagnostics()
            dm = abs(d["mass"] - m0) / m0
            p_exact = steps * g * m0
            dp = abs(d["mom_x"] - p_exact) / p_exact
            err[storage, rounding] = (dm, dp)
            say(f"  uniform flow {storage}/{rounding}: mass drift {dm:.3e}, momentum error {dp:.3e} "
                f"(u = {d['max_u']:.3e})")
            s.close()
    for storage in ("fp16", "bf16"):
        det = min(err[storage, "conserve"][1], err[storage, "nearest"][1])
        assert err[storage, "stochastic"][1] < 0.1 * det
        assert err[storage, "stochastic"][0] < 1e-5


def test_porous_flow_mass_and_momentum_against_oracle():
    n, steps, g = 24, 2000, 1e-5
    case = periodic_box_case(nx=n, ny=n, nz=n, ell=3.0, g=g)
    o = oracle.Oracle(case)
    f, om = o.init()
    c, _ = oracle.lattice()
    m0 = f.sum()
    o.run(f, om, 0, steps)
    m_ref = f.sum()
    p_ref = (f.T @ c).sum(0)
    say(f"  oracle: mass change {abs(m_ref - m0) / m0:.3e}, momentum {p_ref[0]:.6e}")
    for storage in ("fp32", "fp16", "bf16"):
        for rounding in (ROUNDINGS if storage != "fp32" else ("stochastic",)):
            s = Solver.from_case(case, storage=storage, rounding=rounding)
            s.step(steps)
            d = s.diagnostics()
            dm = abs(d["mass"] - m_ref) / m_ref
            dp = np.abs(np.array([d["mom_x"], d["mom_y"], d["mom_z"]]) - p_ref).max() / abs(p_ref[0])
            say(f"  porous flow {storage}/{rounding}: mass error {dm:.3e}, momentum error {dp:.3e}")
            assert np.isfinite(dm) and np.isfinite(dp)
            if storage == "fp32":
                assert dm < 1e-7 and dp < 1e-5
            s.close()
