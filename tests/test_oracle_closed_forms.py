"""Closed-form pins of the FP64 oracle in a plane channel (1 x (H+2) x 1 cells,
periodic in x and z, solid layers at y = 0 and y = H+1, halfway bounce-back walls
at y = 0.5 and y = H + 0.5).

* Newtonian Poiseuille: BGK with halfway bounce-back reproduces the parabola
  exactly at tau = 1/2 + sqrt(3)/4 (textbook "magic" relaxation time).
* Brinkman flow in a uniformly porous channel (model section: Darcy drag with
  the Kozeny-Carman permeability): phi nu u'' - phi^2 nu u / k + g = 0.
* Carreau-Yasuda channel: nu(sqrt(2)|u'|) |u'| = g |s| solved per point and
  integrated (1-D quadrature); also the shear rate the step reports from Pi
  equals sqrt(2)|u'| of that profile (the model section's Frobenius norm of the
  full symmetric gradient).
* Start-up flow of the 32^3 channel configuration: Fourier series.

Second-order convergence (error ratio >= 3 when H doubles) is asserted where the
discrete solution is not exact.
"""

import numpy as np
import pytest
from scipy import integrate, optimize

import oracle
from synth import channel_case


def _run(case, steps):
    o = oracle.Oracle(case)
    f, om = o.init()
    o.run(f, om, 0, steps)
    return o.moments(f, om, steps)


def test_poiseuille_exact_at_magic_tau():
    nu = np.sqrt(3) / 12  # tau = 3 nu + 1/2 = 1/2 + sqrt(3)/4
    H, g = 30, 1e-6
    c = channel_case(H + 2, nx=1, nz=1, g=g, rheology=dict(nu0=nu, nu_inf=nu, lam=0.0, n=1.0, a=2.0))
    m = _run(c, 40000)
    y = np.arange(1, H + 1)
    exact = g / (2 * nu) * (y - 0.5) * (H + 0.5 - y)
    assert np.abs(m["u"][0] - exact).max() / exact.max() < 1e-10
    assert np.abs(m["u"][1:]).max() < 1e-13


def _brinkman_error(H, scale):
    phi, d, g, nu = 0.7, 23.0 * scale, 1e-5 / scale ** 2, 0.1
    c = channel_case(H + 2, nx=1, nz=1, g=g, phi=phi, d=d, rheology=dict(nu0=nu, nu_inf=nu, lam=0.0, n=1.0, a=2.0))
    k = phi ** 3 * d * d / (180 * (1 - phi) ** 2)
    L, h = np.sqrt(k / phi), H / 2
    m = _run(c, 30000 * scale ** 2)
    s = np.arange(1, H + 1) - 0.5 - h
    exact = g * k / (phi ** 2 * nu) * (1 - np.cosh(s / L) / np.cosh(h / L))
    return np.abs(m["u"][0] - exact).max() / exact.max()


def test_brinkman_channel():
    e30 = _brinkman_error(30, 1)  # Brinkman length L = sqrt(k/phi) = 4 cells
    e60 = _brinkman_error(60, 2)
    assert e30 < 5e-3
    assert e60 < 1.5e-3
    assert e30 / e60 > 3.0


def _cy_profile(H, g, rh):
    h = H / 2

    def nu_cy(gd):
        return rh["nu_inf"] + (rh["nu0"] - rh["nu_inf"]) * (1 + (rh["lam"] * gd) ** rh["a"]) ** ((rh["n"] - 1) / rh["a"])

    def du(sabs):
        if sabs == 0:
            return 0.0
        hi = g * sabs / rh["nu_inf"] * 1.01
        return optimize.brentq(lambda x: nu_cy(np.sqrt(2) * x) * x - g * sabs, 0, hi, xtol=1e-17, rtol=1e-14)

    s = np.abs(np.arange(1, H + 1) - 0.5 - h)
    u = np.array([integrate.quad(du, si, h, epsabs=1e-15, epsrel=1e-12)[0] for si in s])
    shear = np.array([np.sqrt(2) * du(si) for si in s])
    return u, shear


def _cy_error(H):
    r = H / 30
    rh = dict(nu0=0.1, nu_inf=0.01, lam=500.0 * r ** 2, n=0.36, a=2.0)
    g = 2e-5 / r ** 3
    c = channel_case(H + 2, nx=1, nz=1, g=g, rheology=rh)
    m = _run(c, int(80000 * r ** 2))
    u, shear = _cy_profile(H, g, rh)
    assert rh["lam"] * shear.max() > 4  # well into the shear-thinning range
    return np.abs(m["u"][0] - u).max() / u.max(), np.abs(m["shear"] - shear).max() / shear.max()


def test_carreau_yasuda_channel():
    e30, s30 = _cy_error(30)
    e60, s60 = _cy_error(60)
    assert e30 < 4e-3 and e60 < 1e-3
    assert e30 / e60 > 3.0
    assert s30 < 1e-4 and s60 < 2e-5


def test_config0_startup_matches_fourier_series():
    """The 32^3 channel configuration (Carreau-Yasuda, g = 1e-6) after 2000 steps
    against Newtonian start-up flow with nu = nu0: at this forcing lambda*gamma
    stays near 0.01, so the viscosity differs from nu0 by ~1e-5 relative."""
    c = channel_case(32, nx=1, nz=1)
    T = 2000
    m = _run(c, T)
    H, nu, g = 30.0, 0.1, 1e-6
    eta = (np.arange(1, 31) - 0.5) / H
    series = np.zeros_like(eta)
    for n in range(1, 400, 2):
        series += 8 / (n * np.pi) ** 3 * np.sin(n * np.pi * eta) * np.exp(-(n * np.pi) ** 2 * nu * T / H ** 2)
    exact = g * H * H / (2 * nu) * (eta * (1 - eta) - series)
    assert np.abs(m["u"][0] - exact).max() / exact.max() < 1e-2
    assert 50 * m["shear"].max() < 0.02
