"""Pins of the FP64 oracle's full step: brute-force agreement on tiny lattices,
the rest state, mass and momentum budgets, and translation invariance."""

import numpy as np
import pytest

import oracle
from oracle import bruteforce as bf
from synth import as_d3q27, channel_case, tiny_case, tiny_random


def _random_state(o, seed, amp=0.1):
    rng = np.random.default_rng(seed)
    f0, om0 = o.init()
    known = f0 != 0
    f = np.ascontiguousarray(f0 * (1 + amp * rng.standard_normal(f0.shape)) * known)
    om = np.ascontiguousarray(om0 * (1 + 0.2 * rng.random(o.nf)))
    return f, om


def _dense(case, cells, f, om):
    q = f.shape[0]
    fd = np.zeros((q, case.n_box))
    fd[:, cells] = f
    od = np.zeros(case.n_box)
    od[cells] = om
    return fd.reshape(q, case.nz, case.ny, case.nx), od.reshape(case.nz, case.ny, case.nx)


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("seed", range(32))
def test_random_lattices_match_bruteforce(seed, q):
    """Random small lattices (extents 1..10, random periodic axes, open faces
    with either outflow, random solids, porosity and body force): C++ oracle
    vs the dense transcription over 6 steps."""
    case = tiny_random(seed)
    if q == 27:
        case = as_d3q27(case)
    o = oracle.Oracle(case)
    cells = o.cells()
    f, om = _random_state(o, seed)
    fd, od = _dense(case, cells, f, om)
    t0 = 3
    o.run(f, om, t0, 6)
    for s in range(6):
        fd, od, _ = bf.step(case, fd, od, t0 + s)
    assert np.abs(fd.reshape(fd.shape[0], -1)[:, cells] - f).max() < 1e-13
    assert np.abs(od.reshape(-1)[cells] - om).max() < 1e-13


@pytest.mark.parametrize("kind", ["open", "open_wave", "open_extrap", "periodic", "periodic_aniso", "periodic3",
                                  "bulk", "degenerate", "open_q27", "open_extrap_q27", "periodic_q27",
                                  "periodic3_q27", "bulk_q27", "degenerate_q27"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_dense_bruteforce(kind, seed):
    """Compact-list C++ oracle vs dense-array NumPy transcription: 1 and 10 steps
    from a random non-equilibrium state with walls, open faces, periodic wrap and
    heterogeneous porosity, on D3Q19 and D3Q27."""
    q27 = kind.endswith("_q27")
    case = tiny_case(kind[:-4] if q27 else kind, seed=seed)
    if q27:
        case = as_d3q27(case)
    o = oracle.Oracle(case)
    cells = o.cells()
    f, om = _random_state(o, seed)
    fd, od = _dense(case, cells, f, om)
    t0 = 7
    f1, o1 = f.copy(), om.copy()
    o.run(f1, o1, t0, 1)
    fd1, od1, _ = bf.step(case, fd, od, t0)
    assert np.abs(fd1.reshape(fd1.shape[0], -1)[:, cells] - f1).max() < 1e-14
    assert np.abs(od1.reshape(-1)[cells] - o1).max() < 1e-13
    o.run(f1, o1, t0 + 1, 9)
    for s in range(1, 10):
        fd1, od1, _ = bf.step(case, fd1, od1, t0 + s)
    assert np.abs(fd1.reshape(fd1.shape[0], -1)[:, cells] - f1).max() < 1e-13
    # moments of the state agree too
    m = o.moments(f1, o1, t0 + 10)
    _, _, fields = bf.step(case, fd1, od1, t0 + 10)
    assert np.abs(fields["u"].reshape(3, -1)[:, cells] - m["u"]).max() < 1e-13
    assert np.abs(fields["shear"].reshape(-1)[cells] - m["shear"]).max() < 1e-12


@pytest.mark.parametrize("kind", ["open", "open_extrap", "periodic", "open_q27", "periodic_q27"])
def test_rest_state_is_stationary(kind):
    """Fluid at rest with heterogeneous porosity, walls and (zero-velocity)
    open faces stays at rest: the porosity-jump term, the porosity-shifted
    equilibrium and bounce-back are mutually consistent."""
    q27 = kind.endswith("_q27")
    kind = kind[:-4] if q27 else kind
    case = tiny_case(kind, seed=3)
    if q27:
        case = as_d3q27(case)
    case.porous = dict(case.porous, g=(0.0, 0.0, 0.0))
    case.wave = (0.0, 0.0, 1.0)
    if kind == "open_extrap":
        # the extrapolation mixes populations of the last three layers, which
        # carry their cells' porosity at rest: uniform porosity there
        case.phi[:, :, -3:] = np.where(case.solid[:, :, -3:] == 0, 1.0, 0.0)
    o = oracle.Oracle(case)
    f, om = o.init()
    f1, o1 = f.copy(), om.copy()
    o.run(f1, o1, 0, 25)
    assert np.abs(f1 - f).max() < 1e-15
    m = o.moments(f1, o1, 25)
    assert np.abs(m["u"]).max() < 1e-15
    assert np.abs(m["rho"] - 1).max() < 1e-14


@pytest.mark.parametrize("q", [19, 27])
def test_mass_exact_for_uniform_porosity(q):
    case = tiny_case("periodic", seed=4)
    case.lattice = q
    case.phi = np.where(case.solid == 0, 0.8, 0.0).astype(np.float32)
    o = oracle.Oracle(case)
    f, om = _random_state(o, 4)
    m0 = f.sum()
    o.run(f, om, 0, 300)
    assert abs(f.sum() - m0) / m0 < 1e-13


def test_mass_budget_heterogeneous_porosity():
    """Closed domain: each step changes the mass by exactly
    sum_x rho(x) sum_i w_i (phi~(x + c_i) - phi(x))."""
    case = tiny_case("periodic", seed=5)
    o = oracle.Oracle(case)
    cells = o.cells()
    kinds = bf._link_kinds(case)
    phi = np.where(case.solid == 0, case.phi.astype(np.float64), 1.0)
    jump = np.zeros(case.phi.shape)
    for i in range(19):
        nb = np.roll(phi, shift=tuple(-int(c) for c in bf.C[i][::-1]), axis=(0, 1, 2))
        jump += bf.W[i] * np.where(kinds[i] == 0, nb - phi, 0.0)
    jump = jump.reshape(-1)[cells]
    f, om = _random_state(o, 5)
    for t in range(20):
        rho = o.moments(f, om, t)["rho"]
        before = f.sum()
        o.run(f, om, t, 1)
        assert abs(f.sum() - before - (rho * jump).sum()) < 1e-15 * before


@pytest.mark.parametrize("q", [19, 27])
def test_momentum_gain_equals_body_force(q):
    """Periodic box without walls, porosity 1: total momentum grows by
    g * sum_x rho(x) per step."""
    case = channel_case(6, g=3e-5)
    case.lattice = q
    case.solid[:] = 0
    case.periodic = (True, True, True)
    case.phi = np.ones(case.phi.shape, np.float32)
    case.porous = dict(case.porous, g=(3e-5, -1e-5, 2e-5))
    o = oracle.Oracle(case)
    f, om = _random_state(o, 6, amp=0.05)
    c, _ = oracle.lattice(q)
    g = np.array(case.porous["g"])
    for t in range(10):
        rho = o.moments(f, om, t)["rho"]
        p0 = (f.T @ c).sum(0)
        o.run(f, om, t, 1)
        p1 = (f.T @ c).sum(0)
        assert np.abs(p1 - p0 - g * rho.sum()).max() < 1e-15


def test_channel_translation_invariance():
    """The 32^3 channel from rest equals the 1x32x1 channel in every column."""
    big = channel_case(32)
    small = channel_case(32, nx=1, nz=1)
    ob, os_ = oracle.Oracle(big), oracle.Oracle(small)
    fb, omb = ob.init()
    fs, oms = os_.init()
    ob.run(fb, omb, 0, 60)
    os_.run(fs, oms, 0, 60)
    ub = ob.moments(fb, omb, 60)["u"][0].reshape(32, 30, 32)
    us = os_.moments(fs, oms, 60)["u"][0]
    assert np.abs(ub - us[None, :, None]).max() < 1e-17 + 1e-12 * np.abs(us).max()


def test_deterministic():
    case = tiny_case("open", seed=6)
    o = oracle.Oracle(case)
    f, om = _random_state(o, 6)
    a, b = (f.copy(), om.copy()), (f.copy(), om.copy())
    o.run(*a, 0, 15)
    o.run(*b, 0, 15)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_inflow_waveform_definition():
    """The pre-run grows linearly from 0 to the waveform's starting value over
    R steps (the simulation section's ramp); afterwards the sampled period is
    reproduced at its sample times, interpolated linearly in between and
    repeated every period."""
    case = tiny_case("open_wave", seed=0)
    o = oracle.Oracle(case)
    R = case.ramp_steps
    tab = case.wave_table
    T = case.wave[2]
    n = tab.size
    amp = [o.amplitude(t) for t in range(R + 4 * int(T) + 1)]
    assert amp[0] == 0.0
    for t in range(R + 1):
        assert abs(amp[t] - tab[0] * t / R) < 1e-15
    # sample times s = k T / n that fall on integer steps (T = 13, n = 9: k = 0 and 9 -> s = 0, 13)
    for m in range(4):
        assert abs(o.amplitude(R + int(T) * m) - tab[0]) < 1e-15
    # every value lies on the piecewise-linear interpolant of the samples
    for t in range(R, R + 3 * int(T)):
        sp = (t - R) % T
        pos = sp / T * n
        k = int(pos)
        lo, hi = tab[k], tab[(k + 1) % n]
        assert min(lo, hi) - 1e-15 <= o.amplitude(t) <= max(lo, hi) + 1e-15
        assert abs(o.amplitude(t) - o.amplitude(t + int(T))) < 1e-15
