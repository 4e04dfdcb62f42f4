"""GPU parity of the HIP step against the FP64 oracle, through the C ABI.

Metric for velocities (and shear rates): max over fluid cells of |u_gpu - u_ref|
divided by max over fluid cells of |u_ref| ("max-relative"), and the relative
L2 norm for the reduced-precision storage forms.  The FP32 bound 1e-5 after
1000 steps is the target of the method's FP32 path; the FP16 bound 1e-3
(relative L2) is the target for FP16 storage on the aneurysm case.
"""

import numpy as np
import pytest

import oracle
from paper_2402_10809_amd import Solver, lbm
from synth import as_d3q27, channel_case, make_config, tiny_case, tiny_random

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def _oracle_run(case, steps):
    o = oracle.Oracle(case)
    f, om = o.init()
    o.run(f, om, 0, steps)
    return o, f, om, o.moments(f, om, steps)


def _gpu_fields(s):
    m = s.moments(sigma=True, tau=True)
    idx = s.fluid_index()
    out = {}
    for k, v in m.items():
        a = v.cpu().numpy()
        out[k] = a.reshape(a.shape[0], -1)[:, idx] if a.ndim == 4 else a.reshape(-1)[idx]
    return out


def max_rel(a, ref):
    """max_x |a(x) - ref(x)| / max_x |ref(x)| for vector (3, n) or scalar (n,) fields."""
    if a.ndim == 2:
        return float(np.sqrt(((a - ref) ** 2).sum(0)).max() / np.sqrt((ref ** 2).sum(0)).max())
    return float(np.abs(a - ref).max() / np.abs(ref).max())


def rel_l2(a, ref):
    return float(np.sqrt(((a - ref) ** 2).sum()) / np.sqrt((ref ** 2).sum()))


def _tiny_any(kind, seed):
    """tiny_case, with a "_q27" suffix for the D3Q27 velocity set."""
    if kind.endswith("_q27"):
        return as_d3q27(tiny_case(kind[:-4], seed=seed))
    return tiny_case(kind, seed=seed)


@pytest.mark.parametrize("kind", ["open", "open_wave", "open_extrap", "periodic", "periodic_aniso", "periodic3",
                                  "bulk", "degenerate", "open_q27", "open_extrap_q27", "periodic_q27",
                                  "periodic3_q27", "bulk_q27", "degenerate_q27"])
@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("t0", [0, 1])
def test_one_step_from_random_state(kind, seed, t0):
    """Every cell type (walls, open faces, periodic wrap, porosity jumps, waves
    of interior cells): one step, even (t0 = 0) or odd (t0 = 1), from a random
    non-equilibrium state, on D3Q19 and D3Q27."""
    case = _tiny_any(kind, seed)
    say(f"one step: {case.name} seed={seed} t0={t0} box={case.nx}x{case.ny}x{case.nz}")
    o = oracle.Oracle(case)
    f0, om0 = o.init()
    rng = np.random.default_rng(seed)
    known = f0 != 0
    f = np.ascontiguousarray(f0 * (1 + 0.1 * rng.standard_normal(f0.shape)) * known)
    om = np.ascontiguousarray((om0 * (1 + 0.2 * rng.random(o.nf))).astype(np.float32).astype(np.float64))
    s = Solver.from_case(case)
    assert np.array_equal(s.fluid_index(), o.cells())
    s.step(t0)
    s.set_state(f, om.astype(np.float32))
    g0, gom0 = s.get_state()
    assert np.abs(g0 - f).max() < 1e-8
    s.step(1)
    g1, gom1 = s.get_state()
    o.run(f, om, t0, 1)
    assert np.all(g1[~known] == 0)
    err = np.abs(g1 - f).max()
    say(f"  max |f_gpu - f_oracle| = {err:.3e}, omega err = {np.abs(gom1 - om).max():.3e}")
    assert err < 2e-6
    assert np.abs(gom1 - om).max() < 2e-6


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("seed", range(32))
def test_one_step_random_lattices(seed, q):
    """Random small lattices (extents 1..10, random periodic axes, open faces
    with either outflow, random solids and porosity): an even and an odd step
    from a random state against the oracle."""
    case = tiny_random(seed)
    if q == 27:
        case = as_d3q27(case)
    say(f"random lattice: {case.name} q={q} box={case.nx}x{case.ny}x{case.nz} periodic={case.periodic} "
        f"outlet={case.outlet}")
    o = oracle.Oracle(case)
    f0, om0 = o.init()
    rng = np.random.default_rng(seed)
    known = f0 != 0
    s = Solver.from_case(case)
    assert np.array_equal(s.fluid_index(), o.cells())
    for t0 in (0, 1):
        f = np.ascontiguousarray(f0 * (1 + 0.1 * rng.standard_normal(f0.shape)) * known)
        om = np.ascontiguousarray((om0 * (1 + 0.2 * rng.random(o.nf))).astype(np.float32).astype(np.float64))
        s.reset()
        s.step(t0)
        s.set_state(f, om.astype(np.float32))
        s.step(1)
        g1, gom1 = s.get_state()
        o.run(f, om, t0, 1)
        assert np.all(g1[~known] == 0)
        assert np.abs(g1 - f).max() < 2e-6
        assert np.abs(gom1 - om).max() < 2e-6


@pytest.mark.parametrize("arith,steps,bound", [
    ("auto", 1000, 1e-5), ("auto", 2000, 1e-5),
    ("fp64", 1000, 1e-5), ("fp64", 2000, 1e-5),
    ("fp32", 1000, 2e-5), ("fp32", 2000, 3e-5),
])
def test_channel_32cube_parity(arith, steps, bound):
    """The 1000-step bound 1e-5 is the FP32 target.  With every per-cell
    scalar rounded to FP32 once per step (arith="fp32"), the rounding of the
    density and velocity is common to all 19 directions and leaves a small
    coherent momentum error in every cell, every step (~1e-5 of the per-step
    body force g = 1e-6); divided by the relaxation rate of the slowest
    channel mode it saturates at 1-1.5e-5 of u_max.  The default FP32 path
    ("auto") re-imposes the collision's momentum balance in FP64 after the
    FP32 arithmetic, which removes that bias; "fp64" does the whole collision
    in FP64.  Both stay within 1e-5 at any step count."""
    case = channel_case(32)
    say(f"channel 32^3 Carreau-Yasuda, {steps} steps, arith={arith}")
    o, f, om, ref = _oracle_run(case, steps)
    s = Solver.from_case(case, arith=arith)
    s.step(steps)
    g = _gpu_fields(s)
    eu = max_rel(g["u"], ref["u"])
    es = max_rel(g["shear"], ref["shear"])
    say(f"  u max-rel {eu:.3e}  shear max-rel {es:.3e}")
    assert eu < bound
    assert es < 1e-4


@pytest.fixture(scope="module")
def aneurysm_ref():
    case = make_config("c1")
    steps = 1000
    say(f"oracle: aneurysm 192x128x128 ({case.n_fluid} fluid cells), {steps} steps")
    o, f, om, ref = _oracle_run(case, steps)
    return case, steps, ref


def test_aneurysm_fp32_parity(aneurysm_ref):
    case, steps, ref = aneurysm_ref
    say("gpu: aneurysm fp32")
    s = Solver.from_case(case)
    s.step(steps)
    g = _gpu_fields(s)
    eu = max_rel(g["u"], ref["u"])
    es = max_rel(g["shear"], ref["shear"])
    say(f"  u max-rel {eu:.3e}  shear max-rel {es:.3e}  rho max-abs {np.abs(g['rho'] - ref['rho']).max():.3e}")
    assert eu < 1e-5
    assert es < 1e-4
    # stress, wall shear stress and relaxation rate of the same state
    et = max_rel(g["tau"], ref["tau"])
    say(f"  sigma max-rel {max_rel(g['sigma'], ref['sigma']):.3e}  tau max-rel {et:.3e}")
    assert max_rel(g["omega"], ref["omega"]) < 1e-5
    assert max_rel(g["sigma"], ref["sigma"]) < 1e-4
    assert et < 1e-4
    # the voxel wall is the same set of cells
    assert np.array_equal(np.abs(g["tau"]).sum(0) > 0, np.abs(ref["tau"]).sum(0) > 0)


def test_aneurysm_ramp_and_sampled_waveform():
    """The simulation section's inflow: a pre-run ramp (400 steps here) to the
    start of a sampled periodic waveform (128 samples per 4000-step period),
    on the 192x128x128 aneurysm, 1000 steps, FP32 storage."""
    from synth import sampled_waveform

    case = make_config("c1")
    case.ramp_steps = 400
    case.wave_table = sampled_waveform(128)
    steps = 1000
    say(f"ramp + sampled waveform: aneurysm {case.nx}x{case.ny}x{case.nz}, {steps} steps")
    o, f, om, ref = _oracle_run(case, steps)
    s = Solver.from_case(case)
    s.step(steps)
    g = _gpu_fields(s)
    eu, es = max_rel(g["u"], ref["u"]), max_rel(g["shear"], ref["shear"])
    say(f"  u max-rel {eu:.3e}  shear max-rel {es:.3e}")
    assert eu < 1e-5 and es < 1e-4


@pytest.mark.parametrize("storage,bound_u", [("fp32", 1e-5), ("fp16", 1e-3)])
def test_aneurysm_extrapolation_outflow(storage, bound_u):
    """The paper's outflow: the 192x128x128 aneurysm with the extrapolation
    outflow, 1000 steps; FP32 by max-relative, FP16 storage by relative L2 of
    the velocity."""
    case = make_config("c1")
    case.outlet = 2
    steps = 1000
    say(f"extrapolation outflow: aneurysm {case.nx}x{case.ny}x{case.nz}, {storage}, {steps} steps")
    o, f, om, ref = _oracle_run(case, steps)
    s = Solver.from_case(case, storage=storage)
    s.step(steps)
    g = _gpu_fields(s)
    eu, el = max_rel(g["u"], ref["u"]), rel_l2(g["u"], ref["u"])
    say(f"  u max-rel {eu:.3e}  u rel-L2 {el:.3e}  shear max-rel {max_rel(g['shear'], ref['shear']):.3e}")
    assert (eu if storage == "fp32" else el) < bound_u


@pytest.mark.parametrize("storage,bound_u", [("fp32", 1e-5), ("fp16", 1e-3)])
def test_aneurysm_anisotropic_permeability(storage, bound_u):
    """The Remark's anisotropic permeability on the 192x128x128 aneurysm: a
    seeded shape with a 3:1 permeability ratio, Forchheimer drag on, six
    fixed-point iterations per cell and step; 1000 steps."""
    from synth import with_anisotropic_drag

    case = with_anisotropic_drag(make_config("c1"))
    steps = 1000
    say(f"anisotropic permeability: aneurysm {case.nx}x{case.ny}x{case.nz}, {storage}, {steps} steps")
    o, f, om, ref = _oracle_run(case, steps)
    s = Solver.from_case(case, storage=storage)
    s.step(steps)
    g = _gpu_fields(s)
    eu, el = max_rel(g["u"], ref["u"]), rel_l2(g["u"], ref["u"])
    say(f"  u max-rel {eu:.3e}  u rel-L2 {el:.3e}  shear max-rel {max_rel(g['shear'], ref['shear']):.3e}")
    assert (eu if storage == "fp32" else el) < bound_u


@pytest.mark.parametrize("storage,shift_mode,bound_u", [("fp32", 0, 1e-5), ("fp16", 0, 1e-3), ("bf16", 0, 2e-2)])
def test_aneurysm_d3q27(storage, shift_mode, bound_u):
    """The method section's D3Q27 velocity set on the 192x128x128 aneurysm,
    1000 steps: FP32 by max-relative velocity error, the 16-bit forms by
    relative L2, against the D3Q27 oracle."""
    case = as_d3q27(make_config("c1"))
    steps = 1000
    say(f"D3Q27: aneurysm {case.nx}x{case.ny}x{case.nz}, {storage}, {steps} steps")
    o, f, om, ref = _oracle_run(case, steps)
    s = Solver.from_case(case, storage=storage, shift_mode=shift_mode)
    s.step(steps)
    g = _gpu_fields(s)
    eu, el = max_rel(g["u"], ref["u"]), rel_l2(g["u"], ref["u"])
    say(f"  u max-rel {eu:.3e}  u rel-L2 {el:.3e}  shear max-rel {max_rel(g['shear'], ref['shear']):.3e}  "
        f"tau max-rel {max_rel(g['tau'], ref['tau']):.3e}")
    assert (eu if storage == "fp32" else el) < bound_u
    if storage == "fp32":
        assert max_rel(g["shear"], ref["shear"]) < 1e-4 and max_rel(g["tau"], ref["tau"]) < 1e-4


def test_d3q27_diagnostics_and_rejections():
    case = as_d3q27(tiny_case("periodic", seed=2))
    s = Solver.from_case(case)
    s.step(30)
    d = s.diagnostics()
    o = oracle.Oracle(case)
    f, om = o.init()
    o.run(f, om, 0, 30)
    c, _ = oracle.lattice(27)
    assert abs(d["mass"] - f.sum()) < 1e-5
    assert np.abs(np.array([d["mom_x"], d["mom_y"], d["mom_z"]]) - (f.T @ c).sum(0)).max() < 1e-6
    assert d["nonfinite"] == 0 and d["t"] == 30
    with pytest.raises(lbm.LBMError):
        s.adjoint(5, 10, 10, 5)


def test_extrapolation_outflow_multi_step_tiny():
    """200 steps on the tiny open case with the extrapolation outflow (one
    outflow cell without a fluid -x neighbour), state compared in full,
    including the outflow's kept unknowns."""
    case = tiny_case("open_extrap", seed=2)
    o = oracle.Oracle(case)
    f, om = o.init()
    o.run(f, om, 0, 200)
    s = Solver.from_case(case)
    s.step(200)
    g, gom = s.get_state()
    err = np.abs(g - f).max() / np.abs(f).max()
    say(f"  tiny extrapolation outflow, 200 steps: max |f_gpu - f_oracle| / max |f| = {err:.3e}")
    assert err < 1e-6


@pytest.mark.parametrize("shift_mode,arith", [(0, "fp64"), (0, "fp32"), (1, "auto"), (1, "fp64")])
def test_aneurysm_fp32_variants(aneurysm_ref, shift_mode, arith):
    case, steps, ref = aneurysm_ref
    say(f"gpu: aneurysm fp32 shift_mode={shift_mode} arith={arith}")
    s = Solver.from_case(case, shift_mode=shift_mode, arith=arith)
    s.step(steps)
    g = _gpu_fields(s)
    eu = max_rel(g["u"], ref["u"])
    es = max_rel(g["shear"], ref["shear"])
    say(f"  u max-rel {eu:.3e}  shear max-rel {es:.3e}")
    assert eu < 1e-5
    assert es < 1e-4


# Bounds of the 16-bit forms (velocity relative L2 / shear-rate relative L2):
# FP16 with the default stochastic rounding meets the FP16 target 1e-3; BF16
# keeps 8 significand bits against FP16's 11, so its bound is the target times
# 2^3.  The shear rate comes from the non-equilibrium stress, which carries the
# rounding noise of the last step undamped; it is bounded at 5x the velocity
# bound.  The deterministic roundings are options, bounded by their own
# measured regime (conserving 2.5e-4 / 2.6e-3, nearest 6.7e-4 / 1.0e-2 after
# 1000 steps): they meet the targets here but not over 20 000 steps (see the
# long-run test).
FP16_U, BF16_U = 1e-3, 8e-3


@pytest.mark.parametrize("storage,rounding,bound_u,bound_s", [
    ("fp16", "stochastic", FP16_U, 5 * FP16_U), ("bf16", "stochastic", BF16_U, 5 * BF16_U),
    ("fp16", "conserve", 5e-4, 5e-3), ("bf16", "conserve", 5e-3, 2e-2),
    ("fp16", "nearest", 1e-3, 1e-2), ("bf16", "nearest", 2e-2, 1e-1),
])
def test_aneurysm_reduced_storage(aneurysm_ref, storage, rounding, bound_u, bound_s):
    """16-bit storage against the FP64 oracle after 1000 steps (relative L2),
    in each rounding of the stored values."""
    case, steps, ref = aneurysm_ref
    say(f"gpu: aneurysm {storage} rounding={rounding}")
    s = Solver.from_case(case, storage=storage, rounding=rounding)
    s.step(steps)
    g = _gpu_fields(s)
    eu, es = rel_l2(g["u"], ref["u"]), rel_l2(g["shear"], ref["shear"])
    say(f"  {storage}/{rounding}: u rel-L2 {eu:.3e}  u max-rel {max_rel(g['u'], ref['u']):.3e}  "
        f"shear rel-L2 {es:.3e}")
    assert eu < bound_u
    assert es < bound_s


@pytest.fixture(scope="module")
def coarse_ref():
    case = make_config("c2c")
    steps = 1000
    say(f"oracle: coarse aneurysm {case.nx}x{case.ny}x{case.nz} ({case.n_fluid} fluid cells), {steps} steps")
    o, f, om, ref = _oracle_run(case, steps)
    return case, steps, ref


@pytest.mark.parametrize("storage,shift_mode,rounding,bound_u,bound_s", [
    ("fp32", 0, "stochastic", 1e-5, 1e-4), ("fp32", 1, "stochastic", 1e-5, 1e-4),
    ("fp16", 0, "stochastic", FP16_U, 5 * FP16_U), ("bf16", 0, "stochastic", BF16_U, 5 * BF16_U),
    ("fp16", 1, "stochastic", 5 * FP16_U, 5 * 5 * FP16_U), ("bf16", 1, "stochastic", 5 * BF16_U, 5 * 5 * BF16_U),
    ("fp16", 0, "conserve", 1e-3, 5e-3), ("fp16", 1, "conserve", 1e-3, 5e-3),
    ("bf16", 0, "conserve", 5e-3, 2e-2), ("bf16", 1, "conserve", 1e-2, 5e-2),
    ("fp16", 0, "nearest", 1.2e-3, 1e-2), ("fp16", 1, "nearest", 5e-3, 1e-2),
    ("bf16", 0, "nearest", 2e-2, 1e-1), ("bf16", 1, "nearest", 5e-2, 1e-1),
])
def test_coarse_aneurysm_every_form(coarse_ref, storage, shift_mode, rounding, bound_u, bound_s):
    """Every storage form, shift mode and 16-bit rounding on the 2x-coarsened
    copy of the large aneurysm (256x160x160, block-mean porosity) against the
    FP64 oracle at the same resolution, 1000 steps.  FP32 is bounded by
    max-relative error, the reduced forms by relative L2 (bounds as for the
    192x128x128 aneurysm).  Shift mode 1 (deviation from w_i rather than
    w_i phi) leaves an O(1 - phi) offset in the sac that the reduced forms
    round with it; its stochastic-rounding bounds are 5x those of shift mode 0.
    The deterministic roundings are bounded by their measured regime
    (conserving FP16 5.1e-4, BF16 1.9e-3; nearest 1.06e-3, 9.7e-3)."""
    case, steps, ref = coarse_ref
    say(f"gpu: coarse aneurysm {storage} shift_mode={shift_mode} rounding={rounding}")
    s = Solver.from_case(case, storage=storage, shift_mode=shift_mode, rounding=rounding)
    s.step(steps)
    g = _gpu_fields(s)
    mu, ms = max_rel(g["u"], ref["u"]), max_rel(g["shear"], ref["shear"])
    lu, ls = rel_l2(g["u"], ref["u"]), rel_l2(g["shear"], ref["shear"])
    say(f"  {storage}/{shift_mode}: u max-rel {mu:.3e} rel-L2 {lu:.3e}; shear max-rel {ms:.3e} rel-L2 {ls:.3e}")
    if storage == "fp32":
        assert mu < bound_u and ms < bound_s
    else:
        assert lu < bound_u and ls < bound_s


def test_state_roundtrip_and_reset():
    case = tiny_case("open", seed=4)
    s = Solver.from_case(case)
    s.step(7)
    f, om = s.get_state()
    s.set_state(f, om)
    f2, om2 = s.get_state()
    assert np.array_equal(f, f2) and np.array_equal(om, om2)
    assert s.t == 7
    s.reset()
    assert s.t == 0
    o = oracle.Oracle(case)
    f0, om0 = o.init()
    g0, gom0 = s.get_state()
    assert np.abs(g0 - f0).max() < 1e-7
    assert np.abs(gom0 - om0).max() < 1e-7


@pytest.mark.parametrize("kind", ["open", "open_extrap", "periodic3", "open_q27", "open_extrap_q27"])
@pytest.mark.parametrize("t_split", [7, 8])
def test_restored_state_continues_trajectory(kind, t_split):
    """get_state / set_state at an odd and an even time (the two slot layouts of
    the in-place streaming) continue the uninterrupted run bit for bit."""
    case = _tiny_any(kind, 5)
    a = Solver.from_case(case)
    a.step(t_split + 5)
    fa, oa = a.get_state()
    b = Solver.from_case(case)
    b.step(t_split)
    f, om = b.get_state()
    b.reset()
    b.step(t_split)
    b.set_state(np.zeros_like(f), np.zeros_like(om))
    b.set_state(f, om)
    b.step(5)
    fb, ob = b.get_state()
    assert np.array_equal(fa, fb) and np.array_equal(oa, ob)


def test_long_calls_match_single_steps():
    """Long lbm_step calls give exactly what one-step calls give (the step
    kernels take the time from a device counter), with other work (moments,
    diagnostics) between the calls, from odd and even start times and across
    a stability check (step 999)."""
    case = tiny_case("open", seed=6)
    a = Solver.from_case(case)   # one step per call
    b = Solver.from_case(case)   # long calls

    def single(n):
        for _ in range(n):
            a.step(1)

    plan = [1, 300, 129, 64, 570, 180]   # odd and even starts, a call across step 999
    for n in plan:
        single(n)
        b.step(n)
        assert a.t == b.t
        fa, oa = a.get_state()
        fb, ob = b.get_state()
        assert np.array_equal(fa, fb) and np.array_equal(oa, ob), f"state differs after t={b.t}"
        # other work between the calls
        a.moments(sigma=True)
        db = b.diagnostics()
        assert db["nonfinite"] == 0


def test_diagnostics_match_oracle():
    case = tiny_case("periodic", seed=2)
    s = Solver.from_case(case)
    s.step(30)
    d = s.diagnostics()
    o = oracle.Oracle(case)
    f, om = o.init()
    o.run(f, om, 0, 30)
    m = o.moments(f, om, 30)
    c, _ = oracle.lattice()
    ke = 0.5 * m["rho"] * (m["u"] ** 2).sum(0)
    sac = case.sac.reshape(-1)[o.cells()]
    assert abs(d["mass"] - f.sum()) < 1e-5
    assert np.abs(np.array([d["mom_x"], d["mom_y"], d["mom_z"]]) - (f.T @ c).sum(0)).max() < 1e-6
    assert abs(d["ke"] - ke.sum()) < 1e-6 * max(ke.sum(), 1e-12) + 1e-12
    assert abs(d["ke_region"] - ke[sac].sum()) < 1e-6 * max(ke.sum(), 1e-12) + 1e-12
    assert abs(d["max_u"] - np.sqrt((m["u"] ** 2).sum(0)).max()) < 1e-6
    assert abs(d["min_omega"] - m["omega"].min()) < 1e-6 and abs(d["max_omega"] - m["omega"].max()) < 1e-6
    assert d["nonfinite"] == 0 and d["t"] == 30
    # region-mean WSS magnitude over the region's wall cells (wall link, m != 0)
    nb = o.neighbours()
    w = np.array([12.0] + [2.0] * 6 + [1.0] * 12)
    mvec = np.einsum("ix,ia->ax", (nb == -1) * w[:, None], c.astype(np.float64))
    on = sac & (np.abs(mvec).sum(0) > 0)
    wss = np.sqrt((m["tau"] ** 2).sum(0))[on].mean()
    say(f"  wss_region gpu {d['wss_region']:.6e} oracle {wss:.6e}")
    assert abs(d["wss_region"] - wss) < 1e-5 * wss


def test_porosity_update_resets():
    case = tiny_case("periodic", seed=5)
    s = Solver.from_case(case)
    s.step(5)
    phi2 = np.where(case.solid == 0, np.clip(case.phi * 0.9, 0.5, 1.0), 0.0).astype(np.float32)
    s.set_porosity(phi2)
    assert s.t == 0
    case2 = case.with_(phi=phi2)
    o = oracle.Oracle(case2)
    f, om = o.init()
    o.run(f, om, 0, 10)
    s.step(10)
    g, _ = s.get_state()
    assert np.abs(g - f).max() < 2e-6


@pytest.mark.parametrize("kind", ["bulk", "bulk_q27"])
def test_wave_records_follow_porosity_updates(kind):
    """The per-wave records of the D3Q19 step (which waves may skip the link
    words) are rebuilt on every porosity upload: uniform middles (plain
    waves), then random porosity everywhere (no plain wave), then uniform
    again, each followed by 12 steps against the oracle (D3Q27, which keeps
    no records, as a control)."""
    case = _tiny_any(kind, 2)
    s = Solver.from_case(case)
    rng = np.random.default_rng(17)
    fluid = case.solid == 0
    x = np.arange(case.nx)[None, None, :]
    face = (x == 0) | (x == case.nx - 1)
    noisy = np.where(fluid, np.where(face, 1.0, rng.uniform(0.6, 1.0, case.solid.shape)), 0.0).astype(np.float32)
    for name, phi in (("uniform", case.phi), ("random", noisy), ("uniform again", case.phi)):
        say(f"wave records: {case.name} porosity {name}")
        s.set_porosity(np.ascontiguousarray(phi, dtype=np.float32))
        s.step(12)
        o = oracle.Oracle(case.with_(phi=phi))
        f, om = o.init()
        o.run(f, om, 0, 12)
        g, _ = s.get_state()
        known = np.isfinite(g)
        assert np.abs(g[known] - f[known]).max() < 2e-6


def test_instability_is_reported():
    """A non-finite population injected through lbm_set_state is caught at the
    next stability check (every 1000th step index) with LBM_E_UNSTABLE."""
    case = tiny_case("periodic", seed=6)
    s = Solver.from_case(case)
    f, om = s.get_state()
    f[3, 5] = np.nan
    s.set_state(f, om)
    with pytest.raises(lbm.LBMError) as e:
        s.step(1000)
    assert e.value.status == lbm.LBM_E_UNSTABLE
    assert "non-finite" in str(e.value)
