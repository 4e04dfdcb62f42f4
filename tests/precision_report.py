"""Accuracy report of every storage form against the FP64 oracle, and the
resolved-versus-averaged coil comparison.  Not a test: it prints tables.

Part A, for the 192x128x128 aneurysm and the 2x-coarsened copy of the
512x320x320 aneurysm: every storage form (FP32, FP16, BF16), shift mode and
16-bit rounding (stochastic "s", the default; conserving "c"; to nearest "n"),
max-relative and relative-L2 errors of u and of the shear rate against the
oracle after 1000 steps and at the final step (20 000 by default, taken from
the oracle fields stored in tests/golden by make_longrun.py).

Part B, the 384x256x256 coil pair: the fully resolved coil (wire voxels solid)
and its volume-averaged twin (porosity 1 - box filter of width 8 of the wire
indicator), each run on the GPU.  Reported: the sac-mean speed of both runs
and the relative L2 difference, over the sac, between the box-filtered
resolved velocity (zero in the wire, hence a superficial average) and phi
times the VANSE velocity (the VANSE u is the intrinsic average).  The paper
compares these flows only qualitatively, so no bound is applied.  The pair is
compared after --coil-steps (5000) steps: in the averaged field about 1 % of
the width-8 windows are almost filled by wire (porosity at the 0.2 floor), and
there the porosity-jump and drag terms drain the density slowly (the FP64
oracle follows the same drift to five digits) until the run diverges near
step 7750.

Run from the repository root on a GPU host:
    python tests/precision_report.py [--steps 20000] [--coil-steps 5000] [--part A|B|AB]
"""

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2402_10809_amd import Solver  # noqa: E402
from synth import make_config  # noqa: E402

# (storage, shift mode, 16-bit rounding)
FORMS = [("fp32", 0, "stochastic"), ("fp32", 1, "stochastic")] + [
    (st, sh, r) for st in ("fp16", "bf16") for r in ("stochastic", "conserve", "nearest") for sh in (0, 1)]
GOLDEN = os.path.join(ROOT, "tests", "golden")


def say(msg):
    print(msg, flush=True)


def max_rel(a, ref):
    if a.ndim == 2:
        return float(np.sqrt(((a - ref) ** 2).sum(0)).max() / np.sqrt((ref ** 2).sum(0)).max())
    return float(np.abs(a - ref).max() / np.abs(ref).max())


def rel_l2(a, ref):
    return float(np.sqrt(((a - ref) ** 2).sum()) / np.sqrt((ref ** 2).sum()))


def gpu_fields(s):
    m = s.moments()
    idx = s.fluid_index()
    u = m["u"].cpu().numpy().reshape(3, -1)[:, idx]
    g = m["shear"].cpu().numpy().reshape(-1)[idx]
    return u, g


def part_a(steps_final):
    checkpoints = [1000, steps_final]
    for key in ("c1", "c2c"):
        case = make_config(key)
        say(f"\n== {key}: {case.nx}x{case.ny}x{case.nz}, {case.n_fluid} fluid cells; oracle on "
            f"{oracle.threads()} threads")
        o = oracle.Oracle(case)
        f, om = o.init()
        refs, t, t0 = {}, 0, time.time()
        for tc in checkpoints:
            stored = os.path.join(GOLDEN, f"longrun_{key}_u.npy")
            if tc == 20000 and os.path.exists(stored):
                refs[tc] = (np.load(stored).astype(np.float64),
                            np.load(os.path.join(GOLDEN, f"longrun_{key}_shear.npy")).astype(np.float64))
                say(f"   oracle at step {tc}: stored fields")
                continue
            while t < tc:
                n = min(2000, tc - t)
                o.run(f, om, t, n)
                t += n
                say(f"   oracle step {t} ({time.time() - t0:.0f} s)")
            m = o.moments(f, om, t)
            refs[tc] = (m["u"], m["shear"])
            say(f"   oracle at step {tc} ({time.time() - t0:.0f} s)")
        say(f"   {'form':10s} {'step':>6s} {'u max-rel':>10s} {'u rel-L2':>10s} {'g max-rel':>10s} {'g rel-L2':>10s}")
        for storage, shift, rounding in FORMS:
            s = Solver.from_case(case, storage=storage, shift_mode=shift, rounding=rounding)
            label = f"{storage}/{shift}" + ("" if storage == "fp32" else f"/{rounding[0]}")
            t = 0
            for tc in checkpoints:
                s.step(tc - t)
                t = tc
                u, g = gpu_fields(s)
                ur, gr = refs[tc]
                say(f"   {label:10s} {tc:6d} {max_rel(u, ur):10.3e} {rel_l2(u, ur):10.3e} "
                    f"{max_rel(g, gr):10.3e} {rel_l2(g, gr):10.3e}")
            s.close()


def part_b(steps):
    from scipy import ndimage

    t0 = time.time()
    res, avg = make_config("c3")
    say(f"\n== coil pair {res.nx}x{res.ny}x{res.nz}: packing {res.extra.get('packing'):.3f}, "
        f"resolved {res.n_fluid} / averaged {avg.n_fluid} fluid cells ({time.time() - t0:.0f} s), {steps} steps")
    out = {}
    for case in (res, avg):
        s = Solver.from_case(case)
        s.step(steps)
        m = s.moments()
        out[case.name] = m["u"].cpu().numpy().reshape(3, case.nz, case.ny, case.nx).astype(np.float64)
        d = s.diagnostics()
        say(f"   {case.name}: max |u| {d['max_u']:.4e}, omega [{d['min_omega']:.4f}, {d['max_omega']:.4f}], "
            f"nonfinite {d['nonfinite']:.0f}")
        s.close()
    sac = avg.sac
    ur, ua = out[res.name], out[avg.name]
    speed_r = np.sqrt((ur ** 2).sum(0))
    speed_a = np.sqrt((ua ** 2).sum(0))
    say(f"   sac-mean |u|: resolved (fluid voxels of the sac) {speed_r[res.sac].mean():.4e}, "
        f"resolved (all sac voxels, 0 in the wire) {speed_r[sac].mean():.4e}, VANSE {speed_a[sac].mean():.4e}")
    filt = np.stack([ndimage.uniform_filter(ur[k], size=8, mode="constant") for k in range(3)])
    sup = ua * avg.phi[None].astype(np.float64)
    diff = np.sqrt(((filt - sup) ** 2).sum(0))[sac]
    ref = np.sqrt((filt ** 2).sum(0))[sac]
    say(f"   rel-L2 over the sac of box8(u_resolved) vs phi u_VANSE: {np.linalg.norm(diff) / np.linalg.norm(ref):.3e}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--coil-steps", type=int, default=5000)
    ap.add_argument("--part", default="AB")
    a = ap.parse_args()
    if "A" in a.part:
        part_a(a.steps)
    if "B" in a.part:
        part_b(a.coil_steps)


if __name__ == "__main__":
    main()
