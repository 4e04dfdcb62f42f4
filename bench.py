"""Throughput of the fused D3Q19 VANSE Carreau-Yasuda step on one GPU.

Prints ONE JSON line.  The workload is the 512x320x320 tube-and-sac aneurysm
(tube radius 32, sac radius 56, GRF sac porosity with correlation length 10,
2 360 212 fluid cells): fluid-cell MLUPS with FP32 population storage is the
headline ``value``; FP16 and BF16 storage and the adjoint (porosity gradient of
the sac kinetic energy: forward pass, checkpointed recompute and reverse sweep,
timed as one call, with checkpoints every 20 steps, and as one segment whose
record of the whole trajectory stays in HBM) are reported on the same geometry
under ``forms``.  A step is one time step of the
whole hot path: pull-streaming with bounce-back and open-face fill, porosity-
weighted moments, drag-corrected velocity, equilibrium and Pi, Carreau-Yasuda
relaxation rate, collision and store (plus the FP64 stability reduction every
1000th step).

Timing: inputs resident in device memory; the flow is first spun up from rest
for ``--spinup`` steps (2000: the pulsatile flow is developed, so the timed
steps see its working state rather than the near-rest start), then
``--warmup`` untimed steps, then exactly ``--steps`` steps between HIP events
on the solver's stream, bracketed by device synchronisation.

Beyond the cache: the aneurysm's FP32 working set (about 217 MB) fits the
256 MB Infinity Cache, so its rate is not an HBM figure; the ``*_hbm`` forms
time the same step on the 512x320x320 all-fluid periodic box (52.4 M cells,
porosity random everywhere), whose state far exceeds the cache.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak
# algorithmic bytes per fluid-cell update: populations read + written, porosity,
# relaxation rate read + written
B_ALG = {"fp32": 164, "fp16": 88, "bf16": 88,
         # D3Q27: 27 populations read + written
         "fp32_q27": 27 * 8 + 12, "fp16_q27": 27 * 4 + 12, "bf16_q27": 27 * 4 + 12}
# The adjoint per reverse cell-step, as the scope of the method counts it:
# the reverse step (pulled values 76, adjoint populations gathered 76 and
# written 76, omega_prev 4, porosity 4, neighbour rho 4, omega adjoint r/w 8,
# porosity adjoint r/w 8 = 256) and the segment recompute (a forward step 164 +
# the rho record 4 = 168); the initial forward pass is implementation overhead.
B_ALG_ADJ = 256 + 168
# what this implementation moves per cell and time step: forward pass 164,
# recompute with the record written (164 + 19 pulled values + omega_prev + rho
# = 248), reverse step (record 80, adjoint populations 152, porosity 4,
# neighbour rho 4, omega adjoint 8, FP64 porosity adjoint 16 = 264)
B_IMPL_ADJ = 164 + 248 + 264
# with one segment (ckpt_every = T: the whole record resident in HBM) the
# forward pass writes the record and nothing is recomputed: 248 + 264
B_IMPL_ADJ_1SEG = 248 + 264


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# the sources that the D3Q19 step kernels and their launches are built from
# (the adjoint's and the D3Q27 kernels' own files are not among them)
STEP_SOURCES = ("fp64math.hpp", "k19_bf16.hip", "k19_f16.hip", "k19_f32.hip", "kmisc.hip", "lattice.hpp",
                "launch19.hpp", "layout.hpp", "lbm.hip", "runtime.hpp", "step.hpp")


def source_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2402_10809_amd", "csrc")
    for n in STEP_SOURCES:
        with open(os.path.join(d, n), "rb") as fh:
            h.update(n.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(key: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        t = json.load(fh)
    if t.get("source_hash") != source_hash():
        return None
    e = t.get("kernels", {}).get(key)
    return None if e is None else e.get("bytes_per_launch")


def time_steps(torch, solver, steps: int, warmup: int, spinup: int = 0):
    solver.step(spinup + warmup)
    torch.cuda.synchronize()
    stream = solver.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    solver.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms per step


def probes(torch, nbytes=4 << 30, reps=10, kinds=("copy", "copy_nt", "read", "write")):
    """Achievable bandwidth on this machine: the plain 16-byte copy, a copy with
    four vectors in flight per work-item and non-temporal accesses, a read-only
    and a write-only stream, each over nbytes per buffer (4 GiB by default;
    GB/s of bytes moved)."""
    from paper_2402_10809_amd import lbm

    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    st = torch.cuda.current_stream()
    out = {}
    for kind in kinds:
        dst = b.data_ptr()
        lbm.lbm_bandwidth_probe(kind, dst, a.data_ptr(), nbytes, st.cuda_stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            lbm.lbm_bandwidth_probe(kind, dst, a.data_ptr(), nbytes, st.cuda_stream)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        moved = 2 * nbytes if kind.startswith("copy") else nbytes
        out[kind] = round(moved / (ms * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def time_adjoint(torch, case, T: int, ckpt: int, fp64: bool = False):
    """Wall time of one lbm_adjoint call (forward pass with checkpoints,
    segment recompute and reverse sweep) over T steps, window [T/2, T)."""
    # the call starts from rest by definition (the forward pass is part of it)
    from paper_2402_10809_amd import Solver

    s = Solver.from_case(case, adjoint_T=T, ckpt=ckpt)
    tb, te = T // 2, T
    s.adjoint(tb, te, T, ckpt, fp64=fp64)  # warm-up call
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, g = s.adjoint(tb, te, T, ckpt, fp64=fp64)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ok = bool(np.isfinite(J)) and bool(torch.isfinite(g).all().item())
    # the same call without a gradient output: the forward pass alone (J, no
    # checkpoints or records), i.e. the initial forward pass that the
    # algorithmic bytes of the adjoint leave out
    s.objective(tb, te, T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Jf = s.objective(tb, te, T)
    torch.cuda.synchronize()
    dtf = time.perf_counter() - t0
    s.close()
    del s, g
    torch.cuda.empty_cache()
    return dt, dtf, ok, Jf == J


def _oracle_rate(case, budget_s: float, max_steps: int = 400):
    """Steps of the oracle within about budget_s (after one untimed step):
    (MLUPS, steps, seconds, fluid cells)."""
    import oracle

    o = oracle.Oracle(case)
    f, om = o.init()
    t0 = time.perf_counter()
    o.run(f, om, 0, 1)
    one = time.perf_counter() - t0
    n = max(1, min(max_steps, int(budget_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    o.run(f, om, 1, n)
    dt = time.perf_counter() - t0
    return o.nf * n / dt / 1e6, n, dt, o.nf


def cpu_baseline(case, budget_s: float):
    """The FP64 oracle (as it stands) on a bounded number of steps of the same
    geometry, on this host's cores, and on one thread."""
    import oracle

    v, n, dt, nf = _oracle_rate(case, budget_s)
    cores = oracle.threads()
    prev = oracle.set_threads(1)
    try:
        v1, n1, dt1, _ = _oracle_rate(case, budget_s / 3)
    finally:
        oracle.set_threads(prev)
    return dict(value=round(v, 3), unit="MLUPS", cores=cores, kind="oracle",
                sample=f"{n} steps (after 1 untimed) of the full {case.nx}x{case.ny}x{case.nz} geometry, "
                       f"{nf} fluid cells, FP64, {dt:.1f} s",
                single_thread={"value": round(v1, 3), "sample": f"{n1} steps, {dt1:.1f} s"})


def cpu_cases(budget_s: float):
    """The oracle on the other workloads (bounded samples, all cores and one
    thread), and its reverse sweep on the gradient workload."""
    import oracle
    from synth import make_config

    out = {}
    cores = oracle.threads()
    for key, steps in (("c0", 2000), ("c1", 1000), ("c2c", 400)):
        case = make_config(key)
        v, n, dt, nf = _oracle_rate(case, budget_s, steps)
        prev = oracle.set_threads(1)
        try:
            v1, n1, dt1, _ = _oracle_rate(case, budget_s / 3, steps)
        finally:
            oracle.set_threads(prev)
        out[key] = {"fluid_cells": nf, "mlups": round(v, 3), "steps": n, "seconds": round(dt, 2),
                    "mlups_1thread": round(v1, 3), "steps_1thread": n1}
        log(f"[bench] oracle {key}: {v:.2f} MLUPS on {cores} threads ({n} steps), {v1:.3f} on one ({n1} steps)")
    case = make_config("c4")
    T, ck = 40, 10
    o = oracle.Oracle(case)
    t0 = time.perf_counter()
    o.grad_reverse(T, T // 2, T, ck)
    dt = time.perf_counter() - t0
    out["c4_reverse"] = {"fluid_cells": o.nf, "T": T, "ckpt": ck, "seconds": round(dt, 2),
                         "cell_steps_per_s": round(o.nf * T / dt, 1)}
    log(f"[bench] oracle c4 forward + reverse sweep, T={T}: {dt:.1f} s ({o.nf * T / dt / 1e6:.3f} M cell-steps/s)")
    return out


def parse_form(name: str):
    """A form name: storage (fp32, fp16, bf16), then optional modifiers: q27
    (D3Q27), aniso (the anisotropic medium), conserve / nearest (16-bit
    rounding other than the default stochastic one), hbm (the all-fluid box
    beyond the cache), slab (the x-slices through the sac centre that hold
    1/8 of the fluid cells, periodic in x: one GPU's share of an 8-way
    decomposition with equal fluid counts)."""
    parts = name.split("_")
    storage, mods = parts[0], set(parts[1:])
    if storage not in ("fp32", "fp16", "bf16") or not mods <= {"q27", "aniso", "conserve", "nearest", "hbm", "slab"}:
        raise SystemExit(f"unknown form {name}")
    rounding = "conserve" if "conserve" in mods else ("nearest" if "nearest" in mods else "stochastic")
    return storage, mods, rounding


def bytes_of(name: str) -> int:
    storage, mods, _ = parse_form(name)
    return B_ALG[storage + ("_q27" if "q27" in mods else "")]


def make_solver(name: str, case, hbm_case):
    import copy

    from paper_2402_10809_amd import Solver
    from synth import as_d3q27, with_anisotropic_drag

    storage, mods, rounding = parse_form(name)
    c = hbm_case if "hbm" in mods else case
    if "slab" in mods:
        # one GPU's share of an 8-way x-decomposition with equal fluid counts
        from synth import slab_of
        c = slab_of(c)
    if "q27" in mods:
        c = as_d3q27(copy.copy(c))
    if "aniso" in mods:
        # the Remark's anisotropic drag: Forchheimer on, 6 fixed-point iterations
        c = with_anisotropic_drag(copy.copy(c))
    return Solver.from_case(c, storage=storage, rounding=rounding)


DEFAULT_FORMS = ("fp16,fp16_conserve,fp16_nearest,bf16,fp32_aniso,fp32_q27,fp16_q27,"
                 "fp32_hbm,fp16_hbm,bf16_hbm,fp32_slab,fp16_slab,adjoint,adjoint_fp64,adjoint_1seg,adjoint_aniso")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--spinup", type=int, default=2000,
                    help="steps from rest before the warm-up (the timed flow is the developed one)")
    ap.add_argument("--config", default="c2")
    ap.add_argument("--forms", default=DEFAULT_FORMS)
    ap.add_argument("--adj-T", type=int, default=400)
    ap.add_argument("--adj-ckpt", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-probe", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-cases", dest="cpu_cases", action="store_false",
                    help="skip the oracle's bounded samples of the channel, small and coarse aneurysm workloads "
                         "and of its reverse sweep on the gradient workload")
    ap.add_argument("--only", default=None, help="time one form only (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (got --gpus {args.gpus}): the solver runs on one GPU, and its sharding is a design only.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from synth import make_config

    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    t0 = time.perf_counter()
    case = make_config(args.config)
    log(f"[bench] geometry {case.name} {case.nx}x{case.ny}x{case.nz}: {case.n_fluid} fluid cells "
        f"({time.perf_counter() - t0:.1f} s)")

    forms = ["fp32"] + [f for f in args.forms.split(",") if f]
    if args.only:
        forms = [args.only]
    hbm_case = None
    if any("hbm" in f for f in forms):
        t0 = time.perf_counter()
        hbm_case = make_config("hbm")
        log(f"[bench] geometry {hbm_case.name}: {hbm_case.n_fluid} cells ({time.perf_counter() - t0:.1f} s)")
    results, adjoints, skipped = {}, {}, {}
    for aform in [f for f in forms if f.startswith("adjoint")]:
        forms.remove(aform)
        T, ck = args.adj_T, args.adj_ckpt
        acase = case
        if aform == "adjoint_aniso":
            # the anisotropic medium (Forchheimer on, 6 fixed-point iterations):
            # the same bytes per cell-step, more arithmetic in both directions
            import copy
            from synth import with_anisotropic_drag
            acase = with_anisotropic_drag(copy.copy(case))
        elif aform == "adjoint_1seg":
            # one segment: the forward pass records the whole trajectory
            # (T + 1 records of 84 B per cell, 80 GB at T = 400 on the
            # aneurysm), so no step is recomputed
            ck = T
        elif aform not in ("adjoint", "adjoint_fp64"):
            raise SystemExit(f"unknown adjoint form {aform}")
        log(f"[bench] {aform}: T={T}, checkpoint every {ck}, window [{T // 2}, {T})")
        dt, dtf, ok, same_j = time_adjoint(torch, acase, T, ck, fp64=aform == "adjoint_fp64")
        rate = case.n_fluid * T / dt
        gbs = rate * B_ALG_ADJ / 1e9
        bi = B_IMPL_ADJ_1SEG if ck >= T else B_IMPL_ADJ
        # the gradient part: the whole call less its initial forward pass
        # (reported, not counted in the algorithmic bytes)
        dtg = dt - dtf
        gg = case.n_fluid * T / dtg * B_ALG_ADJ / 1e9
        adjoints[aform] = dict(T=T, ckpt=ck, seconds=round(dt, 4), us_per_step=round(dt / T * 1e6, 1),
                               reverse_cell_steps_per_s=round(rate, 0), bytes_per_update=B_ALG_ADJ,
                               alg_GBps=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4),
                               impl_bytes_per_update=bi, impl_GBps=round(rate * bi / 1e9, 1),
                               forward_us_per_step=round(dtf / T * 1e6, 1),
                               gradient_us_per_step=round(dtg / T * 1e6, 1),
                               gradient_alg_GBps=round(gg, 1), gradient_frac=round(gg / HBM_PEAK_GBS, 4),
                               forward_J_equal=same_j, finite=ok)
        log(f"[bench] {aform}: {dt * 1e3:.1f} ms ({dt / T * 1e6:.0f} us per time step), {rate / 1e9:.2f} G "
            f"reverse cell-steps/s, {gbs:.0f} GB/s algorithmic; forward pass alone {dtf / T * 1e6:.0f} us per "
            f"step, gradient part {dtg / T * 1e6:.0f} us per step ({gg:.0f} GB/s, {gg / HBM_PEAK_GBS:.3f})")
    for form in forms:
        storage, mods, rounding = parse_form(form)
        if "q27" in mods and "hbm" in mods:
            skipped[form] = ("D3Q27 on the all-fluid box exceeds the 32-bit population offsets "
                             "(39.7 M compact cells at most)")
            log(f"[bench] {form}: skipped ({skipped[form]})")
            continue
        s = make_solver(form, case, hbm_case)
        spin = args.spinup
        log(f"[bench] {form}: {spin} spin-up steps, then timing {args.steps} steps after {args.warmup} warmup")
        ms = time_steps(torch, s, args.steps, args.warmup, spin)
        mlups = s.n_fluid / (ms * 1e-3) / 1e6
        gbs = mlups * 1e6 * bytes_of(form) / 1e9
        results[form] = dict(ms_per_step=ms, mlups=mlups, alg_GBps=gbs, frac=gbs / HBM_PEAK_GBS, cells=s.n_fluid)
        log(f"[bench] {form}: {ms * 1e3:.1f} us/step, {mlups:.0f} MLUPS, {gbs:.0f} GB/s algorithmic")
        d = s.diagnostics()
        assert d["nonfinite"] == 0
        s.close()
        del s
        torch.cuda.empty_cache()

    head_form = "fp32" if "fp32" in results else next(iter(results))
    head = results[head_form]
    probe = None if args.no_probe else probes(torch)
    if probe:
        log(f"[bench] bandwidth probes (GB/s): {probe}")
    # the same copies with a footprint equal to the headline form's working set
    # (two buffers of half of it): the achievable rate when that set stays in
    # the Infinity Cache
    h_storage = parse_form(head_form)[0]
    ws_head = results[head_form]["cells"] * (19 * (4 if h_storage == "fp32" else 2) + 16)
    probe_ws = None if args.no_probe else probes(torch, nbytes=(ws_head // 2) & ~255, reps=200,
                                                 kinds=("copy", "copy_nt"))
    if probe_ws:
        log(f"[bench] copy probes at the working-set footprint (GB/s): {probe_ws}")
    cpu = None
    if not args.no_cpu:
        log("[bench] oracle CPU baseline")
        cpu = cpu_baseline(case, args.cpu_budget)
        log(f"[bench] oracle: {cpu['value']} MLUPS on {cpu['cores']} threads, "
            f"{cpu['single_thread']['value']} on one")
        if args.cpu_cases:
            cpu["cases"] = cpu_cases(args.cpu_budget / 3)

    nf = case.n_fluid
    traffic = traffic_for(f"k_step_{head_form}_{args.config}")
    # working set of the headline form: populations, per-cell code, link word,
    # porosity and relaxation rate, in bytes
    ws_mb = round(ws_head / 1e6, 1)
    roof = {"bound": "hbm", "achieved": round(head["alg_GBps"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(head["frac"], 4), "traffic": traffic,
            "working_set_MB": ws_mb, "cache_resident": ws_mb < 256.0}
    hb = results.get(f"{head_form}_hbm")
    if hb:
        roof["beyond_cache"] = {"workload": f"all-fluid periodic box {hbm_case.nx}x{hbm_case.ny}x{hbm_case.nz}",
                                "achieved": round(hb["alg_GBps"], 1), "frac": round(hb["frac"], 4),
                                "traffic": traffic_for(f"k_step_{head_form}_hbm")}
    if probe:
        roof["achievable_GBps"] = max(probe.values())
    if probe_ws:
        roof["achievable_at_working_set_GBps"] = max(probe_ws.values())
    line = {
        "metric": "fluid MLUPS + % HBM peak, D3Q19 VANSE-CY: FP32 vs FP16-store vs adjoint",
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head_form == "fp32" else head_form,
        "data": "synthetic",
        "config": {"workload": f"aneurysm {case.nx}x{case.ny}x{case.nz}, tube R={case.extra.get('R')}, "
                               f"sac R={case.extra.get('Rs')}, GRF porosity ell={case.extra.get('ell')}, "
                               f"Carreau-Yasuda, pulsatile Zou-He inlet, density outlet",
                   "fluid_cells": nf, "storage": head_form, "spinup_steps": args.spinup,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "forms": {k: {"mlups": round(v["mlups"], 1), "alg_GBps": round(v["alg_GBps"], 1),
                      "frac": round(v["frac"], 4), "bytes_per_update": bytes_of(k),
                      "ms_per_step": round(v["ms_per_step"], 5), "cells": v["cells"]} for k, v in results.items()},
        "bandwidth_probes_GBps": probe,
        "copy_probes_at_working_set_GBps": probe_ws,
    }
    line["forms"].update(adjoints)
    if skipped:
        line["skipped"] = skipped
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
