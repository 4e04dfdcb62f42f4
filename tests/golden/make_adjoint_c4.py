"""Writes the stored expected values of the full-size adjoint check (the
128x96x96 aneurysm: tube radius 8, sac radius 14, GRF sac porosity with
correlation length 4; 4000 steps; objective averaged over steps [3000, 4000):
the sac kinetic energy, or with --kind wss the WSS magnitude over the sac's
wall cells).  Every number comes from the FP64 oracle only:

* J, and its central finite differences at 16 seeded sac voxels (eps = 1e-4
  for the kinetic energy, 1e-5 for the WSS, whose dependence on a wall
  voxel's porosity bends more sharply);
* the exact discrete derivative at the same voxels (dual numbers);
* the checkpointed reverse sweep (checkpoints every 64 steps) over every sac
  voxel.

Run from the repository root: python tests/golden/make_adjoint_c4.py [--kind wss]
(about an hour on 8 cores).  Finished stages are kept in
adjoint_c4[_wss].partial.json (not tracked), so an interrupted run resumes.
Outputs: adjoint_c4[_wss].json and adjoint_c4[_wss]_reverse_sac.npy.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import fd_voxels, make_config  # noqa: E402

T, TB, TE, CKPT = 4000, 3000, 4000, 64
OUT = os.path.dirname(os.path.abspath(__file__))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--kind", choices=["ke", "wss"], default="ke")
    kind = ap.parse_args().kind
    EPS = 1e-4 if kind == "ke" else 1e-5
    stem = "adjoint_c4" if kind == "ke" else "adjoint_c4_wss"
    t0 = time.time()
    part_path = os.path.join(OUT, stem + ".partial.json")
    part = {}
    if os.path.exists(part_path):
        with open(part_path) as fh:
            part = json.load(fh)

    def save():
        with open(part_path, "w") as fh:
            json.dump(part, fh)

    case = make_config("c4")
    vox = fd_voxels(case, 16, seed=16)
    o = oracle.Oracle(case)
    if "J" not in part:
        part["J"] = o.objective(T, TB, TE, kind)
        save()
    J = part["J"]
    print(f"J = {J:.15e} ({time.time() - t0:.0f} s)", flush=True)
    phi0 = case.phi.reshape(-1).astype(np.float64)
    fd = part.setdefault("fd", [])
    for k in range(len(fd), len(vox)):
        v = vox[k]
        js = []
        for sgn in (1.0, -1.0):
            ph = phi0.copy()
            ph[v] += sgn * EPS
            o.set_phi(ph.reshape(case.phi.shape))
            js.append(o.objective(T, TB, TE, kind))
        fd.append((js[0] - js[1]) / (2 * EPS))
        save()
        print(f"fd voxel {k} ({v}): {fd[-1]:.10e} ({time.time() - t0:.0f} s)", flush=True)
    o.set_phi(phi0.reshape(case.phi.shape))
    if "dual" not in part:
        Jd, gd = o.grad_dual(T, TB, TE, vox, kind)
        part["J_dual"], part["dual"] = float(Jd), [float(x) for x in np.asarray(gd)]
        save()
    print(f"dual done ({time.time() - t0:.0f} s)", flush=True)
    Jr, gbox = o.grad_reverse(T, TB, TE, CKPT, kind)
    print(f"reverse done ({time.time() - t0:.0f} s)", flush=True)
    sac = np.flatnonzero(case.sac.reshape(-1))
    gflat = np.asarray(gbox).reshape(-1)
    np.save(os.path.join(OUT, stem + "_reverse_sac.npy"), gflat[sac].astype(np.float64))
    rec = {
        "case": "c4", "objective": kind, "T": T, "t_begin": TB, "t_end": TE, "ckpt": CKPT, "eps": EPS,
        "fd_seed": 16, "voxels": [int(v) for v in vox],
        "J": J, "J_dual": part["J_dual"], "J_reverse": float(Jr),
        "grad_fd": fd, "grad_dual": part["dual"],
        "grad_reverse_at_voxels": [float(gflat[v]) for v in vox],
        "sac_cells": int(sac.size),
    }
    with open(os.path.join(OUT, stem + ".json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    os.remove(part_path)
    print(f"written ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
