"""Writes the FP64 oracle's density drift on the volume-averaged coil twin of
the 384x256x256 coil pair (porosity 1 - box filter of width 8 of the wire,
floored at 0.2), which the GPU test of that drift compares with.

In the few windows almost filled by wire the porosity sits at the floor, and
there the porosity-jump and drag terms drain the density slowly until the run
diverges (near step 7750).  Every 500 steps up to step 7000 the script stores
the minimum density over the fluid cells, the cell where it sits (oracle
fluid-cell order, ascending box index), the fluid mass sum over the cells of
phi rho (the densities as the step's moments give them, open-face fill
included) and the largest speed.  Every number comes from the FP64 oracle
only.

Run from the repository root: python tests/golden/make_coil_drift.py
(about 20 minutes on 8 cores).  Output: coil_drift.json.
"""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import make_config  # noqa: E402

STEPS = 7000
EVERY = 500
OUT = os.path.dirname(os.path.abspath(__file__))


def main():
    case = make_config("c3")[1]
    o = oracle.Oracle(case)
    phi = case.phi.reshape(-1)[o.cells()].astype(np.float64)
    f, om = o.init()
    t0 = time.time()
    rows = []
    done = 0
    while done < STEPS:
        o.run(f, om, done, EVERY)
        done += EVERY
        m = o.moments(f, om, done)
        k = int(np.argmin(m["rho"]))
        rows.append(dict(step=done, min_rho=float(m["rho"][k]), argmin=k, mass=float((phi * m["rho"]).sum()),
                         max_u=float(np.sqrt((m["u"] ** 2).sum(0)).max())))
        print(f"[coil drift] {done} / {STEPS} steps, {time.time() - t0:.0f} s: {rows[-1]}", flush=True)
    meta = dict(case="c3 averaged twin", n_fluid=int(o.nf), threads=oracle.threads(),
                seconds=round(time.time() - t0, 1), every=EVERY, rows=rows)
    with open(os.path.join(OUT, "coil_drift.json"), "w") as fh:
        json.dump(meta, fh, indent=1)


if __name__ == "__main__":
    main()
