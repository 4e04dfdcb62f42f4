"""Writes the stored FP64-oracle fields of the long-run storage-precision check:
the 192x128x128 aneurysm (tube radius 12, sac radius 20, GRF sac porosity with
correlation length 4) and the 2x-coarsened copy of the 512x320x320 aneurysm
(256x160x160), each run 20 000 steps from rest (five periods of the pulsatile
inflow) with the configured Zou-He inflow and constant-density outflow.
Every number comes from the FP64 oracle only.

Per case it stores the velocity u (3, n_fluid) and the shear rate (n_fluid) of
the state at step 20 000, in the oracle's fluid-cell order (ascending box
index), as float32 (their rounding, 6e-8 of each value, is far below the
tolerances they are compared at).

Run from the repository root: python tests/golden/make_longrun.py [c1] [c2c]
(a few minutes for c1, about half an hour for c2c on 8 cores).
Outputs: longrun_<case>_u.npy, longrun_<case>_shear.npy, longrun_<case>.json.
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

STEPS = 20000
OUT = os.path.dirname(os.path.abspath(__file__))


def main():
    keys = sys.argv[1:] or ["c1", "c2c"]
    for key in keys:
        case = make_config(key)
        o = oracle.Oracle(case)
        f, om = o.init()
        t0 = time.time()
        done = 0
        while done < STEPS:
            n = min(1000, STEPS - done)
            o.run(f, om, done, n)
            done += n
            print(f"[{key}] {done} / {STEPS} steps, {time.time() - t0:.0f} s", flush=True)
        m = o.moments(f, om, STEPS)
        np.save(os.path.join(OUT, f"longrun_{key}_u.npy"), m["u"].astype(np.float32))
        np.save(os.path.join(OUT, f"longrun_{key}_shear.npy"), m["shear"].astype(np.float32))
        meta = dict(case=key, steps=STEPS, n_fluid=int(o.nf), threads=oracle.threads(),
                    seconds=round(time.time() - t0, 1),
                    max_u=float(np.sqrt((m["u"] ** 2).sum(0)).max()), max_shear=float(m["shear"].max()),
                    mass=float(f.sum()))
        with open(os.path.join(OUT, f"longrun_{key}.json"), "w") as fh:
            json.dump(meta, fh, indent=1)
        print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
