"""The storage forms over the configured run length: the 192x128x128 aneurysm
and the 2x-coarsened copy of the 512x320x320 aneurysm, 20 000 steps from rest
(five periods of the pulsatile inflow), against the FP64 oracle's fields at
step 20 000 (stored by tests/golden/make_longrun.py, which calls only the
oracle).

Bounds: FP32 storage, velocity max-relative error 1e-5 (the FP32 target) and
shear rate 1e-4; FP16 with the default stochastic rounding, velocity relative
L2 1e-3 (the FP16 target); BF16 (3 fewer significand bits) 8e-3.  Shear-rate
relative L2 of the 16-bit forms: 5x the velocity bound (the stress carries the
last step's rounding noise)."""

import json
import os

import numpy as np
import pytest

from paper_2402_10809_amd import Solver
from synth import make_config

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
STEPS = 20000


def say(msg):
    print(msg, flush=True)


def _ref(key):
    with open(os.path.join(GOLDEN, f"longrun_{key}.json")) as fh:
        meta = json.load(fh)
    assert meta["steps"] == STEPS
    u = np.load(os.path.join(GOLDEN, f"longrun_{key}_u.npy")).astype(np.float64)
    sh = np.load(os.path.join(GOLDEN, f"longrun_{key}_shear.npy")).astype(np.float64)
    return u, sh


@pytest.mark.parametrize("key", ["c1", "c2c"])
@pytest.mark.parametrize("storage,bound_u,bound_s", [("fp32", 1e-5, 1e-4), ("fp16", 1e-3, 5e-3),
                                                      ("bf16", 8e-3, 4e-2)])
def test_storage_forms_over_20000_steps(key, storage, bound_u, bound_s):
    case = make_config(key)
    uref, sref = _ref(key)
    say(f"long run: {key} {case.nx}x{case.ny}x{case.nz}, {storage} (default rounding), {STEPS} steps")
    s = Solver.from_case(case, storage=storage)
    s.step(STEPS)
    m = s.moments()
    idx = s.fluid_index()
    assert idx.size == uref.shape[1]
    u = m["u"].cpu().numpy().reshape(3, -1)[:, idx].astype(np.float64)
    sh = m["shear"].cpu().numpy().reshape(-1)[idx].astype(np.float64)
    du = np.sqrt(((u - uref) ** 2).sum(0))
    u_max = np.sqrt((uref ** 2).sum(0)).max()
    mr_u = float(du.max() / u_max)
    l2_u = float(np.sqrt((du ** 2).sum() / (uref ** 2).sum()))
    mr_s = float(np.abs(sh - sref).max() / np.abs(sref).max())
    l2_s = float(np.linalg.norm(sh - sref) / np.linalg.norm(sref))
    say(f"  u max-rel {mr_u:.3e} rel-L2 {l2_u:.3e}; shear max-rel {mr_s:.3e} rel-L2 {l2_s:.3e}")
    if storage == "fp32":
        assert mr_u < bound_u and mr_s < bound_s
    else:
        assert l2_u < bound_u and l2_s < bound_s


@pytest.fixture(scope="module")
def full_fp32():
    case = make_config("c2")
    say(f"full resolution: {case.nx}x{case.ny}x{case.nz}, {case.n_fluid} fluid cells, fp32, {STEPS} steps")
    s = Solver.from_case(case, storage="fp32")
    s.step(STEPS)
    m = s.moments()
    idx = s.fluid_index()
    u = m["u"].cpu().numpy().reshape(3, -1)[:, idx].astype(np.float64)
    sh = m["shear"].cpu().numpy().reshape(-1)[idx].astype(np.float64)
    s.close()
    return case, u, sh


@pytest.mark.parametrize("storage,bound_u,bound_s", [("fp16", 1e-3, 5e-3), ("bf16", 8e-3, 4e-2)])
def test_full_resolution_16bit_against_fp32(full_fp32, storage, bound_u, bound_s):
    case, uref, sref = full_fp32
    # the pulsatile inflow (peak 0.05 at the axis) has developed: the reference is a flow, not the rest state
    assert np.sqrt((uref ** 2).sum(0)).max() > 0.02
    say(f"full resolution: {storage} (default rounding) against fp32, {STEPS} steps")
    s = Solver.from_case(case, storage=storage)
    s.step(STEPS)
    m = s.moments()
    idx = s.fluid_index()
    assert idx.size == uref.shape[1]
    u = m["u"].cpu().numpy().reshape(3, -1)[:, idx].astype(np.float64)
    sh = m["shear"].cpu().numpy().reshape(-1)[idx].astype(np.float64)
    s.close()
    du = np.sqrt(((u - uref) ** 2).sum(0))
    l2_u = float(np.sqrt((du ** 2).sum() / (uref ** 2).sum()))
    l2_s = float(np.linalg.norm(sh - sref) / np.linalg.norm(sref))
    say(f"  u rel-L2 {l2_u:.3e}; shear rel-L2 {l2_s:.3e}")
    assert l2_u < bound_u and l2_s < bound_s
