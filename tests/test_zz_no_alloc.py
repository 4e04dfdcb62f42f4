"""lbm_diagnostics_noalloc, the entry point for callers that cannot allocate:
the same diagnostics as lbm_diagnostics with the scratch in the library's
fixed device array, checked through the C ABI against lbm_diagnostics on two
calls in a row (the second on a smaller context), and its size limit."""

import ctypes as ct

import numpy as np
import pytest

from paper_2402_10809_amd import Solver, lbm
from synth import as_d3q27, make_config, periodic_box_case, tiny_case

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def _abi(name, s):
    out = np.full(lbm.NDIAG, np.nan)
    lbm.check(getattr(lbm.lib(), name)(s.ctx, out.ctypes.data_as(ct.c_void_p)))
    return out


def test_noalloc_matches_workspace_diagnostics():
    say("noalloc diagnostics: 512x320x320 aneurysm after 40 steps, then a tiny periodic case after 30")
    big = Solver.from_case(make_config("c2"))
    big.step(40)
    small = Solver.from_case(tiny_case("periodic", seed=2))
    small.step(30)
    a1 = _abi("lbm_diagnostics_noalloc", big)
    a2 = _abi("lbm_diagnostics_noalloc", small)
    r1 = _abi("lbm_diagnostics", big)
    r2 = _abi("lbm_diagnostics", small)
    say(f"  big: mass {a1[0]:.9e} ke {a1[4]:.6e} max|u| {a1[6]:.6e}; small: mass {a2[0]:.9e}")
    assert np.array_equal(a1, r1)
    assert np.array_equal(a2, r2)
    assert a1[10] == 40 and a2[10] == 30
    # the same state again after more steps (the array keeps the previous call's contents)
    small.step(3)
    assert np.array_equal(_abi("lbm_diagnostics_noalloc", small), _abi("lbm_diagnostics", small))
    big.close()
    small.close()


def test_noalloc_d3q27_16bit():
    s = Solver.from_case(as_d3q27(tiny_case("open", seed=1)), storage="fp16")
    s.step(11)
    assert np.array_equal(_abi("lbm_diagnostics_noalloc", s), _abi("lbm_diagnostics", s))


def test_noalloc_rejects_beyond_its_array():
    """160x150x150 all-fluid box: 3.6 M compact cells, more than the 3 049 472
    whose partials fit the fixed array."""
    case = periodic_box_case(nx=160, ny=150, nz=150, ell=4.0)
    s = Solver.from_case(case)
    with pytest.raises(lbm.LBMError) as e:
        _abi("lbm_diagnostics_noalloc", s)
    assert e.value.status == lbm.LBM_E_INVALID
    assert "bytes of scratch" in str(e.value)
    # the context is not poisoned and the workspace version still works
    d = _abi("lbm_diagnostics", s)
    assert d[9] == 0
