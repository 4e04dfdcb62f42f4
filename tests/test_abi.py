"""C-ABI checks that need no GPU: every function include/lbm.h declares is
exported by liblbm.so, and invalid arguments are rejected by host-side
validation before any device work."""

import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_2402_10809_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported():
    names = _declared()
    assert "lbm_create" in names and "lbm_step" in names and "lbm_adjoint" in names
    L = lbm.lib()
    for n in names:
        assert hasattr(L, n), n
    # and nothing else with the lbm_ prefix is required by the binding
    assert len(names) == 18


def _grid(nx=8, ny=6, nz=5, storage=0, periodic=(0, 0, 0)):
    g = lbm.lbm_grid()
    g.nx, g.ny, g.nz = nx, ny, nz
    for a in range(3):
        g.periodic[a] = periodic[a]
    g.storage = storage
    g.shift_mode = 0
    return g


def test_workspace_size_and_validation():
    g = _grid()
    solid = np.zeros((5, 6, 8), np.uint8)
    n0 = lbm.lbm_workspace_size(g, solid)
    n1 = lbm.lbm_workspace_size(g, solid, 100, 10)
    assert n0 > 2 * 19 * 240 * 4 and n1 > n0
    g16 = _grid(storage=1)
    assert lbm.lbm_workspace_size(g16, solid) < n0
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_workspace_size(_grid(nx=0), solid)
    assert e.value.status == lbm.LBM_E_INVALID
    with pytest.raises(lbm.LBMError):
        lbm.lbm_workspace_size(_grid(nx=4096), np.zeros((5, 6, 4096), np.uint8))
    with pytest.raises(lbm.LBMError):
        lbm.lbm_workspace_size(g, np.ones((5, 6, 8), np.uint8))  # no fluid
    g_round = _grid(storage=1)
    g_round.rounding = lbm.LBM_ROUND_NEAREST
    assert lbm.lbm_workspace_size(g_round, solid) == lbm.lbm_workspace_size(g16, solid)
    g_round.rounding = 3  # not an lbm_rounding value
    with pytest.raises(lbm.LBMError):
        lbm.lbm_workspace_size(g_round, solid)
    g_round.rounding = -1
    with pytest.raises(lbm.LBMError):
        lbm.lbm_workspace_size(g_round, solid)
    # more compact cells than 32-bit byte offsets into 19 FP32 planes allow
    # (58.7 M all-fluid cells); the same box with a sparse mask is accepted
    big = np.zeros((224, 512, 512), np.uint8)
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_workspace_size(_grid(nx=512, ny=512, nz=224), big)
    assert "offsets" in str(e.value)
    big[:, :, 256:] = 1
    assert lbm.lbm_workspace_size(_grid(nx=512, ny=512, nz=224), big) > 0
    # D3Q27: 27 planes and 64-bit link words, a lower compact-cell limit (39.7 M)
    g27 = _grid()
    g27.velocity_set = 27
    assert lbm.lbm_workspace_size(g27, solid) > n0
    big27 = np.zeros((224, 512, 512), np.uint8)
    big27[:, :, 384:] = 1  # 44 M cells: within the D3Q19 limit, beyond the D3Q27 one
    assert lbm.lbm_workspace_size(_grid(nx=512, ny=512, nz=224), big27) > 0
    g27b = _grid(nx=512, ny=512, nz=224)
    g27b.velocity_set = 27
    with pytest.raises(lbm.LBMError):
        lbm.lbm_workspace_size(g27b, big27)
    g23 = _grid()
    g23.velocity_set = 23
    with pytest.raises(lbm.LBMError):
        lbm.lbm_workspace_size(g23, solid)


def _create(g, solid, phi, rh=(0.1, 0.01, 50.0, 0.36, 2.0), po=(0.1, 2.0, 180.0), op=None, ws=4096,
            ws_bytes=1 << 30, aniso=None, aniso_iters=6):
    L = lbm.lib()
    r = lbm.lbm_rheology(*rh)
    p = lbm.lbm_porous()
    p.nu_darcy, p.d, p.kc = po
    if aniso is not None:
        for k in range(6):
            p.aniso[k] = aniso[k]
        p.aniso_iters = aniso_iters
    ctx = ct.c_void_p()
    s = np.ascontiguousarray(solid, np.uint8)
    f = np.ascontiguousarray(phi, np.float32)
    return L.lbm_create(ct.byref(g), s.ctypes.data_as(ct.c_void_p), f.ctypes.data_as(ct.c_void_p), None,
                        ct.byref(r), ct.byref(p), ct.byref(op) if op is not None else None, ct.c_void_p(ws),
                        ct.c_size_t(ws_bytes), None, ct.byref(ctx))


def test_create_rejects_bad_inputs_before_device_work():
    g = _grid()
    solid = np.zeros((5, 6, 8), np.uint8)
    phi = np.ones((5, 6, 8), np.float32)
    bad_phi = phi.copy()
    bad_phi[2, 3, 4] = 0.0
    assert _create(g, solid, bad_phi) == lbm.LBM_E_INVALID
    bad_phi[2, 3, 4] = 1.5
    assert _create(g, solid, bad_phi) == lbm.LBM_E_INVALID
    assert _create(g, solid, phi, rh=(0.0, 0.01, 50.0, 0.36, 2.0)) == lbm.LBM_E_INVALID
    assert _create(g, solid, phi, rh=(0.1, -0.01, 50.0, 0.36, 2.0)) == lbm.LBM_E_INVALID
    assert _create(g, solid, phi, po=(0.1, 0.0, 180.0)) == lbm.LBM_E_INVALID
    # misaligned or small workspace
    assert _create(g, solid, phi, ws=4097) == lbm.LBM_E_WORKSPACE
    assert _create(g, solid, phi, ws_bytes=1000) == lbm.LBM_E_WORKSPACE
    # open face on a periodic x axis
    shape = np.ones((5, 6), np.float32)
    op = lbm.lbm_open()
    op.inlet, op.shape_yz, op.a0, op.a1, op.period = 1, shape.ctypes.data_as(ct.c_void_p), 0.01, 0.0, 10.0
    assert _create(_grid(periodic=(1, 0, 0)), solid, phi, op=op) == lbm.LBM_E_INVALID
    # porosity must be 1 on open-face cells
    p2 = phi.copy()
    p2[:, :, 0] = 0.9
    assert _create(g, solid, p2, op=op) == lbm.LBM_E_INVALID
    msg = lbm.lib().lbm_last_error().decode()
    assert "open-face" in msg
    # outflow kind, ramp and waveform table
    op2 = lbm.lbm_open()
    op2.outlet = 3
    assert _create(g, solid, phi, op=op2) == lbm.LBM_E_INVALID
    op.ramp_steps = -1
    assert _create(g, solid, phi, op=op) == lbm.LBM_E_INVALID
    op.ramp_steps = 0
    table = np.ones(2000, np.float64)
    op.wave_table, op.table_len = table.ctypes.data_as(ct.c_void_p), 2000
    assert _create(g, solid, phi, op=op) == lbm.LBM_E_INVALID
    # anisotropic permeability: positive definite shape, 1..64 iterations, D3Q19 only
    assert _create(g, solid, phi, aniso=(1.0, 1.0, -0.5, 0.0, 0.0, 0.0)) == lbm.LBM_E_INVALID
    assert _create(g, solid, phi, aniso=(1.0, 1.0, 1.0, 2.0, 0.0, 0.0)) == lbm.LBM_E_INVALID
    assert _create(g, solid, phi, aniso=(2.0, 1.0, 1.0, 0.3, 0.0, 0.0), aniso_iters=0) == lbm.LBM_E_INVALID
    assert "aniso_iters" in lbm.lib().lbm_last_error().decode()
    g27 = _grid()
    g27.velocity_set = 27
    assert _create(g27, solid, phi, aniso=(2.0, 1.0, 1.0, 0.3, 0.0, 0.0)) == lbm.LBM_E_INVALID


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: asked for more it exits with status 2 and a
    message, before touching a device."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], cwd=root,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
