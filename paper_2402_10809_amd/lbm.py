"""ctypes binding of liblbm.so: the C ABI of include/lbm.h under the same names,
plus a small ``Solver`` class that owns a context and its device workspace.

PyTorch provides the device memory (the workspace and output tensors) and the
stream; every step of the method runs in the library's HIP kernels.  There is
no CPU fallback: if liblbm.so is missing or no HIP device is present the calls
raise.
"""

from __future__ import annotations

import ctypes as ct
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_E_INVALID, LBM_E_DEVICE, LBM_E_UNSTABLE, LBM_E_STATE, LBM_E_WORKSPACE = range(6)
STORAGE = {"fp32": 0, "fp16": 1, "bf16": 2}
ARITH = {"auto": 0, "fp32": 1, "fp64": 2}
ROUNDING = {"stochastic": 0, "conserve": 1, "nearest": 2}
LBM_ROUND_STOCHASTIC, LBM_ROUND_CONSERVE, LBM_ROUND_NEAREST = 0, 1, 2
NDIAG = 12
DIAG_NAMES = ["mass", "mom_x", "mom_y", "mom_z", "ke", "ke_region", "max_u", "min_omega", "max_omega",
              "nonfinite", "t", "wss_region"]
OBJECTIVE = {"ke": 0, "wss": 1}


class lbm_grid(ct.Structure):
    _fields_ = [("nx", ct.c_int), ("ny", ct.c_int), ("nz", ct.c_int), ("periodic", ct.c_int * 3),
                ("storage", ct.c_int), ("shift_mode", ct.c_int), ("arith", ct.c_int), ("velocity_set", ct.c_int),
                ("rounding", ct.c_int)]


class lbm_rheology(ct.Structure):
    _fields_ = [("nu0", ct.c_double), ("nu_inf", ct.c_double), ("lam", ct.c_double), ("n", ct.c_double),
                ("a", ct.c_double)]


class lbm_porous(ct.Structure):
    _fields_ = [("nu_darcy", ct.c_double), ("d", ct.c_double), ("kc", ct.c_double), ("forchheimer", ct.c_int),
                ("g", ct.c_double * 3), ("aniso", ct.c_double * 6), ("aniso_iters", ct.c_int)]


class lbm_open(ct.Structure):
    _fields_ = [("inlet", ct.c_int), ("shape_yz", ct.c_void_p), ("a0", ct.c_double), ("a1", ct.c_double),
                ("period", ct.c_double), ("outlet", ct.c_int), ("rho_out", ct.c_double),
                ("ramp_steps", ct.c_int), ("wave_table", ct.c_void_p), ("table_len", ct.c_int)]


class lbm_objective(ct.Structure):
    _fields_ = [("t_begin", ct.c_int), ("t_end", ct.c_int), ("kind", ct.c_int), ("fp64_adjoint", ct.c_int)]


class LBMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lbm status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2402_10809_amd.build.build()")
        L = ct.CDLL(LIB_PATH)
        vp, i32, i64, dbl, sz = ct.c_void_p, ct.c_int, ct.c_int64, ct.c_double, ct.c_size_t
        P = ct.POINTER
        L.lbm_workspace_size.argtypes = [P(lbm_grid), vp, i32, i32, P(sz)]
        L.lbm_create.argtypes = [P(lbm_grid), vp, vp, vp, P(lbm_rheology), P(lbm_porous), P(lbm_open), vp, sz, vp,
                                 P(vp)]
        L.lbm_step.argtypes = [vp, i32]
        L.lbm_moments.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.lbm_diagnostics.argtypes = [vp, vp]
        L.lbm_diagnostics_noalloc.argtypes = [vp, vp]
        L.lbm_get_state.argtypes = [vp, vp, vp]
        L.lbm_set_state.argtypes = [vp, vp, vp]
        L.lbm_set_porosity.argtypes = [vp, vp]
        L.lbm_reset.argtypes = [vp]
        L.lbm_adjoint.argtypes = [vp, P(lbm_objective), i32, i32, P(dbl), vp]
        L.lbm_fluid_cells.argtypes = [vp, P(i64)]
        L.lbm_fluid_index.argtypes = [vp, vp]
        L.lbm_time.argtypes = [vp, P(i64)]
        L.lbm_copy_probe.argtypes = [vp, vp, sz, vp]
        L.lbm_bandwidth_probe.argtypes = [i32, vp, vp, sz, vp]
        L.lbm_last_error.restype = ct.c_char_p
        L.lbm_destroy.argtypes = [vp]
        L.lbm_destroy.restype = None
        for name in ("lbm_workspace_size", "lbm_create", "lbm_step", "lbm_moments", "lbm_diagnostics",
                     "lbm_diagnostics_noalloc",
                     "lbm_get_state", "lbm_set_state", "lbm_set_porosity", "lbm_reset", "lbm_adjoint",
                     "lbm_fluid_cells", "lbm_fluid_index", "lbm_time", "lbm_copy_probe", "lbm_bandwidth_probe"):
            getattr(L, name).restype = ct.c_int
        _lib = L
    return _lib


def check(status: int):
    if status != LBM_OK:
        raise LBMError(status, lib().lbm_last_error().decode(errors="replace"))


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


# --- thin wrappers with the ABI's names (argument marshalling only) ---------

def lbm_workspace_size(grid: lbm_grid, solid: np.ndarray, adjoint_T: int = 0, ckpt_every: int = 0) -> int:
    n = ct.c_size_t(0)
    s = np.ascontiguousarray(solid.reshape(-1), dtype=np.uint8)
    check(lib().lbm_workspace_size(ct.byref(grid), _p(s), int(adjoint_T), int(ckpt_every), ct.byref(n)))
    return int(n.value)


def lbm_step(ctx, n: int):
    check(lib().lbm_step(ctx, int(n)))


def lbm_copy_probe(dst_ptr: int, src_ptr: int, nbytes: int, stream_ptr: int = 0):
    check(lib().lbm_copy_probe(ct.c_void_p(dst_ptr), ct.c_void_p(src_ptr), ct.c_size_t(nbytes),
                               ct.c_void_p(stream_ptr)))


PROBE = {"copy": 0, "copy_nt": 1, "read": 2, "write": 3}
PROBE_BLOCKS = 8192


def lbm_bandwidth_probe(kind: str, dst_ptr: int, src_ptr: int, nbytes: int, stream_ptr: int = 0):
    check(lib().lbm_bandwidth_probe(PROBE[kind], ct.c_void_p(dst_ptr), ct.c_void_p(src_ptr), ct.c_size_t(nbytes),
                                    ct.c_void_p(stream_ptr)))


class Solver:
    """One simulation context on the current HIP device.

    solid, phi, region: arrays of shape (nz, ny, nx) (box index x + nx*(y + ny*z)).
    rheology: dict(nu0, nu_inf, lam, n, a); porous: dict(nu_d, d, kc, forchheimer, g[, aniso=(M xx yy zz xy xz yz),
    aniso_iters]).
    inlet: None or dict(shape=(nz, ny) array, a0, a1, period[, ramp=steps][, table=FP64 samples of one period]);
    outlet: None, rho_out (constant-density outflow) or "extrapolation" (the non-reflecting outflow).
    adjoint_T/ckpt: reserve workspace for lbm_adjoint runs of up to adjoint_T steps.
    lattice: 19 (D3Q19) or 27 (D3Q27).
    rounding: the rounding of FP16/BF16 storage: "stochastic" (default), "conserve" or "nearest".
    """

    def __init__(self, solid, phi, *, periodic=(False, False, False), storage="fp32", shift_mode=0, arith="auto",
                 region=None, rheology=None, porous=None, inlet=None, outlet=None, adjoint_T=0, ckpt=64,
                 lattice=19, rounding="stochastic", device=None, stream=None):
        import torch

        self.torch = torch
        solid = np.ascontiguousarray(solid, dtype=np.uint8)
        nz, ny, nx = solid.shape
        self.shape = (nz, ny, nx)
        self.nbox = nx * ny * nz
        self.device = torch.device("cuda" if device is None else device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        g = lbm_grid()
        g.nx, g.ny, g.nz = nx, ny, nz
        for a in range(3):
            g.periodic[a] = int(bool(periodic[a]))
        g.storage = STORAGE[storage]
        g.shift_mode = int(shift_mode)
        g.arith = ARITH[arith]
        g.velocity_set = int(lattice)
        g.rounding = ROUNDING[rounding]
        self.q = 27 if int(lattice) == 27 else 19
        self.grid = g
        self.storage = storage
        rh = dict(nu0=0.1, nu_inf=0.01, lam=50.0, n=0.36, a=2.0) if rheology is None else rheology
        po = dict(nu_d=0.1, d=2.0, kc=180.0, forchheimer=0, g=(0.0, 0.0, 0.0)) if porous is None else porous
        r = lbm_rheology(rh["nu0"], rh["nu_inf"], rh["lam"], rh["n"], rh["a"])
        p = lbm_porous()
        p.nu_darcy, p.d, p.kc, p.forchheimer = po["nu_d"], po["d"], po["kc"], int(po.get("forchheimer", 0))
        for a in range(3):
            p.g[a] = float(po["g"][a])
        if po.get("aniso") is not None:
            for k in range(6):
                p.aniso[k] = float(po["aniso"][k])
            p.aniso_iters = int(po.get("aniso_iters", 8))
        o = lbm_open()
        self._shape_yz = None
        if inlet is not None:
            self._shape_yz = np.ascontiguousarray(inlet["shape"], dtype=np.float32)
            o.inlet, o.shape_yz = 1, _p(self._shape_yz)
            o.a0, o.a1, o.period = float(inlet["a0"]), float(inlet["a1"]), float(inlet["period"])
            o.ramp_steps = int(inlet.get("ramp", 0) or 0)
            if inlet.get("table") is not None:
                self._wave = np.ascontiguousarray(inlet["table"], dtype=np.float64)
                o.wave_table, o.table_len = _p(self._wave), int(self._wave.size)
        if isinstance(outlet, str):
            if outlet != "extrapolation":
                raise ValueError(f"unknown outlet {outlet!r}")
            o.outlet = 2
        elif outlet is not None:
            o.outlet, o.rho_out = 1, float(outlet)
        self.adjoint_T, self.ckpt = int(adjoint_T), int(ckpt)
        nbytes = lbm_workspace_size(g, solid, self.adjoint_T, self.ckpt)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        ph = np.ascontiguousarray(phi, dtype=np.float32)
        reg = None if region is None else np.ascontiguousarray(region, dtype=np.uint8)
        ctx = ct.c_void_p()
        check(lib().lbm_create(ct.byref(g), _p(solid), _p(ph), _p(reg), ct.byref(r), ct.byref(p), ct.byref(o),
                               ct.c_void_p(base + off), ct.c_size_t(nbytes), ct.c_void_p(self.stream.cuda_stream),
                               ct.byref(ctx)))
        self.ctx = ctx
        n = ct.c_int64(0)
        check(lib().lbm_fluid_cells(ctx, ct.byref(n)))
        self.n_fluid = int(n.value)

    @classmethod
    def from_case(cls, case, **kw):
        """Build from a case object with the attributes of ``synth.Case``."""
        inlet = None
        if getattr(case, "inlet", False):
            a0, a1, period = case.wave
            inlet = dict(shape=case.inlet_shape, a0=a0, a1=a1, period=period,
                         ramp=getattr(case, "ramp_steps", 0), table=getattr(case, "wave_table", None))
        kind = int(getattr(case, "outlet", 0) or 0)
        outlet = "extrapolation" if kind == 2 else (case.rho_out if kind == 1 else None)
        kw.setdefault("lattice", int(getattr(case, "lattice", 19) or 19))
        return cls(case.solid, case.phi, periodic=case.periodic, region=case.sac, rheology=case.rheology,
                   porous=case.porous, inlet=inlet, outlet=outlet, **kw)

    def close(self):
        if getattr(self, "ctx", None):
            lib().lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stepping -------------------------------------------------------------
    def step(self, n: int = 1):
        check(lib().lbm_step(self.ctx, int(n)))

    def reset(self):
        check(lib().lbm_reset(self.ctx))

    @property
    def t(self) -> int:
        v = ct.c_int64(0)
        check(lib().lbm_time(self.ctx, ct.byref(v)))
        return int(v.value)

    def fluid_index(self) -> np.ndarray:
        out = np.empty(self.n_fluid, np.int64)
        check(lib().lbm_fluid_index(self.ctx, _p(out)))
        return out

    # -- outputs --------------------------------------------------------------
    def moments(self, sigma: bool = False, tau: bool = False):
        """Dense device tensors rho, u (3, nz, ny, nx), shear, omega [, sigma (6, ...)]
        [, tau (3, ...): the wall shear stress on the voxel wall]."""
        t = self.torch
        nz, ny, nx = self.shape
        kw = dict(dtype=t.float32, device=self.device)
        out = dict(rho=t.empty((nz, ny, nx), **kw), u=t.empty((3, nz, ny, nx), **kw),
                   shear=t.empty((nz, ny, nx), **kw), omega=t.empty((nz, ny, nx), **kw))
        if sigma:
            out["sigma"] = t.empty((6, nz, ny, nx), **kw)
        if tau:
            out["tau"] = t.empty((3, nz, ny, nx), **kw)
        check(lib().lbm_moments(self.ctx, ct.c_void_p(out["rho"].data_ptr()), ct.c_void_p(out["u"].data_ptr()),
                                ct.c_void_p(out["shear"].data_ptr()), ct.c_void_p(out["omega"].data_ptr()),
                                ct.c_void_p(out["sigma"].data_ptr()) if sigma else None,
                                ct.c_void_p(out["tau"].data_ptr()) if tau else None))
        return out

    def diagnostics(self) -> dict:
        out = np.zeros(NDIAG, np.float64)
        check(lib().lbm_diagnostics(self.ctx, _p(out)))
        return dict(zip(DIAG_NAMES, out.tolist()))

    def diagnostics_noalloc(self) -> dict:
        """As diagnostics(), through lbm_diagnostics_noalloc (scratch in the
        library's fixed device array instead of the workspace)."""
        out = np.zeros(NDIAG, np.float64)
        check(lib().lbm_diagnostics_noalloc(self.ctx, _p(out)))
        return dict(zip(DIAG_NAMES, out.tolist()))

    def get_state(self):
        f = np.empty((self.q, self.n_fluid), np.float64)
        om = np.empty(self.n_fluid, np.float32)
        check(lib().lbm_get_state(self.ctx, _p(f), _p(om)))
        return f, om

    def set_state(self, f: Optional[np.ndarray] = None, omega: Optional[np.ndarray] = None):
        fa = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
        oa = None if omega is None else np.ascontiguousarray(omega, dtype=np.float32)
        check(lib().lbm_set_state(self.ctx, _p(fa), _p(oa)))

    def set_porosity(self, phi):
        """Replace the porosity (box layout (nz, ny, nx)) and reset to rest.  A
        torch tensor on the solver's device is passed as is (FP32, contiguous);
        anything else is first copied to the device."""
        t = self.torch
        if not (isinstance(phi, t.Tensor) and phi.device == self.device and phi.dtype == t.float32
                and phi.is_contiguous()):
            phi = t.as_tensor(np.ascontiguousarray(phi, dtype=np.float32) if not isinstance(phi, t.Tensor) else phi,
                              dtype=t.float32).to(self.device).contiguous()
        if phi.numel() != self.nbox:
            raise ValueError(f"porosity has {phi.numel()} values, the box {self.nbox}")
        # the copy above (if any) runs on torch's current stream: order it before the library's
        t.cuda.current_stream(self.device).synchronize()
        check(lib().lbm_set_porosity(self.ctx, ct.c_void_p(phi.data_ptr())))

    def objective(self, t_begin: int, t_end: int, T: int, kind: str = "ke") -> float:
        """J alone (forward pass from rest, no gradient); the context ends at rest.
        kind: "ke" (region kinetic energy) or "wss" (WSS over the region's wall)."""
        obj = lbm_objective(int(t_begin), int(t_end), OBJECTIVE[kind], 0)
        J = ct.c_double(0.0)
        check(lib().lbm_adjoint(self.ctx, ct.byref(obj), int(T), 1, ct.byref(J), None))
        return float(J.value)

    def adjoint(self, t_begin: int, t_end: int, T: int, ckpt: Optional[int] = None, kind: str = "ke",
                fp64: bool = False):
        """J and dJ/dphi (device tensor, box layout) of the region objective:
        kind "ke" (kinetic energy) or "wss" (wall shear stress magnitude);
        fp64: FP64 adjoint populations in the reverse sweep."""
        t = self.torch
        ck = self.ckpt if ckpt is None else int(ckpt)
        obj = lbm_objective(int(t_begin), int(t_end), OBJECTIVE[kind], 1 if fp64 else 0)
        J = ct.c_double(0.0)
        grad = t.empty(self.shape, dtype=t.float32, device=self.device)
        check(lib().lbm_adjoint(self.ctx, ct.byref(obj), int(T), ck, ct.byref(J), ct.c_void_p(grad.data_ptr())))
        return float(J.value), grad
