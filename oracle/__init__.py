"""FP64 CPU oracle for the VANSE Carreau-Yasuda lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg use this package; the product path never imports
it.  It shares no code with the GPU path: the C++ in ``lbm_oracle.cpp`` is a
plain per-cell FP64 implementation written from the paper's method section,
and ``bruteforce.py`` is a second, dense-array NumPy transcription used to
cross-check it on tiny lattices.
"""

from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.cpp")
# one library per velocity set (the source is compiled with ORACLE_Q = 19 / 27);
# ORACLE_LIB_DIR selects another directory of the same two libraries (the
# sanitizer builds of tests/test_sanitizers.py)
_DIR = os.environ.get("ORACLE_LIB_DIR", _HERE)
_LIBS = {19: os.path.join(_DIR, "liboracle.so"), 27: os.path.join(_DIR, "liboracle27.so")}
_LIB = _LIBS[19]
Q = 19
SANITIZE_FLAGS = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def build(force: bool = True, out_dir: str = None, sanitize: bool = False) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` (D3Q19) and
    ``oracle/liboracle27.so`` (D3Q27) (g++, OpenMP); into ``out_dir`` instead
    if given, and with AddressSanitizer and UndefinedBehaviorSanitizer if
    ``sanitize``."""
    libs = _LIBS if out_dir is None else {q: os.path.join(out_dir, os.path.basename(p)) for q, p in _LIBS.items()}
    for q, path in libs.items():
        if force or not os.path.exists(path):
            opt = SANITIZE_FLAGS if sanitize else ["-O2"]
            cmd = ["g++"] + opt + ["-std=c++17", "-fopenmp", "-fPIC", "-shared", f"-DORACLE_Q={q}", "-o",
                                   path + ".tmp", _SRC]
            subprocess.check_call(cmd)
            os.replace(path + ".tmp", path)
    return libs[19]


class _Case(ct.Structure):
    _fields_ = [
        ("nx", ct.c_int), ("ny", ct.c_int), ("nz", ct.c_int),
        ("periodic", ct.c_int * 3),
        ("solid", ct.c_void_p), ("phi", ct.c_void_p), ("sac", ct.c_void_p),
        ("inlet", ct.c_int), ("outlet", ct.c_int),
        ("inlet_shape", ct.c_void_p),
        ("a0", ct.c_double), ("a1", ct.c_double), ("period", ct.c_double),
        ("rho_out", ct.c_double),
        ("nu0", ct.c_double), ("nu_inf", ct.c_double), ("lam", ct.c_double), ("n", ct.c_double), ("a", ct.c_double),
        ("nu_d", ct.c_double), ("kc", ct.c_double), ("d", ct.c_double),
        ("forchheimer", ct.c_int),
        ("g", ct.c_double * 3),
        ("ramp", ct.c_int), ("wave_table", ct.c_void_p), ("table_len", ct.c_int),
        ("aniso", ct.c_double * 6), ("aniso_iters", ct.c_int),
    ]


_libs = {}


def lattice_of(case) -> int:
    """Velocity-set size of a case (attribute ``lattice``, default 19)."""
    return int(getattr(case, "lattice", 19) or 19)


def lib(q: int = 19):
    if q not in _libs:
        if not os.path.exists(_LIBS[q]):
            build(force=False)
        L = ct.CDLL(_LIBS[q])
        vp, i32, i64, dbl = ct.c_void_p, ct.c_int, ct.c_int64, ct.c_double
        L.oracle_new.restype = vp
        L.oracle_new.argtypes = [ct.POINTER(_Case)]
        L.oracle_free.argtypes = [vp]
        L.oracle_nfluid.restype = i64
        L.oracle_nfluid.argtypes = [vp]
        L.oracle_cells.argtypes = [vp, vp]
        L.oracle_neighbours.argtypes = [vp, vp]
        L.oracle_amplitude.restype = dbl
        L.oracle_amplitude.argtypes = [vp, i32]
        L.oracle_set_phi.argtypes = [vp, vp]
        L.oracle_init.argtypes = [vp, vp, vp]
        L.oracle_run.argtypes = [vp, vp, vp, i32, i32, vp]
        L.oracle_moments.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp, vp]
        L.oracle_cell.argtypes = [ct.POINTER(_Case), vp, dbl, dbl, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.oracle_zouhe_inlet.argtypes = [vp, dbl, dbl, dbl]
        L.oracle_zouhe_outlet.argtypes = [vp, dbl]
        L.oracle_lattice.argtypes = [vp, vp]
        L.oracle_objective.restype = dbl
        L.oracle_objective.argtypes = [vp, i32, i32, i32, i32]
        L.oracle_grad_dual.argtypes = [vp, i32, i32, i32, vp, i32, vp, vp, i32]
        L.oracle_grad_reverse.argtypes = [vp, i32, i32, i32, i32, vp, vp, i32]
        L.oracle_threads.restype = i32
        L.oracle_set_threads.restype = i32
        L.oracle_set_threads.argtypes = [i32]
        L.oracle_q.restype = i32
        assert L.oracle_q() == q
        _libs[q] = L
    return _libs[q]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p) if a is not None else None


def make_struct(case, keep: list, **override) -> _Case:
    """Fill the C case description from a ``synth.Case``; ``keep`` holds the
    arrays so they outlive the struct."""
    solid = np.ascontiguousarray(case.solid.reshape(-1), dtype=np.uint8)
    phi = np.ascontiguousarray(override.get("phi", case.phi).reshape(-1), dtype=np.float64)
    sac = np.ascontiguousarray(case.sac.reshape(-1), dtype=np.uint8)
    shape = None
    if case.inlet_shape is not None:
        shape = np.ascontiguousarray(case.inlet_shape.reshape(-1), dtype=np.float64)
    keep.extend([solid, phi, sac, shape])
    s = _Case()
    s.nx, s.ny, s.nz = case.nx, case.ny, case.nz
    for a in range(3):
        s.periodic[a] = int(bool(case.periodic[a]))
    s.solid, s.phi, s.sac = _ptr(solid), _ptr(phi), _ptr(sac)
    s.inlet, s.outlet = int(case.inlet), int(case.outlet)
    s.inlet_shape = _ptr(shape)
    s.a0, s.a1, s.period = (float(v) for v in case.wave)
    s.rho_out = float(case.rho_out)
    rh = case.rheology
    s.nu0, s.nu_inf, s.lam, s.n, s.a = rh["nu0"], rh["nu_inf"], rh["lam"], rh["n"], rh["a"]
    po = case.porous
    s.nu_d, s.kc, s.d = po["nu_d"], po["kc"], po["d"]
    s.forchheimer = int(po.get("forchheimer", 0))
    for a in range(3):
        s.g[a] = float(po["g"][a])
    s.ramp = int(getattr(case, "ramp_steps", 0) or 0)
    an = po.get("aniso")
    if an is not None:
        for k in range(6):
            s.aniso[k] = float(an[k])
        s.aniso_iters = int(po.get("aniso_iters", 8))
    table = getattr(case, "wave_table", None)
    if table is not None:
        table = np.ascontiguousarray(table, dtype=np.float64)
        keep.append(table)
        s.wave_table, s.table_len = _ptr(table), int(table.size)
    return s


OBJECTIVE = {"ke": 0, "wss": 1}


class Oracle:
    """One case on the CPU.  State arrays: ``f`` of shape (19, n_fluid) with the
    pre-collision populations in canonical D3Q19 order (rest, +x, -x, +y, -y,
    +z, -z, then the 12 edge directions in opposite pairs), ``omega`` of shape
    (n_fluid,) with the previous step's relaxation rate."""

    def __init__(self, case, phi=None):
        self.case = case
        self._keep = []
        kw = {} if phi is None else dict(phi=phi)
        self._struct = make_struct(case, self._keep, **kw)
        self.q = lattice_of(case)
        self._L = lib(self.q)
        self.h = self._L.oracle_new(ct.byref(self._struct))
        self.nf = int(self._L.oracle_nfluid(self.h))

    def __del__(self):
        if getattr(self, "h", None):
            self._L.oracle_free(self.h)
            self.h = None

    def cells(self) -> np.ndarray:
        out = np.empty(self.nf, np.int64)
        self._L.oracle_cells(self.h, _ptr(out))
        return out

    def neighbours(self) -> np.ndarray:
        out = np.empty((self.q, self.nf), np.int32)
        self._L.oracle_neighbours(self.h, _ptr(out))
        return out

    def amplitude(self, t: int) -> float:
        return float(self._L.oracle_amplitude(self.h, int(t)))

    def set_phi(self, phi_box: np.ndarray):
        p = np.ascontiguousarray(phi_box.reshape(-1), dtype=np.float64)
        self._L.oracle_set_phi(self.h, _ptr(p))

    def init(self):
        f = np.empty((self.q, self.nf), np.float64)
        om = np.empty(self.nf, np.float64)
        self._L.oracle_init(self.h, _ptr(f), _ptr(om))
        return f, om

    def run(self, f, omega, t0: int, nsteps: int, want_ke: bool = False):
        """Advance ``nsteps`` steps from step index ``t0`` (in place)."""
        assert f.dtype == np.float64 and f.flags.c_contiguous and f.shape == (self.q, self.nf)
        assert omega.dtype == np.float64 and omega.flags.c_contiguous
        ke = np.empty(nsteps, np.float64) if want_ke else None
        self._L.oracle_run(self.h, _ptr(f), _ptr(omega), int(t0), int(nsteps), _ptr(ke))
        return ke

    def moments(self, f, omega, t: int):
        nf = self.nf
        rho = np.empty(nf)
        u = np.empty((3, nf))
        shear = np.empty(nf)
        om = np.empty(nf)
        sigma = np.empty((6, nf))
        tau = np.empty((3, nf))
        self._L.oracle_moments(self.h, _ptr(np.ascontiguousarray(f)), _ptr(np.ascontiguousarray(omega)), int(t),
                             _ptr(rho), _ptr(u), _ptr(shear), _ptr(om), _ptr(sigma), _ptr(tau))
        return dict(rho=rho, u=u, shear=shear, omega=om, sigma=sigma, tau=tau)

    def objective(self, T: int, tb: int, te: int, kind: str = "ke") -> float:
        """J over steps [tb, te) of a T-step run from rest; kind "ke" (region
        kinetic energy) or "wss" (WSS magnitude over the region's wall cells)."""
        return float(self._L.oracle_objective(self.h, int(T), int(tb), int(te), OBJECTIVE[kind]))

    def grad_dual(self, T: int, tb: int, te: int, box_cells, kind: str = "ke"):
        cells = np.ascontiguousarray(np.asarray(box_cells, dtype=np.int64))
        assert cells.size <= 16
        J = np.zeros(1)
        g = np.zeros(cells.size)
        self._L.oracle_grad_dual(self.h, int(T), int(tb), int(te), _ptr(cells), int(cells.size), _ptr(J), _ptr(g),
                               OBJECTIVE[kind])
        return float(J[0]), g

    def grad_reverse(self, T: int, tb: int, te: int, ckpt: int, kind: str = "ke"):
        J = np.zeros(1)
        g = np.zeros(self.case.n_box)
        self._L.oracle_grad_reverse(self.h, int(T), int(tb), int(te), int(ckpt), _ptr(J), _ptr(g), OBJECTIVE[kind])
        if np.isnan(J[0]):
            raise ValueError("the reverse sweep supports the density outflow only")
        return float(J[0]), g.reshape(self.case.nz, self.case.ny, self.case.nx)


def cell(case, f, omega_prev, phi, phit):
    """Evaluate one cell's update (no open-face fill).  Returns a dict with rho,
    u, F, feq, Pi (xx yy zz xy xz yz), shear, nu, omega and q."""
    keep = []
    s = make_struct(case, keep)
    q = lattice_of(case)
    f = np.ascontiguousarray(f, dtype=np.float64)
    phit = np.ascontiguousarray(phit, dtype=np.float64)
    out = {k: np.zeros(n) for k, n in dict(rho=1, u=3, F=3, feq=q, Pi=6, shear=1, nu=1, omega=1, q=q).items()}
    lib(q).oracle_cell(ct.byref(s), _ptr(f), float(omega_prev), float(phi), _ptr(phit),
                       *[_ptr(out[k]) for k in ("rho", "u", "F", "feq", "Pi", "shear", "nu", "omega", "q")])
    for k in ("rho", "shear", "nu", "omega"):
        out[k] = float(out[k][0])
    return out


def zouhe_inlet(f, ux, uy=0.0, uz=0.0):
    """Zou-He inflow fill of one cell's populations (the set of len(f))."""
    f = np.array(f, dtype=np.float64)
    lib(f.size).oracle_zouhe_inlet(_ptr(f), float(ux), float(uy), float(uz))
    return f


def zouhe_outlet(f, rho_out):
    """Zou-He constant-density outflow fill (the set of len(f))."""
    f = np.array(f, dtype=np.float64)
    lib(f.size).oracle_zouhe_outlet(_ptr(f), float(rho_out))
    return f


def lattice(q: int = 19):
    c = np.zeros((q, 3), np.int32)
    w = np.zeros(q, np.float64)
    lib(q).oracle_lattice(_ptr(c), _ptr(w))
    return c, w


def threads() -> int:
    return int(lib().oracle_threads())


def set_threads(n: int) -> int:
    """Thread count of the oracle's later parallel loops, in both velocity-set
    libraries; returns the previous count."""
    prev = int(lib(19).oracle_set_threads(int(n)))
    lib(27).oracle_set_threads(int(n))
    return prev
