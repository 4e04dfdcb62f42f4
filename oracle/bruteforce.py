"""Dense-array NumPy transcription of one lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  A second FP64 implementation of the paper's method
section, written over whole (nz, ny, nx) arrays with explicit shifts instead of
the C++ oracle's compact cell list and neighbour table, so that indexing, wall
and open-face mistakes in either show up as a mismatch on tiny lattices.

State layout here: ``f`` of shape (Q, nz, ny, nx) (Q = 19 or 27, the case's
``lattice``), pre-collision populations,
0 on solid voxels and on the unknown links of open-face cells (an extrapolation
outflow keeps its extrapolated values there).
"""

from __future__ import annotations

import numpy as np

# D3Q19: rest, +-x, +-y, +-z, then xy, xz, yz edges, each followed by its opposite
C = np.array([(0, 0, 0),
              (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
              (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
              (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
              (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)], dtype=np.int64)
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
OPP = np.array([int(np.flatnonzero((C == -C[i]).all(axis=1))[0]) for i in range(19)])
CS2 = 1.0 / 3.0

# D3Q27: the 19 above, then the 8 corners in opposite pairs; the weight of a
# velocity with n nonzero components is (2/3)^(3-n) (1/6)^n
C27 = np.concatenate([C, np.array([(1, 1, 1), (-1, -1, -1), (1, 1, -1), (-1, -1, 1),
                                   (1, -1, 1), (-1, 1, -1), (-1, 1, 1), (1, -1, -1)], dtype=np.int64)])
W27 = np.array([(2 / 3) ** (3 - n) * (1 / 6) ** n for n in np.abs(C27).sum(1)])
OPP27 = np.array([int(np.flatnonzero((C27 == -C27[i]).all(axis=1))[0]) for i in range(27)])


def lattice(case):
    """(C, W, OPP) of the case's velocity set."""
    if int(getattr(case, "lattice", 19) or 19) == 27:
        return C27, W27, OPP27
    return C, W, OPP


def _shift(a, c, periodic, fill):
    """b[x] = a[x - c] along the three axes (array axes are z, y, x)."""
    b = a
    for ax_xyz, s in enumerate(c):
        if s == 0:
            continue
        axis = 2 - ax_xyz
        if periodic[ax_xyz]:
            b = np.roll(b, s, axis=axis)
        else:
            b = np.roll(b, s, axis=axis)
            idx = [slice(None)] * b.ndim
            idx[axis] = slice(0, s) if s > 0 else slice(b.shape[axis] + s, None)
            b = b.copy()
            b[tuple(idx)] = fill
    return b


def _link_kinds(case):
    """For each direction i and cell x: 0 if x + c_i is a fluid cell, 1 if it is
    a wall (solid voxel or outside a wall face), 2 if it is outside an open face."""
    C, _, _ = lattice(case)
    fluid = case.solid == 0
    nz, ny, nx = fluid.shape
    kinds = np.zeros((len(C),) + fluid.shape, np.int8)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for i in range(len(C)):
        cx, cy, cz = C[i]
        tx, ty, tz = xx + cx, yy + cy, zz + cz
        out_wall = np.zeros_like(fluid)
        out_open = np.zeros_like(fluid)
        coords = []
        for a, (t, n) in enumerate(((tx, nx), (ty, ny), (tz, nz))):
            outside = (t < 0) | (t >= n)
            if case.periodic[a]:
                t = t % n
            else:
                if a == 0:
                    opn = ((t < 0) & bool(case.inlet)) | ((t >= n) & bool(case.outlet))
                    out_open |= opn
                    out_wall |= outside & ~opn
                else:
                    out_wall |= outside
                t = np.clip(t, 0, n - 1)
            coords.append(t)
        tgt_fluid = fluid[coords[2], coords[1], coords[0]]
        k = np.where(out_wall, 1, np.where(out_open, 2, np.where(tgt_fluid, 0, 1)))
        kinds[i] = k
    return kinds


def inflow_amplitude(case, t):
    """Pre-run ramp to the waveform's starting value over ``case.ramp_steps``
    steps, then the waveform: the sine of ``case.wave`` or the sampled period
    ``case.wave_table`` (linear interpolation, periodic)."""
    a0, a1, period = case.wave
    ramp = int(getattr(case, "ramp_steps", 0) or 0)
    table = getattr(case, "wave_table", None)

    def w(s):
        if table is None:
            return a0 * (1.0 + a1 * np.sin(2.0 * np.pi * s / period))
        tab = np.asarray(table, dtype=np.float64)
        pos = (s / period - np.floor(s / period)) * tab.size
        k = min(int(pos), tab.size - 1)
        return tab[k] + (pos - k) * (tab[(k + 1) % tab.size] - tab[k])

    if t < ramp:
        return (t / ramp) * w(0.0)
    return w(float(t - ramp))


def _zouhe_solve(case, fx, side, rho, ux, uy, uz):
    """D3Q27 Zou-He fill of one face (side +1: the c_x = +1 unknowns of an
    inflow, -1: the c_x = -1 unknowns of an outflow): f_i = f_opp(i) +
    2 w_i rho c_i.u / c_s^2 - 18 w_i (c_iy N_y + c_iz N_z), with (N_y, N_z)
    solved from the transverse momentum balance as a 2x2 linear system."""
    C, W, OPP = lattice(case)
    unk = np.flatnonzero(C[:, 0] == side)
    u = np.stack([np.broadcast_to(ux, rho.shape), np.broadcast_to(uy, rho.shape), np.broadcast_to(uz, rho.shape)])
    base = {}
    for i in unk:
        cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
        base[i] = fx[OPP[i]] + 2 * W[i] * rho * cu / CS2
    known = np.flatnonzero(C[:, 0] != side)
    # transverse momentum with N = 0, and its derivative in N (a constant matrix)
    m0 = [sum(fx[j] * C[j, a] for j in known) + sum(base[i] * C[i, a] for i in unk) for a in (1, 2)]
    D = np.array([[-18 * sum(W[i] * C[i, a] * C[i, b] for i in unk) for b in (1, 2)] for a in (1, 2)])
    rhs = np.stack([rho * u[1] - m0[0], rho * u[2] - m0[1]], axis=-1)
    N = np.linalg.solve(D, rhs[..., None])[..., 0]
    out = fx.copy()
    for i in unk:
        out[i] = base[i] - 18 * W[i] * (C[i, 1] * N[..., 0] + C[i, 2] * N[..., 1])
    return out


def step(case, f, omega_prev, t):
    """One step on dense arrays; returns (f_next, omega_new, fields)."""
    C, W, OPP = lattice(case)
    Q = len(W)
    fluid = case.solid == 0
    phi = np.where(fluid, case.phi.astype(np.float64), 1.0)
    nz, ny, nx = fluid.shape
    kinds = _link_kinds(case)
    f = f.copy()
    # open-face fill: Zou-He inflow on x = 0; constant-density or extrapolation
    # outflow on x = nx-1
    if case.inlet and Q == 27:
        amp = inflow_amplitude(case, t)
        fx = f[:, :, :, 0]
        ux = amp * case.inlet_shape.astype(np.float64)
        rho = (fx[C[:, 0] == 0].sum(0) + 2 * fx[C[:, 0] == -1].sum(0)) / (1 - ux)
        fx = _zouhe_solve(case, fx, 1, rho, ux, 0.0, 0.0)
        f[:, :, :, 0] = np.where(fluid[:, :, 0][None], fx, f[:, :, :, 0])
    elif case.inlet:
        amp = inflow_amplitude(case, t)
        fx = f[:, :, :, 0]
        ux = amp * case.inlet_shape.astype(np.float64)
        zero = C[:, 0] == 0
        neg = C[:, 0] == -1
        rho = (fx[zero].sum(0) + 2 * fx[neg].sum(0)) / (1 - ux)
        ny_ = 0.5 * (fx[zero] * C[zero, 1][:, None, None]).sum(0)
        nz_ = 0.5 * (fx[zero] * C[zero, 2][:, None, None]).sum(0)
        fx[1] = fx[2] + rho * ux / 3
        fx[7] = fx[8] + rho * ux / 6 - ny_
        fx[9] = fx[10] + rho * ux / 6 + ny_
        fx[11] = fx[12] + rho * ux / 6 - nz_
        fx[13] = fx[14] + rho * ux / 6 + nz_
        m = fluid[:, :, 0]
        f[:, :, :, 0] = np.where(m[None], fx, f[:, :, :, 0])
    if int(case.outlet) == 1 and Q == 27:
        fx = f[:, :, :, nx - 1]
        ro = case.rho_out
        ux = (fx[C[:, 0] == 0].sum(0) + 2 * fx[C[:, 0] == 1].sum(0)) / ro - 1
        fx = _zouhe_solve(case, fx, -1, np.full(ux.shape, ro), ux, 0.0, 0.0)
        f[:, :, :, nx - 1] = np.where(fluid[:, :, nx - 1][None], fx, f[:, :, :, nx - 1])
    elif int(case.outlet) == 1:
        fx = f[:, :, :, nx - 1]
        ro = case.rho_out
        zero = C[:, 0] == 0
        pos = C[:, 0] == 1
        ux = (fx[zero].sum(0) + 2 * fx[pos].sum(0)) / ro - 1
        ny_ = 0.5 * (fx[zero] * C[zero, 1][:, None, None]).sum(0)
        nz_ = 0.5 * (fx[zero] * C[zero, 2][:, None, None]).sum(0)
        fx[2] = fx[1] - ro * ux / 3
        fx[8] = fx[7] - ro * ux / 6 + ny_
        fx[10] = fx[9] - ro * ux / 6 - ny_
        fx[12] = fx[11] - ro * ux / 6 + nz_
        fx[14] = fx[13] - ro * ux / 6 - nz_
        m = fluid[:, :, nx - 1]
        f[:, :, :, nx - 1] = np.where(m[None], fx, f[:, :, :, nx - 1])

    rp = case.rheology
    po = case.porous
    g = np.array(po["g"], dtype=np.float64)
    sumf = f.sum(0)
    sumf = np.where(fluid, sumf, 1.0)
    rho = sumf / phi
    mom = np.einsum("iz...,ia->az...", f, C.astype(np.float64))
    v = mom / (phi * rho)[None] + g[:, None, None, None] / (2 * phi)[None]
    invk = po["kc"] * (1 - phi) ** 2 / (po["d"] ** 2 * phi ** 3)
    cf = 1.75 / np.sqrt(150 * phi ** 3) if po.get("forchheimer", 0) else np.zeros_like(phi)
    c0 = 0.5 + phi * po["nu_d"] * invk / 4
    c1 = phi ** 2 * cf * np.sqrt(invk) / 2
    vn = np.sqrt((v ** 2).sum(0))
    an = po.get("aniso")
    if an is None:
        u = v / (c0 + np.sqrt(c0 ** 2 + c1 * vn))[None]
        un = np.sqrt((u ** 2).sum(0))
        F = rho[None] * (g[:, None, None, None] - (phi ** 2 * po["nu_d"] * invk)[None] * u
                         - (phi ** 3 * cf * np.sqrt(invk) * un)[None] * u)
    else:
        # anisotropic permeability K = k M: the Remark's fixed point, batched
        M = np.array([[an[0], an[3], an[4]], [an[3], an[1], an[5]], [an[4], an[5], an[2]]], dtype=np.float64)
        lam, V = np.linalg.eigh(M)
        Kinv = invk[..., None, None] * np.linalg.inv(M)
        Khalf = np.sqrt(invk)[..., None, None] * (V @ np.diag(lam ** -0.5) @ V.T)
        A = np.eye(3) + (0.5 * phi * po["nu_d"])[..., None, None] * Kinv
        B = (0.5 * phi ** 2 * cf)[..., None, None] * Khalf
        vl = np.moveaxis(v, 0, -1)
        ul = vl.copy()
        for _ in range(int(po.get("aniso_iters", 8))):
            X = A + np.linalg.norm(ul, axis=-1)[..., None, None] * B
            ul = np.linalg.solve(X, vl[..., None])[..., 0]
        u = np.moveaxis(ul, -1, 0)
        un = np.sqrt((u ** 2).sum(0))
        kd = np.moveaxis(np.einsum("...ab,...b->...a", Kinv, ul), -1, 0)
        kf = np.moveaxis(np.einsum("...ab,...b->...a", Khalf, ul), -1, 0)
        F = rho[None] * (g[:, None, None, None] - (phi ** 2 * po["nu_d"])[None] * kd
                         - (phi ** 3 * cf * un)[None] * kf)
    cu = np.einsum("ia,az...->iz...", C.astype(np.float64), u)
    uu = (u ** 2).sum(0)
    feq = W[:, None, None, None] * (phi * rho)[None] * (1 + cu / CS2 + cu ** 2 / (2 * CS2 ** 2) - uu[None] / (2 * CS2))
    neq = f - feq
    Pi = np.zeros((3, 3) + fluid.shape)
    for a in range(3):
        for b in range(3):
            Pi[a, b] = (neq * (C[:, a] * C[:, b])[:, None, None, None]).sum(0) + 0.5 * (F[a] * u[b] + u[a] * F[b])
    pn = np.sqrt((Pi ** 2).sum((0, 1)))
    shear = omega_prev * pn / (CS2 * rho)
    lam_s = rp["lam"] * shear
    nu = rp["nu_inf"] + (rp["nu0"] - rp["nu_inf"]) * (1 + np.where(lam_s > 0, lam_s, 0.0) ** rp["a"]) ** ((rp["n"] - 1) / rp["a"])
    omega = 2 * rho * CS2 / (2 * nu + rho * CS2)
    phi_t = np.empty((Q,) + fluid.shape)
    for i in range(Q):
        # porosity at x + c_i, or phi(x) across walls and open faces
        nb = _shift(phi, -C[i], case.periodic, 0.0)
        phi_t[i] = np.where(kinds[i] == 0, nb, phi)
    guo = np.zeros_like(f)
    for i in range(Q):
        s = np.zeros(fluid.shape)
        for a in range(3):
            s += ((C[i, a] - u[a]) / CS2 + cu[i] * C[i, a] / CS2 ** 2) * F[a]
        guo[i] = W[i] * (1 - omega / 2) * s
    q = f + W[:, None, None, None] * rho[None] * (phi_t - phi[None]) + guo - omega[None] * neq
    q = np.where(fluid[None], q, 0.0)
    # push streaming with halfway bounce-back; open-face links are dropped
    fn = np.zeros_like(f)
    for i in range(Q):
        moved = _shift(np.where(kinds[i] == 0, q[i], 0.0), C[i], case.periodic, 0.0)
        fn[i] += moved
        fn[OPP[i]] += np.where(kinds[i] == 1, q[i], 0.0)
    if int(case.outlet) == 2:
        # extrapolation outflow: each unknown population (c_x = -1) of an
        # outflow cell is advected out at the speed of sound, upwind in x:
        # next = (1 - c_s) * (its value now) + c_s * (value now one cell
        # upstream, or its own value if that cell is solid)
        cs = np.sqrt(CS2)
        for i in np.flatnonzero(C[:, 0] == -1):
            own = f[i, :, :, nx - 1]
            up = np.where(fluid[:, :, nx - 2], f[i, :, :, nx - 2], own)
            unk = fluid[:, :, nx - 1] & (kinds[OPP[i]][:, :, nx - 1] == 2)
            fn[i, :, :, nx - 1] = np.where(unk, (1 - cs) * own + cs * up, fn[i, :, :, nx - 1])
    fn = np.where(fluid[None], fn, 0.0)
    fields = dict(rho=rho, u=u, shear=shear, omega=omega, Pi=Pi)
    return fn, np.where(fluid, omega, 0.0), fields
