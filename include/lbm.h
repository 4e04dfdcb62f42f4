/*
 * lbm.h -- C ABI of liblbm.so: the D3Q19 lattice Boltzmann step for the
 * volume-averaged Navier-Stokes equations (VANSE) with Carreau-Yasuda blood
 * rheology and a coil modelled as a porous medium, on one AMD Instinct GPU.
 *
 * What the library computes is defined by the paper (Horvat, Lunowa, Sytnyk,
 * Wohlmuth, "A Lattice Boltzmann Method for Non-Newtonian Blood Flow in Coiled
 * Intracranial Aneurysms", arXiv:2402.10809):
 *   - the model: VANSE mass and momentum, porosity phi in (0, 1], shear-strain
 *     rate with the Frobenius norm, Carreau-Yasuda viscosity (eq. carreau),
 *     Darcy/Forchheimer drag with the Kozeny-Carman permeability (section
 *     "Volume-Averaged Navier-Stokes Equations for Blood Flow");
 *   - the step: porosity-weighted moments, explicit velocity with C0 and C1,
 *     collide-and-stream with the porosity-jump, Guo-forcing and BGK terms,
 *     relaxation rate from the viscosity, semi-explicit shear rate from the
 *     corrected second moment Pi, deviatoric stress (section "Lattice
 *     Boltzmann Method for Volume-Averaged Navier-Stokes");
 *   - the boundaries: halfway bounce-back walls, Zou-He velocity inflow with a
 *     Hagen-Poiseuille profile, extrapolation outflow, pre-run ramp (section
 *     "Numerical Simulations in a Realistic Aneurysm", boundary-condition
 *     paragraph and the paragraph after the parameter table).
 * The library uses the D3Q19 velocity set and a Kozeny-Carman constant that is
 * a parameter; the outflow is the paper's extrapolation or a constant-density
 * (Zou-He pressure) outflow, the inflow amplitude a sine or a sampled waveform
 * with an optional linear pre-run ramp; all quantities are in lattice units
 * (dx = dt = 1, c_s^2 = 1/3, reference density 1).
 *
 * Conventions
 *   - Box of nx*ny*nz voxels; box index b = x + nx*(y + ny*z) (x fastest).
 *   - Fluid cells are the non-solid voxels, numbered in ascending box index;
 *     "per fluid cell" arrays use that order (lbm_fluid_index gives it).
 *   - D3Q19 directions in the order: rest; +x, -x, +y, -y, +z, -z;
 *     (+1,+1,0), (-1,-1,0), (+1,-1,0), (-1,+1,0); (+1,0,+1), (-1,0,-1),
 *     (+1,0,-1), (-1,0,+1); (0,+1,+1), (0,-1,-1), (0,+1,-1), (0,-1,+1).
 *     D3Q27 continues with the corners (+1,+1,+1), (-1,-1,-1), (+1,+1,-1),
 *     (-1,-1,+1), (+1,-1,+1), (-1,+1,-1), (-1,+1,+1), (+1,-1,-1).  Arrays
 *     "[19]" below hold 27 entries on D3Q27.  On D3Q27 the storage unit U is
 *     216 (216 * 2^9 for FP16) and the Zou-He faces use a weight-proportional
 *     transverse correction that reduces to the D3Q19 closure.
 *   - "Host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory (e.g. a torch tensor's data_ptr()).
 *
 * Ownership
 *   - Host inputs are read during the call only (copied as needed).
 *   - The library never allocates device memory.  The caller supplies one
 *     device workspace of lbm_workspace_size() bytes (256-byte aligned) that
 *     must outlive the context, and owns every device output buffer.
 *   - All device work is enqueued on the HIP stream given to lbm_create.
 *     Calls that return host data synchronise that stream.
 *   - A context is not thread-safe; distinct contexts are independent.
 *
 * Errors
 *   - Every call returns an lbm_status; nothing is thrown across the ABI.
 *   - LBM_E_INVALID: bad arguments, detected before any device work.
 *   - LBM_E_DEVICE: a HIP call failed; the context is poisoned and every later
 *     call on it returns LBM_E_STATE.
 *   - LBM_E_UNSTABLE: a non-finite value, or a speed above 0.3 c_s, was seen at
 *     a diagnostics check; the state is kept.
 *   - lbm_last_error() returns a thread-local message for the last failure.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
  LBM_OK = 0,
  LBM_E_INVALID = 1,
  LBM_E_DEVICE = 2,
  LBM_E_UNSTABLE = 3,
  LBM_E_STATE = 4,
  LBM_E_WORKSPACE = 5
} lbm_status;

/* Storage precision of the populations.  What is stored is U times the
 * deviation of each population from a rest value (see shift_mode), with
 * U = 36 (so that U w_i is an exact integer for every direction) and an extra
 * factor 2^10 for FP16 (keeps typical deviations in the normal range).  FP16
 * and BF16 round as lbm_grid.rounding says. */
typedef enum { LBM_STORE_FP32 = 0, LBM_STORE_FP16 = 1, LBM_STORE_BF16 = 2 } lbm_storage;

/* Rounding of FP16/BF16 storage (FP32 storage ignores the field).
 *   STOCHASTIC (default): every value rounds up or down at random with the
 *     probabilities that make its expected value exact (MI355X's
 *     stochastic-rounding conversion; the random bits come from a
 *     counter-based hash of the cell and the step, so a run is reproducible).
 *   CONSERVE: each cell's outputs round to nearest even, except that the
 *     rounding residuals of the non-axis values' mass and momentum move onto
 *     the axis pairs before those round, and the whole mass residual onto the
 *     rest value, rounded last: the cell's stored mass and momentum each carry
 *     one rounding.
 *   NEAREST: every value rounds to nearest even on its own.
 * Deterministic rounding of a smooth, nearly periodic flow repeats the same
 * error at the same place every step, a steady forcing that slowly damped
 * modes integrate (next to a constant-density outflow a plane-by-plane
 * alternating velocity grows to ~1e-3 of the flow in 20 000 steps); with
 * stochastic rounding the errors have mean zero.  Measured on the 192x128x128
 * aneurysm after 20 000 steps, FP16 velocity relative L2 error: stochastic
 * 2.6e-4, conserving 1.1e-3, nearest 2.4e-3. */
typedef enum { LBM_ROUND_STOCHASTIC = 0, LBM_ROUND_CONSERVE = 1, LBM_ROUND_NEAREST = 2 } lbm_rounding;

/* Arithmetic of the moments, velocity, force and collision (the shear rate and
 * the Carreau-Yasuda law are FP32 except in FP64 mode).  FP32 rounding of the per-cell
 * scalars (velocity, relaxation rate) is common to all 19 directions and acts
 * as a small persistent momentum source; in slowly evolving flows it
 * accumulates to ~1e-5 of the velocity.  AUTO with FP32 storage therefore
 * computes in FP32 and then projects each cell's output onto the intended
 * momentum, evaluated in FP64 on the FP32 values (exact conservation up to the
 * final rounding of each stored value).  FP32 = plain FP32, FP64 = the whole
 * collision in FP64 (FP32 storage only).  Reduced-precision storage is limited
 * by its own rounding and computes in plain FP32. */
typedef enum { LBM_ARITH_AUTO = 0, LBM_ARITH_FP32 = 1, LBM_ARITH_FP64 = 2 } lbm_arith;

typedef struct {
  int nx, ny, nz;      /* box size; nx <= 2048, ny <= 1024, nz <= 1024 */
  int periodic[3];     /* 1: axis wraps around; 0: faces are walls (or open, see lbm_open) */
  int storage;         /* lbm_storage */
  int shift_mode;      /* 0: stored value f_i - w_i phi(consumer cell) (default)
                          1: stored value f_i - w_i */
  int arith;           /* lbm_arith: AUTO = projected FP32 with FP32 storage, FP32 with
                          FP16/BF16 storage; FP64 is only available with FP32 storage */
  int velocity_set;    /* 19 (or 0): D3Q19; 27: D3Q27, the method section's lattice (weights
                          8/27, 2/27, 1/54, 1/216; no adjoint, no anisotropic permeability) */
  int rounding;        /* lbm_rounding of FP16/BF16 storage (0: stochastic, the default) */
} lbm_grid;

/* Carreau-Yasuda law (eq. carreau) in kinematic lattice units:
 *   nu(g) = nu_inf + (nu0 - nu_inf) (1 + (lambda g)^a)^((n-1)/a);
 * dynamic viscosity mu = nu (reference density 1); relaxation rate
 *   omega = 2 rho c_s^2 / (2 mu + rho c_s^2) with the local density rho.
 * n = 1 or lambda = 0 gives a Newtonian fluid with nu0. */
typedef struct { double nu0, nu_inf, lambda, n, a; } lbm_rheology;

/* Porous medium (model section):  1/k = kc (1-phi)^2 / (d^2 phi^3)  (finite,
 * and 0 at phi = 1);  Darcy drag -phi^2 nu_darcy u / k;  Forchheimer drag
 * -phi^3 C_F |u| u / sqrt(k) with C_F = 1.75/sqrt(150 phi^3) when
 * forchheimer = 1, else 0;  g: body force per unit mass, added to the drag.
 * Anisotropic permeability (the method section's Remark): if aniso (the
 * symmetric shape M, order xx yy zz xy xz yz) is not all zero, K = k(phi) M,
 * the drag is -phi^2 nu_darcy K^-1 u - phi^3 C_F |u| K^-1/2 u, and the
 * velocity is the Remark's fixed-point iteration u_{m+1} = (A + |u_m| B)^-1 v,
 * A = Id + (phi nu_darcy / 2) K^-1, B = (phi^2 C_F / 2) K^-1/2, from u_0 = v,
 * exactly aniso_iters times (1..64; one suffices without Forchheimer drag).
 * M must be positive definite.  Fields after g may be left zero. */
typedef struct {
  double nu_darcy, d, kc;
  int forchheimer;
  double g[3];
  double aniso[6];
  int aniso_iters;
} lbm_porous;

/* Open faces.  inlet: the x = 0 face is a Zou-He velocity inflow with
 * u = (A(t) * shape_yz[y + ny*z], 0, 0), t the step index; shape_yz is host
 * memory (ny*nz floats), e.g. the normalised Hagen-Poiseuille profile
 * 1 - r^2/R^2 of the paper's inflow (simulation section).  The waveform W(s)
 * is a0 (1 + a1 sin(2 pi s / period)), or, when wave_table is set, the
 * table_len samples (host, FP64, 1 <= table_len <= 1024) of one period of
 * `period` steps, sample k at s = k period / table_len, interpolated linearly
 * and repeated periodically (a sampled waveform such as a 1D-0D network
 * model's mean inflow velocity).  ramp_steps = R > 0 adds the paper's pre-run:
 * A(t) = (t / R) W(0) for t < R, then A(t) = W(t - R); R = 0: A(t) = W(t).
 * outlet (x = nx-1 face): 0 none (wall); LBM_OUTLET_DENSITY, a Zou-He
 * constant-density outflow with density rho_out and zero tangential velocity;
 * LBM_OUTLET_EXTRAPOLATION, the non-reflecting extrapolation outflow the
 * paper's boundary-condition paragraph uses (after Geier et al.): each unknown
 * population i (c_x = -1) is carried out at the speed of sound, upwind in x,
 *   f_i(t+1, x) = (1 - c_s) f_i(t, x) + c_s f_i(t, x - e_x),
 * with pre-collision values (f_i(t, x) alone where x - e_x is solid); these
 * unknowns are then part of the state (see lbm_get_state), and rho_out is
 * unused.  Fluid cells on an open face must have phi = 1.  Fluid cells on
 * other non-periodic faces see the outside as wall.  Fields after rho_out may
 * be left zero. */
enum { LBM_OUTLET_NONE = 0, LBM_OUTLET_DENSITY = 1, LBM_OUTLET_EXTRAPOLATION = 2 };
typedef struct {
  int inlet;
  const float* shape_yz;
  double a0, a1, period;
  int outlet;
  double rho_out;
  int ramp_steps;
  const double* wave_table;
  int table_len;
} lbm_open;

/* Objective for lbm_adjoint: J = (1/(t_end - t_begin)) sum_{t=t_begin}^{t_end-1} e(t),
 * evaluated from the pre-collision state of step t (the region is given to
 * lbm_create):
 *   kind LBM_OBJ_KINETIC: e(t) = mean over the region cells of (1/2) rho |u|^2;
 *   kind LBM_OBJ_WSS:     e(t) = mean over the region's wall cells of |tau|,
 *                         the wall shear stress of lbm_moments (the quantity
 *                         the paper averages over the aneurysm wall). */
enum { LBM_OBJ_KINETIC = 0, LBM_OBJ_WSS = 1 };
typedef struct {
  int t_begin, t_end;
  int kind;
  /* nonzero: the reverse sweep stores the adjoint populations in FP64 instead
   * of FP32 (152 more bytes moved per reverse cell-step; removes the FP32
   * rounding of those populations, the largest term of the gradient's error
   * budget).  Needs 19 * 8 bytes per compact cell below 2 GiB. */
  int fp64_adjoint;
} lbm_objective;

/* Diagnostics vector (lbm_diagnostics), all FP64, of the current state:
 *   [0] mass  sum_x phi rho            [1..3] momentum sum_x sum_i f_i c_i
 *   [4] kinetic energy sum_x rho|u|^2/2 [5] same over the region cells
 *   [6] max |u|   [7] min omega   [8] max omega
 *   [9] number of cells with a non-finite value   [10] step index t
 *   [11] mean wall shear stress |tau| over the region's wall cells (0 if none) */
#define LBM_NDIAG 12

/* Bytes of device workspace a context needs.  adjoint_T > 0 adds room for an
 * lbm_adjoint run of adjoint_T steps with checkpoints every ckpt_every steps.
 * solid: host, nx*ny*nz bytes, nonzero = solid. */
lbm_status lbm_workspace_size(const lbm_grid* grid, const uint8_t* solid, int adjoint_T, int ckpt_every,
                              size_t* bytes);

/* Create a context at the rest state (rho = 1, u = 0, omega = omega(nu0)), t = 0.
 *   solid:   host, nx*ny*nz, nonzero = solid voxel
 *   phi:     host, nx*ny*nz porosity; must be in (0, 1] on fluid cells (ignored on solid)
 *   region:  host, nx*ny*nz, nonzero = objective region (e.g. the sac); may be NULL
 *   open:    may be NULL (no open faces)
 *   workspace/ws_bytes: device memory of at least lbm_workspace_size() bytes
 *   stream:  hipStream_t (NULL = default stream)
 * Errors (LBM_E_INVALID): NULL required pointers, bad sizes, phi out of range
 * on fluid, nu0 <= 0 or nu_inf <= 0, rheology a <= 0, open face on a periodic x
 * axis, phi != 1 on an open-face fluid cell, no fluid cell; LBM_E_WORKSPACE: the
 * workspace is too small or misaligned. */
lbm_status lbm_create(const lbm_grid* grid, const uint8_t* solid, const float* phi, const uint8_t* region,
                      const lbm_rheology* rheology, const lbm_porous* porous, const lbm_open* open,
                      void* workspace, size_t ws_bytes, void* stream, lbm_ctx** out);

/* Advance n time steps (collide and stream every fluid cell n times).  Every
 * 1000th step index the state is checked (see LBM_E_UNSTABLE); that check
 * synchronises the stream. */
lbm_status lbm_step(lbm_ctx* ctx, int n);

/* Macroscopic fields of the current state (what the next step's collision
 * uses): density rho, velocity u [3][nx*ny*nz], shear rate, the relaxation
 * rate omega the next collision will use, the deviatoric stress
 * sigma = (omega/2 - 1) Pi [6][nx*ny*nz] in the order xx yy zz xy xz yz, and
 * the wall shear stress tau = sigma n - (n . sigma n) n [3][nx*ny*nz]
 * (simulation section) on the voxel wall: the fluid cells with a bounce-back
 * link, whose outer normal n is the normalised sum over their wall links
 * x + c_i of w_i c_i (0 where that sum vanishes and off the wall).
 * Device outputs in box layout, 0 on solid voxels; any may be NULL. */
lbm_status lbm_moments(lbm_ctx* ctx, float* rho, float* u, float* shear, float* omega, float* sigma, float* tau);

/* FP64 diagnostics of the current state into out[LBM_NDIAG] (host); syncs. */
lbm_status lbm_diagnostics(lbm_ctx* ctx, double* out);

/* For callers that cannot allocate device memory or set aside workspace for
 * scratch (code under HIP graph capture, allocation-free serving loops):
 * lbm_diagnostics with its scratch -- the per-block partials and the reduced
 * vector -- in a fixed device array of LBM_NOALLOC_SCRATCH_BYTES that the
 * library holds on each GPU it runs on until the process ends, instead of the
 * context's workspace.  Same kernels and the same fixed reduction order, so the
 * result equals lbm_diagnostics' bit for bit.  Allocates nothing.
 * Limit: contexts of at most 3 049 472 compact cells (the partials of one
 * block per 256 cells must fit); larger ones get LBM_E_INVALID, naming the
 * bytes needed.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (other host threads, other streams) race; one call at a
 * time per GPU.  The array needs no clearing (every block writes all of its
 * partials).  Syncs the context's stream. */
#define LBM_NOALLOC_SCRATCH_BYTES (1u << 20)
lbm_status lbm_diagnostics_noalloc(lbm_ctx* ctx, double* out);

/* State transfer (host memory, per fluid cell): f[19][n_fluid] pre-collision
 * populations (unshifted, FP64), omega[n_fluid] the relaxation rate of the
 * previous step.  Populations that would arrive through an open face are
 * unknown: get writes 0 there, set ignores them; the extrapolation outflow's
 * are part of the state instead (get returns them, set uses them).  Both sync
 * the stream. */
lbm_status lbm_get_state(lbm_ctx* ctx, double* f, float* omega);
lbm_status lbm_set_state(lbm_ctx* ctx, const double* f, const float* omega);

/* Replace the porosity field and reset to the rest state at t = 0 (model
 * section: phi is the volume fraction of fluid, a per-voxel input of the
 * method; the gradient of lbm_adjoint is taken with respect to it).
 *   phi: DEVICE memory, nx*ny*nz floats in box layout (e.g. a torch tensor's
 *        data_ptr()), read during the call; values on solid voxels are
 *        ignored.
 * The rules of lbm_create apply: phi in (0, 1] on fluid cells and 1 on
 * open-face cells.  They are checked on the device before anything changes;
 * a violation returns LBM_E_INVALID naming a box index and leaves the
 * context as it was.  The porosity-dependent flags of the cells are
 * recomputed on the device; nothing passes through host memory.  Syncs the
 * stream (to read the check's result). */
lbm_status lbm_set_porosity(lbm_ctx* ctx, const float* phi);

/* Reset to the rest state at t = 0. */
lbm_status lbm_reset(lbm_ctx* ctx);

/* Gradient of the region objective (kinetic energy or wall shear stress) with
 * respect to the porosity of every fluid cell.  Resets to rest, runs T steps forward while
 * accumulating J and storing a checkpoint every ckpt_every steps, then sweeps
 * back through the segments (recompute forward, then reverse steps).  The
 * forward pass records the last segment itself, so that segment is not
 * recomputed; with ckpt_every >= T nothing is recomputed (the record of the
 * whole run, 84 bytes per fluid cell and step, must then fit the workspace).
 * J and the gradient do not depend on ckpt_every (the recompute reproduces
 * the forward trajectory bit for bit).  The forward passes compute the collision, the shear rate and the Carreau-Yasuda
 * law in FP64 (LBM_ARITH_FP64) whatever the context's arithmetic mode, and
 * store the trajectory in FP32; the reverse steps are FP64 arithmetic with
 * FP32 adjoint populations (FP64 with obj->fp64_adjoint) and an FP64
 * relaxation-rate adjoint.  Either outflow kind; with the extrapolation outflow
 * the outflow cells' unknowns are state, and their dependence on the previous
 * step's values is part of the reverse sweep.  Needs a workspace sized for
 * (T, ckpt_every) or larger; FP32 storage, shift mode 0, D3Q19 (with or
 * without Forchheimer drag, isotropic or anisotropic permeability: the
 * fixed-point iterates are differentiated as iterated), a region with a
 * fluid cell (with a wall cell for LBM_OBJ_WSS), 0 <= t_begin < t_end <= T.
 * Non-differentiable points take derivative 0: tau = 0 at a wall cell (|tau|),
 * u = 0 and v = 0 in the Forchheimer drag (|u|, |v|); at phi = 1 the
 * derivative is the one from below (phi <= 1).
 *   J:       host, 1 double
 *   dJ_dphi: device, nx*ny*nz floats (box layout, 0 off the fluid), or NULL:
 *            then only J is computed (the forward pass, no checkpoints; the
 *            workspace of lbm_create suffices)
 * Leaves the context at the rest state (t = 0); syncs the stream. */
lbm_status lbm_adjoint(lbm_ctx* ctx, const lbm_objective* obj, int T, int ckpt_every, double* J, float* dJ_dphi);

lbm_status lbm_fluid_cells(lbm_ctx* ctx, int64_t* n_fluid);
/* Box index of every fluid cell (host, n_fluid int64) in the library's order. */
lbm_status lbm_fluid_index(lbm_ctx* ctx, int64_t* box_index);
/* Current step index. */
lbm_status lbm_time(lbm_ctx* ctx, int64_t* t);

/* Measurement aid: device-to-device copy of `bytes` (multiple of 16) by a plain
 * streaming kernel on `stream`, for an achievable-bandwidth reference. */
lbm_status lbm_copy_probe(void* dst, const void* src, size_t bytes, void* stream);

/* Measurement aid: achievable-bandwidth references on `stream`, over `bytes`
 * (a positive multiple of 16) of device memory.
 *   LBM_PROBE_COPY:    the plain copy of lbm_copy_probe (dst <- src);
 *   LBM_PROBE_COPY_NT: copy with four 16-byte vectors in flight per work-item
 *                      and non-temporal loads and stores;
 *   LBM_PROBE_READ:    reads src only (four vectors in flight, non-temporal);
 *                      writes one 4-byte word per work-item to dst, which
 *                      must hold LBM_PROBE_BLOCKS * 256 words;
 *   LBM_PROBE_WRITE:   writes dst only (src unused, may be NULL).
 * The grid is LBM_PROBE_BLOCKS workgroups of 256 work-items (grid-stride). */
enum { LBM_PROBE_COPY = 0, LBM_PROBE_COPY_NT = 1, LBM_PROBE_READ = 2, LBM_PROBE_WRITE = 3 };
#define LBM_PROBE_BLOCKS 8192
lbm_status lbm_bandwidth_probe(int kind, void* dst, const void* src, size_t bytes, void* stream);

const char* lbm_last_error(void);
void lbm_destroy(lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
