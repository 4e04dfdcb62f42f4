// Host runtime of liblbm.so: the C ABI declared in include/lbm.h.
//
// The library never allocates device memory: the caller's workspace is carved
// into the population buffer (one, streamed in place), the per-cell arrays of
// the compact row layout (position code, link word, porosity, relaxation rate),
// the per-row tables (neighbour-row deltas, inflow profile, box offset), plus
// the adjoint's checkpoints and records when asked for.  Every kernel runs on
// the context's stream.
#include "lbm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "runtime.hpp"

using namespace lbm;

namespace {
thread_local std::string g_err;
}  // namespace

namespace lbmrt {

lbm_status fail(lbm_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

}  // namespace lbmrt

using namespace lbmrt;

namespace {

constexpr int CHECK_EVERY = 1000;                       // steps between stability checks
constexpr double MAX_SPEED = 0.3 / 1.7320508075688772;  // 0.3 c_s

// Storage unit U: stored value = U (f - rest).  36 w_i is an integer; FP16 adds
// 2^10 so that typical deviations sit in the normal range.
// (2^9 on D3Q27, whose rest weight is larger relative to U.)
double storage_unit(int storage, int q) {
  if (q == 27) return storage == LBM_STORE_FP16 ? 216.0 * 512.0 : 216.0;
  return storage == LBM_STORE_FP16 ? 36.0 * 1024.0 : 36.0;
}
// Symmetric 3x3 matrices as full arrays: inverse by the adjugate.
using M3 = std::array<std::array<double, 3>, 3>;
bool inv3(const M3& a, M3& r) {
  const double c00 = a[1][1] * a[2][2] - a[1][2] * a[2][1], c01 = a[1][2] * a[2][0] - a[1][0] * a[2][2],
               c02 = a[1][0] * a[2][1] - a[1][1] * a[2][0];
  const double det = a[0][0] * c00 + a[0][1] * c01 + a[0][2] * c02;
  if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return false;
  const double id = 1.0 / det;
  r[0][0] = c00 * id; r[1][0] = c01 * id; r[2][0] = c02 * id;
  r[0][1] = (a[0][2] * a[2][1] - a[0][1] * a[2][2]) * id;
  r[1][1] = (a[0][0] * a[2][2] - a[0][2] * a[2][0]) * id;
  r[2][1] = (a[0][1] * a[2][0] - a[0][0] * a[2][1]) * id;
  r[0][2] = (a[0][1] * a[1][2] - a[0][2] * a[1][1]) * id;
  r[1][2] = (a[0][2] * a[1][0] - a[0][0] * a[1][2]) * id;
  r[2][2] = (a[0][0] * a[1][1] - a[0][1] * a[1][0]) * id;
  return true;
}

// Anisotropic permeability shape M (xx yy zz xy xz yz): checks positive
// definiteness (leading minors) and returns M^-1 and M^-1/2, the latter by the
// Denman-Beavers iteration Y <- (Y + Z^-1)/2, Z <- (Z + Y^-1)/2 from Y = M,
// Z = Id, whose Z converges quadratically to M^-1/2.
bool aniso_shape(const double m6[6], double inv6[6], double ihalf6[6]) {
  const M3 M = {{{m6[0], m6[3], m6[4]}, {m6[3], m6[1], m6[5]}, {m6[4], m6[5], m6[2]}}};
  const double d1 = M[0][0], d2 = M[0][0] * M[1][1] - M[0][1] * M[0][1];
  const double d3 = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[1][2]) -
                    M[0][1] * (M[0][1] * M[2][2] - M[1][2] * M[0][2]) + M[0][2] * (M[0][1] * M[1][2] - M[1][1] * M[0][2]);
  if (!(d1 > 0.0 && d2 > 0.0 && d3 > 0.0)) return false;
  M3 Mi, Y = M, Z = {{{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}};
  if (!inv3(M, Mi)) return false;
  for (int it = 0; it < 100; ++it) {
    M3 Yi, Zi;
    if (!inv3(Y, Yi) || !inv3(Z, Zi)) return false;
    double ch = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double yn = 0.5 * (Y[i][j] + Zi[i][j]), zn = 0.5 * (Z[i][j] + Yi[i][j]);
        ch = std::max(ch, std::fabs(zn - Z[i][j]));
        Y[i][j] = yn;
        Z[i][j] = zn;
      }
    if (ch < 1e-15 * (1.0 + std::fabs(Z[0][0]) + std::fabs(Z[1][1]) + std::fabs(Z[2][2]))) break;
  }
  const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
  for (int k = 0; k < 6; ++k) {
    inv6[k] = 0.5 * (Mi[ia[k]][ib[k]] + Mi[ib[k]][ia[k]]);
    ihalf6[k] = 0.5 * (Z[ia[k]][ib[k]] + Z[ib[k]][ia[k]]);
  }
  return true;
}

}  // namespace

namespace lbmrt {

Layout make_layout(const lbm_grid& g, int64_t nc, int64_t nrow, int T, int ckpt) {
  Layout L{};
  const size_t ss = store_bytes(g.storage);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
  const int q = qof(g);
  L.A = take((size_t)q * (size_t)plane_cells(nc) * ss);
  L.code = take((size_t)nc * 4);
  L.links = take((size_t)nc * (q == 27 ? 8 : 4));
  L.phi = take((size_t)nc * 4);
  L.omega = take((size_t)nc * 4);
  L.delta = take((size_t)nrow * 8 * 4);
  L.rel = take((size_t)nrow * 8 * 4);
  L.winfo = take((size_t)wave_records(nc) * sizeof(lbm::WaveInfo));
  L.shape = take((size_t)nrow * 4);
  L.rowbox = take((size_t)nrow * 4);
  L.stage = take((size_t)(q + 1) * nc * 4);
  const size_t nbmax = (size_t)blocks_for_nt(nc, STEP_NT_MIN);  // most blocks any launch uses
  L.part = take(nbmax * NDIAGP * 8);
  L.diag = take(64 * 8);
  L.obj = take(nbmax * 8);
  L.tc = take(2 * sizeof(uint32_t));
  L.wave = take(MAX_WAVE_TABLE * sizeof(double));
  L.side = take((size_t)2 * nrow * (q == 27 ? 18 : 10) * sizeof(float));
  L.T = T;
  L.ckpt = ckpt;
  if (T > 0) {
    L.nck = (T + ckpt - 1) / ckpt;
    L.ck = take((size_t)L.nck * (Q + 1) * nc * 4);
    L.rec = take((size_t)(ckpt + 1) * (Q + 1) * nc * 4);
    L.rho = take((size_t)(ckpt + 1) * nc * 4);
    L.ah0 = take(Q * (size_t)nc * 8);  // adjoint populations: room for FP64
    L.ah1 = take(Q * (size_t)nc * 8);
    L.omh = take((size_t)nc * 8);
    L.phih = take((size_t)nc * 8);
    L.aside = take((size_t)2 * nrow * 5 * 8);
  }
  L.total = o;
  return L;
}

Bufs bufs(lbm_ctx* c) {
  Bufs b{};
  b.A = c->ws + c->L.A;
  b.code = (const uint32_t*)(c->ws + c->L.code);
  b.links = (const uint32_t*)(c->ws + c->L.links);
  b.delta = (const int*)(c->ws + c->L.delta);
  b.rel = (const int*)(c->ws + c->L.rel);
  b.winfo = (const WaveInfo*)(c->ws + c->L.winfo);
  b.phi = (const float*)(c->ws + c->L.phi);
  b.omega = (float*)(c->ws + c->L.omega);
  b.shape = (const float*)(c->ws + c->L.shape);
  b.rowbox = (const uint32_t*)(c->ws + c->L.rowbox);
  b.part = (double*)(c->ws + c->L.part);
  b.rec = nullptr;
  b.rho_rec = nullptr;
  b.tc = (uint32_t*)(c->ws + c->L.tc);
  b.wave = (const double*)(c->ws + c->L.wave);
  b.side = (float*)(c->ws + c->L.side);
  return b;
}


q27::Bufs27 bufs27(lbm_ctx* c) {
  q27::Bufs27 b{};
  b.A = c->ws + c->L.A;
  b.code = (const uint32_t*)(c->ws + c->L.code);
  b.links = (const uint64_t*)(c->ws + c->L.links);
  b.delta = (const int*)(c->ws + c->L.delta);
  b.phi = (const float*)(c->ws + c->L.phi);
  b.omega = (float*)(c->ws + c->L.omega);
  b.shape = (const float*)(c->ws + c->L.shape);
  b.rowbox = (const uint32_t*)(c->ws + c->L.rowbox);
  b.part = (double*)(c->ws + c->L.part);
  b.tc = (uint32_t*)(c->ws + c->L.tc);
  b.wave = (const double*)(c->ws + c->L.wave);
  b.side = (float*)(c->ws + c->L.side);
  return b;
}

}  // namespace lbmrt

namespace {

lbm_status validate_grid(const lbm_grid* g) {
  if (!g) return fail(LBM_E_INVALID, "grid is NULL");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(LBM_E_INVALID, "grid dimensions must be positive");
  if (g->nx > 2048 || g->ny > 1024 || g->nz > 1024) return fail(LBM_E_INVALID, "grid exceeds 2048 x 1024 x 1024");
  if (g->storage < 0 || g->storage > 2) return fail(LBM_E_INVALID, "unknown storage format");
  if (g->shift_mode < 0 || g->shift_mode > 1) return fail(LBM_E_INVALID, "shift_mode must be 0 or 1");
  if (g->rounding < LBM_ROUND_STOCHASTIC || g->rounding > LBM_ROUND_NEAREST)
    return fail(LBM_E_INVALID, "rounding must be one of the lbm_rounding values");
  if (g->arith < 0 || g->arith > 2) return fail(LBM_E_INVALID, "unknown arithmetic mode");
  if (g->arith == LBM_ARITH_FP64 && g->storage != LBM_STORE_FP32)
    return fail(LBM_E_INVALID, "FP64 arithmetic is only available with FP32 storage");
  if (g->velocity_set != 0 && g->velocity_set != 19 && g->velocity_set != 27)
    return fail(LBM_E_INVALID, "velocity_set must be 19 or 27");
  return LBM_OK;
}

// Limits of the compact layout for a given mask: 32-bit byte offsets into the
// population planes (also the FP32 adjoint planes) and the position code.
lbm_status check_rows(const lbm_grid* g, const Rows& r) {
  if (r.nf == 0) return fail(LBM_E_INVALID, "no fluid cell");
  if ((double)plane_cells(r.nc) * qof(*g) * 4.0 >= 4294967296.0)
    return fail(LBM_E_INVALID, std::string("more than ") + (qof(*g) == 27 ? "39.7" : "56.5") +
                                   " M compact cells (kernels address the population planes with 32-bit byte "
                                   "offsets)");
  const int xb = xbits_for(g->nx);
  if ((uint64_t)r.y.size() >= ((uint64_t)1 << (32 - xb)))
    return fail(LBM_E_INVALID, "too many fluid rows for the 32-bit position code");
  return LBM_OK;
}

lbm_status check_phi(const lbm_ctx* c, const float* phi) {
  for (size_t k = 0; k < c->fluid_box.size(); ++k) {
    const float v = phi[c->fluid_box[k]];
    if (!(v > 0.0f && v <= 1.0f))
      return fail(LBM_E_INVALID, "porosity must lie in (0, 1] on every fluid cell (box index " +
                                     std::to_string(c->fluid_box[k]) + ")");
    if (c->openface[k] && v != 1.0f)
      return fail(LBM_E_INVALID, "porosity must be 1 on open-face cells (box index " +
                                     std::to_string(c->fluid_box[k]) + ")");
  }
  return LBM_OK;
}

// Upload the porosity and the link words (which depend on it).
lbm_status upload_phi(lbm_ctx* c, const float* phi) {
  std::vector<float> box(c->nbox, 0.0f), comp(c->nc, 0.0f);
  c->phi_f.resize(c->nf);
  for (int64_t k = 0; k < c->nf; ++k) {
    const float v = phi[c->fluid_box[k]];
    box[c->fluid_box[k]] = v;
    comp[c->fluid_c[k]] = v;
    c->phi_f[k] = v;
  }
  std::vector<uint32_t> links;
  std::vector<uint64_t> links64;
  if (c->q == 27) c->nwss = build_links27(*c, box, links64);
  else c->nwss = build_links(*c, box, links);
  HIP_TRY(c, hipMemcpyAsync(c->ws + c->L.phi, comp.data(), comp.size() * 4, hipMemcpyHostToDevice, c->stream));
  if (c->q == 27)
    HIP_TRY(c, hipMemcpyAsync(c->ws + c->L.links, links64.data(), links64.size() * 8, hipMemcpyHostToDevice,
                              c->stream));
  else
    HIP_TRY(c, hipMemcpyAsync(c->ws + c->L.links, links.data(), links.size() * 4, hipMemcpyHostToDevice, c->stream));
  lbm_status s = launch_wave_info(c);
  if (s != LBM_OK) return s;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

}  // namespace

namespace lbmrt {

lbm_status launch_init(lbm_ctx* c) {
  with_storage(c->grid.storage, [&](auto tag) {
    using S = typename decltype(tag)::T;
    if (c->q == 27) init27<S>(c, bufs27(c));
    else init19<S>(c, bufs(c));
  });
  HIP_TRY(c, hipGetLastError());
  // extrapolation outflow: the kept values of the rest state (phi = 1 on the
  // outflow cells, so w_i, i.e. deviation 0; the -x neighbour's values are
  // those the rest state's outflow populations extrapolate from)
  HIP_TRY(c, hipMemsetAsync(c->ws + c->L.side, 0, (size_t)2 * c->nrow * (c->q == 27 ? 18 : 10) * sizeof(float),
                            c->stream));
  c->t = 0;
  return LBM_OK;
}

// One step at time t (in place).  diag: 0 none, 1 diagnostics partials, 2
// region kinetic energy, 3 region wall shear stress, accumulated into the
// objective partials.  rec: record the step for the adjoint (FP32, shift
// mode 0 only).
lbm_status launch_step(lbm_ctx* c, int diag, float* rec, float* rho_rec) {
  if (c->q == 27) {
    const q27::Bufs27 b = bufs27(c);
    with_storage(c->grid.storage, [&](auto tag) { step27<typename decltype(tag)::T>(c, b, diag); });
  } else {
    Bufs b = bufs(c);
    if (diag >= 2) b.part = (double*)(c->ws + c->L.obj);
    if (rec) {
      b.rec = rec;
      b.rho_rec = rho_rec;
    }
    with_storage(c->grid.storage, [&](auto tag) { step19<typename decltype(tag)::T>(c, b, diag, rec != nullptr); });
  }
  HIP_TRY(c, hipGetLastError());
  c->t += 1;
  return LBM_OK;
}

lbm_status finalize(lbm_ctx* c, const double* part, int nparts, int n, uint32_t ops, double* host_out,
                    double* dev_out) {
  double* dout = dev_out ? dev_out : (double*)(c->ws + c->L.diag);
  launch_finalize(c->stream, part, nparts, n, ops, dout);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipMemcpyAsync(host_out, dout, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

// Pulled state of time t (raw stored values as FP32, [19][nc], compact order)
// into dst (device).
lbm_status gather_state(lbm_ctx* c, float* dst) {
  with_storage(c->grid.storage, [&](auto tag) {
    using S = typename decltype(tag)::T;
    if (c->q == 27) gather27<S>(c, bufs27(c), dst);
    else gather19<S>(c, bufs(c), dst);
  });
  HIP_TRY(c, hipGetLastError());
  return LBM_OK;
}

// Inverse of gather_state, into the slots of time t's parity.
lbm_status scatter_state(lbm_ctx* c, const float* src) {
  with_storage(c->grid.storage, [&](auto tag) {
    using S = typename decltype(tag)::T;
    if (c->q == 27) scatter27<S>(c, bufs27(c), src);
    else scatter19<S>(c, bufs(c), src);
  });
  HIP_TRY(c, hipGetLastError());
  return LBM_OK;
}

}  // namespace lbmrt

namespace {

const uint32_t DIAG_OPS = (1u << 12) | (2u << 14) | (1u << 16);  // max |u|, min omega, max omega; rest sums

// Fixed device scratch of lbm_diagnostics_noalloc: the per-block partials and
// the reduced vector.  Each GPU the library runs on holds its own copy for the
// life of the process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (kept per device below).
constexpr size_t STATIC_SCRATCH_BYTES = size_t(1) << 20;
constexpr int MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void* g_scratch_dev[MAX_DEVICES] = {};

// Largest compact-cell count whose partials fit the static scratch.
size_t noalloc_need(int64_t nblk) { return align_up((size_t)nblk * NDIAGP * sizeof(double)) + NDIAGP * sizeof(double); }
int64_t max_noalloc_cells() {
  int64_t nb = (int64_t)(STATIC_SCRATCH_BYTES / (NDIAGP * sizeof(double)));
  while (nb > 0 && noalloc_need(nb) > STATIC_SCRATCH_BYTES) --nb;
  return nb * BLOCK;
}

// The device address of `scratch` on the current device `dev`, looked up once
// per device.
lbm_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(LBM_E_DEVICE, "device index out of range for the static scratch");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(LBM_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return LBM_OK;
}

// nparts: the block count of the launch that wrote the partials
lbm_status read_diag(lbm_ctx* c, int nparts, double* out) {
  return finalize(c, (const double*)(c->ws + c->L.part), nparts, NDIAGP, DIAG_OPS, out);
}

lbm_status check_stable(lbm_ctx* c, const double* dg) {
  if (dg[9] > 0.0 || !std::isfinite(dg[0]) || !(dg[6] <= MAX_SPEED)) {
    char m[256];
    std::snprintf(m, sizeof(m), "unstable at step %lld: %g non-finite cells, max |u| = %g (limit %g)",
                  (long long)c->t, dg[9], dg[6], MAX_SPEED);
    return fail(LBM_E_UNSTABLE, m);
  }
  return LBM_OK;
}

// part: where the diagnostics partials go (nullptr: the workspace's area)
lbm_status moments_launch(lbm_ctx* c, bool diag, float* rho, float* u, float* shear, float* omega, float* sigma,
                          float* tau, double* part = nullptr) {
  with_storage(c->grid.storage, [&](auto tag) {
    using S = typename decltype(tag)::T;
    if (c->q == 27) {
      q27::Bufs27 b = bufs27(c);
      if (part) b.part = part;
      moments27<S>(c, b, diag, rho, u, shear, omega, sigma, tau);
    } else {
      Bufs b = bufs(c);
      if (part) b.part = part;
      moments19<S>(c, b, diag, rho, u, shear, omega, sigma, tau);
    }
  });
  HIP_TRY(c, hipGetLastError());
  return LBM_OK;
}

// The host copy of the porosity per fluid cell (for the state transfer's rest
// values), refreshed from the device after lbm_set_porosity.
lbm_status refresh_phi_host(lbm_ctx* c) {
  if (!c->phi_stale) return LBM_OK;
  std::vector<float> comp(c->nc);
  HIP_TRY(c, hipMemcpyAsync(comp.data(), c->ws + c->L.phi, comp.size() * 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int64_t k = 0; k < c->nf; ++k) c->phi_f[k] = comp[c->fluid_c[k]];
  c->phi_stale = false;
  return LBM_OK;
}

double rest_value(const lbm_ctx* c, int i, int64_t k) {
  const double w = c->q == 27 ? q27::kw(i) / 216.0 : (i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0));
  return w * (c->grid.shift_mode ? 1.0 : c->phi_f[k]);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* lbm_last_error(void) { return g_err.c_str(); }

lbm_status lbm_workspace_size(const lbm_grid* grid, const uint8_t* solid, int adjoint_T, int ckpt_every,
                              size_t* bytes) {
  lbm_status s = validate_grid(grid);
  if (s != LBM_OK) return s;
  if (!solid || !bytes) return fail(LBM_E_INVALID, "solid and bytes must not be NULL");
  if (adjoint_T < 0 || (adjoint_T > 0 && ckpt_every < 1)) return fail(LBM_E_INVALID, "bad adjoint_T / ckpt_every");
  const Rows r = find_rows(*grid, solid);
  s = check_rows(grid, r);
  if (s != LBM_OK) return s;
  *bytes = make_layout(*grid, r.nc, (int64_t)r.y.size(), adjoint_T, adjoint_T > 0 ? ckpt_every : 0).total;
  return LBM_OK;
}

lbm_status lbm_create(const lbm_grid* grid, const uint8_t* solid, const float* phi, const uint8_t* region,
                      const lbm_rheology* rh, const lbm_porous* po, const lbm_open* op, void* workspace,
                      size_t ws_bytes, void* stream, lbm_ctx** out) {
  if (!out) return fail(LBM_E_INVALID, "out is NULL");
  *out = nullptr;
  lbm_status s = validate_grid(grid);
  if (s != LBM_OK) return s;
  if (!solid || !phi || !rh || !po) return fail(LBM_E_INVALID, "solid, phi, rheology and porous must not be NULL");
  if (!(rh->nu0 > 0) || !(rh->nu_inf > 0)) return fail(LBM_E_INVALID, "nu0 and nu_inf must be positive");
  if (!(rh->a > 0) || !(rh->lambda >= 0) || !std::isfinite(rh->n))
    return fail(LBM_E_INVALID, "bad Carreau-Yasuda a, lambda or n");
  if (!(po->kc >= 0) || !(po->d > 0) || !(po->nu_darcy >= 0)) return fail(LBM_E_INVALID, "bad porous parameters");
  bool aniso = false;
  double an_inv[6] = {0}, an_ih[6] = {0};
  for (int k = 0; k < 6; ++k) aniso = aniso || po->aniso[k] != 0.0;
  if (aniso && grid->velocity_set == 27)
    return fail(LBM_E_INVALID, "anisotropic permeability is built for D3Q19 only");
  if (aniso) {
    if (po->aniso_iters < 1 || po->aniso_iters > 64) return fail(LBM_E_INVALID, "aniso_iters must lie in [1, 64]");
    if (!aniso_shape(po->aniso, an_inv, an_ih))
      return fail(LBM_E_INVALID, "the anisotropic permeability shape must be symmetric positive definite");
  }
  if (op && (op->inlet || op->outlet)) {
    if (grid->periodic[0]) return fail(LBM_E_INVALID, "open faces need a non-periodic x axis");
    if (op->inlet && (!op->shape_yz || !(op->period > 0)))
      return fail(LBM_E_INVALID, "inlet needs shape_yz and period > 0");
    if (op->inlet && op->ramp_steps < 0) return fail(LBM_E_INVALID, "ramp_steps must be >= 0");
    if (op->inlet && op->wave_table && (op->table_len < 1 || op->table_len > MAX_WAVE_TABLE))
      return fail(LBM_E_INVALID, "table_len must lie in [1, " + std::to_string(MAX_WAVE_TABLE) + "]");
    if (op->outlet < 0 || op->outlet > 2) return fail(LBM_E_INVALID, "outlet must be 0, 1 or 2");
    if (op->outlet == 1 && !(op->rho_out > 0)) return fail(LBM_E_INVALID, "outlet density must be positive");
  }
  if (!workspace) return fail(LBM_E_WORKSPACE, "workspace is NULL");
  if (((uintptr_t)workspace & 255) != 0) return fail(LBM_E_WORKSPACE, "workspace must be 256-byte aligned");
  Rows rows = find_rows(*grid, solid);
  s = check_rows(grid, rows);
  if (s != LBM_OK) return s;
  const int64_t nrow = (int64_t)rows.y.size();
  const Layout L0 = make_layout(*grid, rows.nc, nrow, 0, 0);
  if (ws_bytes < L0.total)
    return fail(LBM_E_WORKSPACE, "workspace too small: need " + std::to_string(L0.total) + " bytes");

  lbm_ctx* c = new lbm_ctx();
  c->grid = *grid;
  c->rh = *rh;
  c->po = *po;
  if (op) c->op = *op;
  c->op.shape_yz = nullptr;
  c->op.wave_table = nullptr;
  c->nbox = (size_t)grid->nx * grid->ny * grid->nz;
  c->stream = (hipStream_t)stream;
  c->q = qof(*grid);
  c->U = storage_unit(grid->storage, c->q);
  build_host_layout(*c, *grid, solid, region, op && op->inlet, op ? op->outlet : 0);
  const int nx = grid->nx, xb = c->xbits;
  std::vector<float> shape(nrow, 0.0f);
  if (op && op->inlet)
    for (int64_t r = 0; r < nrow; ++r) shape[r] = op->shape_yz[(size_t)c->rows.z[r] * grid->ny + c->rows.y[r]];
  s = check_phi(c, phi);
  if (s != LBM_OK) { delete c; return s; }
  {
    // the device that holds the workspace (current now), and its copy of the
    // static scratch of lbm_diagnostics_noalloc
    const hipError_t e = hipGetDevice(&c->device);
    void* sp = nullptr;
    if (e != hipSuccess) {
      delete c;
      return fail(LBM_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    s = scratch_address(c->device, &sp);
    if (s != LBM_OK) { delete c; return s; }
  }
  c->nblk = blocks_for(c->nc);
  c->sblk = blocks_for_nt(c->nc, step_nt(grid->storage));
  // populations, position code, link word, porosity and relaxation rate
  c->beyond_cache = (size_t)c->nc * ((size_t)c->q * store_bytes(grid->storage) + 16) > INFINITY_CACHE_BYTES;
  c->L = L0;
  c->ws = (char*)workspace;
  c->ws_bytes = ws_bytes;

  Params& P = c->P;
  P.nx = nx;
  P.nc = (int)c->nc;
  P.px = grid->periodic[0] ? 1 : 0;
  P.inlet = (op && op->inlet) ? 1 : 0;
  P.outlet = op ? op->outlet : 0;
  P.nrow = (int)nrow;
  P.xbits = xb;
  const size_t pc = (size_t)plane_cells(c->nc);
  for (int i = 0; i < c->q; ++i) P.plb[i] = (uint32_t)((size_t)i * pc * store_bytes(grid->storage));
  P.abytes = (uint32_t)((size_t)c->q * pc * store_bytes(grid->storage));
  {
    Params::K<double> k{};
    k.U = c->U; k.iU = 1.0 / c->U; k.ks = c->U / (c->q == 27 ? 216.0 : 36.0);  // U w_i = ks * (integer weight)
    k.nu0 = rh->nu0; k.nu_inf = rh->nu_inf; k.dnu = rh->nu0 - rh->nu_inf;
    k.lam = rh->lambda; k.cy_e = (rh->n - 1.0) / rh->a; k.cy_a = rh->a;
    k.nu_d = po->nu_darcy; k.kcd = po->kc / (po->d * po->d);
    k.gx = po->g[0]; k.gy = po->g[1]; k.gz = po->g[2];
    k.rho_out = (op && op->outlet == 1) ? op->rho_out : 1.0;
    k.fk2 = 1.75 * std::sqrt(k.kcd / 150.0);
    P.d = k;
    P.f = Params::K<float>{(float)k.U, (float)k.iU, (float)k.ks, (float)k.nu0, (float)k.nu_inf, (float)k.dnu,
                           (float)k.lam, (float)k.cy_e, (float)k.cy_a, (float)k.nu_d, (float)k.kcd,
                           (float)k.gx, (float)k.gy, (float)k.gz, (float)k.rho_out, (float)k.fk2};
  }
  P.in_a0 = (op && op->inlet) ? op->a0 : 0.0;
  P.in_a1 = (op && op->inlet) ? op->a1 : 0.0;
  P.in_period = (op && op->inlet) ? op->period : 1.0;
  P.in_table = (op && op->inlet && op->wave_table) ? op->table_len : 0;
  P.in_ramp = (op && op->inlet) ? (uint32_t)op->ramp_steps : 0u;
  P.cy_a2 = rh->a == 2.0 ? 1 : 0;
  P.forch = po->forchheimer ? 1 : 0;
  P.an_iters = aniso ? po->aniso_iters : 0;
  for (int k = 0; k < 6; ++k) {
    P.d.Mi[k] = an_inv[k];
    P.d.Mh[k] = an_ih[k];
    P.f.Mi[k] = (float)an_inv[k];
    P.f.Mh[k] = (float)an_ih[k];
  }
  c->amode = grid->arith == LBM_ARITH_FP64 ? 2
             : (grid->arith == LBM_ARITH_AUTO && grid->storage == LBM_STORE_FP32) ? 1 : 0;
  c->omega0 = (float)(2.0 / (6.0 * rh->nu0 + 1.0));

  auto bail = [&](lbm_status st) { delete c; return st; };
#define HIP_TRY0(expr)                                                                              \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess) return bail(fail(LBM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_))); \
  } while (0)
  // slots that no consumer reads are never written by the kernels; clear them once
  HIP_TRY0(hipMemsetAsync(c->ws + c->L.A, 0, c->L.code - c->L.A, c->stream));
  HIP_TRY0(hipMemcpyAsync(c->ws + c->L.code, c->code.data(), c->code.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY0(hipMemcpyAsync(c->ws + c->L.delta, c->delta.data(), c->delta.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY0(hipMemcpyAsync(c->ws + c->L.rel, c->rel.data(), c->rel.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY0(hipMemcpyAsync(c->ws + c->L.shape, shape.data(), shape.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY0(hipMemcpyAsync(c->ws + c->L.rowbox, c->rowbox.data(), c->rowbox.size() * 4, hipMemcpyHostToDevice, c->stream));
  if (P.in_table > 0)
    HIP_TRY0(hipMemcpyAsync(c->ws + c->L.wave, op->wave_table, (size_t)P.in_table * sizeof(double),
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY0(hipMemsetAsync(c->ws + c->L.omega, 0, c->nc * 4, c->stream));
  HIP_TRY0(hipStreamSynchronize(c->stream));
#undef HIP_TRY0
  s = upload_phi(c, phi);
  if (s != LBM_OK) return bail(s);
  s = launch_init(c);
  if (s != LBM_OK) return bail(s);
  *out = c;
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int n) {
  CTX_CHECK(c);
  if (n < 0) return fail(LBM_E_INVALID, "n must be >= 0");
  for (int s = 0; s < n; ++s) {
    const bool check = ((c->t + 1) % CHECK_EVERY) == 0;
    lbm_status st = launch_step(c, check ? 1 : 0, nullptr, nullptr);
    if (st != LBM_OK) return st;
    if (check) {
      double dg[NDIAGP];
      st = read_diag(c, c->sblk, dg);
      if (st != LBM_OK) return st;
      st = check_stable(c, dg);
      if (st != LBM_OK) return st;
    }
  }
  return LBM_OK;
}

lbm_status lbm_moments(lbm_ctx* c, float* rho, float* u, float* shear, float* omega, float* sigma, float* tau) {
  CTX_CHECK(c);
  const size_t nb = c->nbox * 4;
  if (rho) HIP_TRY(c, hipMemsetAsync(rho, 0, nb, c->stream));
  if (u) HIP_TRY(c, hipMemsetAsync(u, 0, 3 * nb, c->stream));
  if (shear) HIP_TRY(c, hipMemsetAsync(shear, 0, nb, c->stream));
  if (omega) HIP_TRY(c, hipMemsetAsync(omega, 0, nb, c->stream));
  if (sigma) HIP_TRY(c, hipMemsetAsync(sigma, 0, 6 * nb, c->stream));
  if (tau) HIP_TRY(c, hipMemsetAsync(tau, 0, 3 * nb, c->stream));
  return moments_launch(c, false, rho, u, shear, omega, sigma, tau);
}

lbm_status lbm_diagnostics(lbm_ctx* c, double* out) {
  CTX_CHECK(c);
  if (!out) return fail(LBM_E_INVALID, "out is NULL");
  lbm_status s = moments_launch(c, true, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  if (s != LBM_OK) return s;
  double dg[NDIAGP];
  s = read_diag(c, c->nblk, dg);
  if (s != LBM_OK) return s;
  for (int k = 0; k < 10; ++k) out[k] = dg[k];
  out[10] = (double)c->t;
  out[11] = c->nwss > 0 ? dg[10] / (double)c->nwss : 0.0;
  return LBM_OK;
}

lbm_status lbm_diagnostics_noalloc(lbm_ctx* c, double* out) {
  CTX_CHECK(c);
  if (!out) return fail(LBM_E_INVALID, "out is NULL");
  const size_t part_bytes = align_up((size_t)c->nblk * NDIAGP * sizeof(double));
  const size_t need = noalloc_need(c->nblk);
  if (need > STATIC_SCRATCH_BYTES)
    return fail(LBM_E_INVALID, "lbm_diagnostics_noalloc needs " + std::to_string(need) +
                                   " bytes of scratch; the static area holds " +
                                   std::to_string(STATIC_SCRATCH_BYTES) + " (at most " +
                                   std::to_string(max_noalloc_cells()) + " compact cells)");
  void* base = nullptr;
  lbm_status s = scratch_address(c->device, &base);
  if (s != LBM_OK) return s;
  double* part = (double*)base;                      // every block writes all its partials
  double* dout = (double*)((char*)base + part_bytes);
  s = moments_launch(c, true, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, part);
  if (s != LBM_OK) return s;
  double dg[NDIAGP];
  s = finalize(c, part, c->nblk, NDIAGP, DIAG_OPS, dg, dout);
  if (s != LBM_OK) return s;
  for (int k = 0; k < 10; ++k) out[k] = dg[k];
  out[10] = (double)c->t;
  out[11] = c->nwss > 0 ? dg[10] / (double)c->nwss : 0.0;
  return LBM_OK;
}

lbm_status lbm_get_state(lbm_ctx* c, double* f, float* omega) {
  CTX_CHECK(c);
  if (!f && !omega) return fail(LBM_E_INVALID, "nothing to get");
  if (f) {
    lbm_status s = refresh_phi_host(c);
    if (s != LBM_OK) return s;
  }
  float* stage = (float*)(c->ws + c->L.stage);
  const size_t nf = (size_t)c->nf, nc = (size_t)c->nc;
  if (f) {
    lbm_status s = gather_state(c, stage);
    if (s != LBM_OK) return s;
    const int q = c->q;
    std::vector<float> h(q * nc);
    HIP_TRY(c, hipMemcpyAsync(h.data(), stage, h.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const double iU = 1.0 / c->U;
    for (int i = 0; i < q; ++i)
      for (size_t k = 0; k < nf; ++k) {
        const float v = h[i * nc + c->fluid_c[k]];
        f[i * nf + k] = std::isnan(v) ? 0.0 : (double)v * iU + rest_value(c, i, (int64_t)k);
      }
  }
  if (omega) {
    std::vector<float> h(nc);
    HIP_TRY(c, hipMemcpyAsync(h.data(), c->ws + c->L.omega, nc * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (size_t k = 0; k < nf; ++k) omega[k] = h[c->fluid_c[k]];
  }
  return LBM_OK;
}

lbm_status lbm_set_state(lbm_ctx* c, const double* f, const float* omega) {
  CTX_CHECK(c);
  if (!f && !omega) return fail(LBM_E_INVALID, "nothing to set");
  if (f) {
    lbm_status s = refresh_phi_host(c);
    if (s != LBM_OK) return s;
  }
  float* stage = (float*)(c->ws + c->L.stage);
  const size_t nf = (size_t)c->nf, nc = (size_t)c->nc;
  if (f) {
    const int q = c->q;
    std::vector<float> h(q * nc, 0.0f);
    for (int i = 0; i < q; ++i)
      for (size_t k = 0; k < nf; ++k)
        h[i * nc + c->fluid_c[k]] = (float)((f[i * nf + k] - rest_value(c, i, (int64_t)k)) * c->U);
    HIP_TRY(c, hipMemcpyAsync(stage, h.data(), h.size() * 4, hipMemcpyHostToDevice, c->stream));
    lbm_status s = scatter_state(c, stage);
    if (s != LBM_OK) return s;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  if (omega) {
    std::vector<float> h(nc, 0.0f);
    for (size_t k = 0; k < nf; ++k) h[c->fluid_c[k]] = omega[k];
    HIP_TRY(c, hipMemcpyAsync(c->ws + c->L.omega, h.data(), nc * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  return LBM_OK;
}

lbm_status lbm_reset(lbm_ctx* c) {
  CTX_CHECK(c);
  return launch_init(c);
}

lbm_status lbm_set_porosity(lbm_ctx* c, const float* phi) {
  CTX_CHECK(c);
  if (!phi) return fail(LBM_E_INVALID, "phi is NULL");
  uint32_t bad = 0;
  lbm_status s = set_porosity_device(c, phi, &bad);
  if (s != LBM_OK) return s;
  if (bad != 0xffffffffu) {
    const auto it = std::lower_bound(c->fluid_c.begin(), c->fluid_c.end(), (int64_t)bad);
    const int64_t box = it != c->fluid_c.end() && *it == (int64_t)bad ? c->fluid_box[it - c->fluid_c.begin()] : -1;
    return fail(LBM_E_INVALID, "porosity must lie in (0, 1] on every fluid cell and be 1 on open-face cells "
                               "(box index " + std::to_string(box) + ")");
  }
  c->phi_stale = true;
  return launch_init(c);
}

lbm_status lbm_fluid_cells(lbm_ctx* c, int64_t* n) {
  CTX_CHECK(c);
  if (!n) return fail(LBM_E_INVALID, "n is NULL");
  *n = c->nf;
  return LBM_OK;
}

lbm_status lbm_fluid_index(lbm_ctx* c, int64_t* box_index) {
  CTX_CHECK(c);
  if (!box_index) return fail(LBM_E_INVALID, "box_index is NULL");
  std::memcpy(box_index, c->fluid_box.data(), c->fluid_box.size() * 8);
  return LBM_OK;
}

lbm_status lbm_time(lbm_ctx* c, int64_t* t) {
  CTX_CHECK(c);
  if (!t) return fail(LBM_E_INVALID, "t is NULL");
  *t = c->t;
  return LBM_OK;
}

lbm_status lbm_copy_probe(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src || bytes % 16 != 0) return fail(LBM_E_INVALID, "copy probe needs non-null buffers and bytes % 16 == 0");
  const size_t n = bytes / 16;
  size_t blocks = (n + BLOCK - 1) / BLOCK;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) return LBM_OK;
  launch_copy((hipStream_t)stream, src, dst, n, (unsigned)blocks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LBM_E_DEVICE, std::string("copy probe: ") + hipGetErrorString(e));
  return LBM_OK;
}

lbm_status lbm_bandwidth_probe(int kind, void* dst, const void* src, size_t bytes, void* stream) {
  if (kind < LBM_PROBE_COPY || kind > LBM_PROBE_WRITE) return fail(LBM_E_INVALID, "unknown probe kind");
  if (bytes % 16 != 0 || bytes == 0) return fail(LBM_E_INVALID, "probe bytes must be a positive multiple of 16");
  if (!dst || (kind != LBM_PROBE_WRITE && !src)) return fail(LBM_E_INVALID, "probe buffers must not be NULL");
  const size_t n = bytes / 16;
  const unsigned blocks = LBM_PROBE_BLOCKS;
  launch_probe((hipStream_t)stream, kind, src, dst, n, blocks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LBM_E_DEVICE, std::string("bandwidth probe: ") + hipGetErrorString(e));
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* c) { delete c; }

}  // extern "C"

