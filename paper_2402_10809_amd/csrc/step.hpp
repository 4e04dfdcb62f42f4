// Fused D3Q19 VANSE Carreau-Yasuda stream-collide step and its companions
// (rest-state init, moments/diagnostics, state gather/scatter).
//
// One work-item per fluid cell, 1-D grid over the compact fluid list.  The
// populations live in two structure-of-arrays buffers over the dense box
// (plane stride nbox); a step pulls from A at x - c_i and writes B at x.
//
// Stored values are deviations from a rest value.  With shift mode 0 the
// producer at x stores q_i(x) - w_i phi~(x + c_i), where phi~ is the porosity of
// the consumer cell (its own porosity when the link bounces back), so every
// consumer reads delta_i = f_i - w_i phi(x) and the whole collision runs on
// deltas:
//   rho - 1 = sum(delta)/phi,  m = sum(delta c),
//   delta_eq_i = w_i phi [(rho - 1) + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)],
//   stored_i = delta_i - omega (delta_i - delta_eq_i) + G_i + w_i (rho - 1)(phi~_i - phi).
// This is the paper's collide-and-stream update (method section) with f_eq,
// Omega^phi, Guo's Omega^f and Omega^SRT expanded around the rest state, which
// keeps the O(u) signal far above FP32/FP16 rounding of the O(1) rest value.
// Shift mode 1 stores f_i - w_i instead and converts on load and store.
#pragma once
#include "lattice.hpp"

namespace lbm {

struct Params {
  int nx, ny, nz, nf;
  uint32_t nxy, nbox;
  int px, py, pz;
  int inlet, outlet;
  float nu0, nu_inf, lam, cy_e, cy_a;  // Carreau-Yasuda; cy_e = (n-1)/a
  int cy_a2;                           // a == 2: (lambda g)^a is one multiply
  float nu_d, kcd;                     // Darcy viscosity, kc/d^2
  int forch;
  float gx, gy, gz;
  float rho_out;
};

struct Bufs {
  const void* A;
  void* B;
  const uint32_t* cells;
  const float* phi;       // dense box porosity, 0 = solid
  float* omega;           // per fluid cell, previous relaxation rate
  const float* shape;     // inflow profile, ny*nz
  double* part;           // per-block partials
  float* rec;             // recompute record: [20][nf] (pulled deltas, omega_prev)
  float* rho_box;         // recompute record: dense rho of the step
};

// Per-axis offsets from a cell to its -1 / +1 neighbour, with periodic wrap,
// and whether that neighbour lies outside a non-periodic face.
struct Nb {
  int oxm, oxp, oym, oyp, ozm, ozp;
  bool nxm, nxp, nym, nyp, nzm, nzp;
  __device__ __forceinline__ Nb(const Params& p, int x, int y, int z) {
    nxm = (x == 0) && !p.px;
    nxp = (x == p.nx - 1) && !p.px;
    nym = (y == 0) && !p.py;
    nyp = (y == p.ny - 1) && !p.py;
    nzm = (z == 0) && !p.pz;
    nzp = (z == p.nz - 1) && !p.pz;
    oxm = x > 0 ? -1 : (p.px ? p.nx - 1 : 0);
    oxp = x < p.nx - 1 ? 1 : (p.px ? -(p.nx - 1) : 0);
    const int sy = p.nx, sz = (int)p.nxy;
    oym = y > 0 ? -sy : (p.py ? (p.ny - 1) * sy : 0);
    oyp = y < p.ny - 1 ? sy : (p.py ? -(p.ny - 1) * sy : 0);
    ozm = z > 0 ? -sz : (p.pz ? (p.nz - 1) * sz : 0);
    ozp = z < p.nz - 1 ? sz : (p.pz ? -(p.nz - 1) * sz : 0);
  }
  // Offset and outside flag of x + s (s a lattice vector with entries in {-1,0,1}).
  template <int SX, int SY, int SZ>
  __device__ __forceinline__ int off(bool& out) const {
    int o = 0;
    out = false;
    if (SX == -1) { o += oxm; out |= nxm; }
    if (SX == 1) { o += oxp; out |= nxp; }
    if (SY == -1) { o += oym; out |= nym; }
    if (SY == 1) { o += oyp; out |= nyp; }
    if (SZ == -1) { o += ozm; out |= nzm; }
    if (SZ == 1) { o += ozp; out |= nzp; }
    return o;
  }
  // Whether x + s is outside the open x face only (not also outside a wall face).
  template <int SX, int SY, int SZ>
  __device__ __forceinline__ bool open_only(const Params& p, int x) const {
    bool ox = (SX == -1 && x == 0 && p.inlet) || (SX == 1 && x == p.nx - 1 && p.outlet);
    bool wall = (SY == -1 && nym) || (SY == 1 && nyp) || (SZ == -1 && nzm) || (SZ == 1 && nzp);
    return ox && !wall;
  }
};

template <int I> struct Dir {
  static constexpr int cx = CX[I], cy = CY[I], cz = CZ[I], opp = OPP[I];
};

// Pull: delta_i(x) = stored value at x - c_i, or the cell's own opposite value
// when x - c_i is solid or outside a wall/open face (halfway bounce-back; the
// open-face unknowns are replaced by the Zou-He fill afterwards).  Also returns
// pt[j] = porosity of x + c_j (phi(x) across walls), for the producer side.
template <class S, bool SHW>
__device__ __forceinline__ void pull(const Params& p, const S* __restrict__ A, const float* __restrict__ phi,
                                     uint32_t idx, const Nb& nb, float phx, float d[Q], float pt[Q]) {
  pt[0] = phx;
  d[0] = Store<S>::ld(A, idx, 0);
#define LBM_PULL(I)                                                                   \
  {                                                                                   \
    bool out;                                                                         \
    const int o = nb.template off<-Dir<I>::cx, -Dir<I>::cy, -Dir<I>::cz>(out);        \
    const uint32_t src = idx + (uint32_t)o;                                           \
    const float pn = ldo(phi, src);                                                   \
    const bool bb = out || (pn == 0.0f);                                              \
    pt[Dir<I>::opp] = bb ? phx : pn;                                                  \
    const uint32_t e = bb ? (uint32_t)Dir<I>::opp * p.nbox + idx : (uint32_t)I * p.nbox + src; \
    d[I] = Store<S>::ld(A, e, I);                                                     \
  }
  LBM_PULL(1) LBM_PULL(2) LBM_PULL(3) LBM_PULL(4) LBM_PULL(5) LBM_PULL(6)
  LBM_PULL(7) LBM_PULL(8) LBM_PULL(9) LBM_PULL(10) LBM_PULL(11) LBM_PULL(12)
  LBM_PULL(13) LBM_PULL(14) LBM_PULL(15) LBM_PULL(16) LBM_PULL(17) LBM_PULL(18)
#undef LBM_PULL
  if (SHW) {
    const float s = phx - 1.0f;
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] -= wgt(i) * s;
  }
}

// Zou-He fill of the unknown populations on the open faces (phi = 1 there, so
// delta = f - w and the closures hold for deltas as for populations).
__device__ __forceinline__ void open_fill(const Params& p, int x, int y, int z, float amp,
                                          const float* __restrict__ shape, float d[Q]) {
  const bool in = p.inlet && x == 0;
  const bool outl = p.outlet && x == p.nx - 1;
  if (!(in || outl)) return;
  const float s0 = d[0] + d[3] + d[4] + d[5] + d[6] + d[15] + d[16] + d[17] + d[18];
  const float ny_ = 0.5f * (d[3] - d[4] + d[15] - d[16] + d[17] - d[18]);
  const float nz_ = 0.5f * (d[5] - d[6] + d[15] - d[16] - d[17] + d[18]);
  // inflow: prescribed u = (ux, 0, 0); density from mass and normal momentum
  const float uin = in ? amp * shape[y + p.ny * z] : 0.0f;
  const float sm = d[2] + d[8] + d[10] + d[12] + d[14];
  const float rin = (1.0f + s0 + 2.0f * sm) / (1.0f - uin);
  // outflow: prescribed density, normal velocity from mass and the known half
  const float sp = d[1] + d[7] + d[9] + d[11] + d[13];
  const float ro = p.rho_out;
  const float uout = (1.0f + s0 + 2.0f * sp) / ro - 1.0f;
  const float r3i = rin * uin * (1.0f / 3.0f), r6i = rin * uin * (1.0f / 6.0f);
  const float r3o = ro * uout * (1.0f / 3.0f), r6o = ro * uout * (1.0f / 6.0f);
  const float i1 = d[2] + r3i, i7 = d[8] + r6i - ny_, i9 = d[10] + r6i + ny_, i11 = d[12] + r6i - nz_,
              i13 = d[14] + r6i + nz_;
  const float o2 = d[1] - r3o, o8 = d[7] - r6o + ny_, o10 = d[9] - r6o - ny_, o12 = d[11] - r6o + nz_,
              o14 = d[13] - r6o - nz_;
  d[1] = in ? i1 : d[1];
  d[7] = in ? i7 : d[7];
  d[9] = in ? i9 : d[9];
  d[11] = in ? i11 : d[11];
  d[13] = in ? i13 : d[13];
  d[2] = outl ? o2 : d[2];
  d[8] = outl ? o8 : d[8];
  d[10] = outl ? o10 : d[10];
  d[12] = outl ? o12 : d[12];
  d[14] = outl ? o14 : d[14];
}

// Macroscopic state of one cell for one step.
struct Macro {
  float rho, rm1;         // density and rho - 1
  float ux, uy, uz, uu;   // velocity
  float Fx, Fy, Fz;       // force density rho f(u)
  float P[6];             // corrected second moment Pi (xx yy zz xy xz yz)
  float shear, omega;
};

// Hardware reciprocal refined by one Newton step (the raw v_rcp_f32 result is
// biased by up to an ulp, which accumulates over thousands of steps).
__device__ __forceinline__ float fast_rcp(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}

// Moments, explicit velocity with drag, force, Pi, shear rate and the new
// relaxation rate from the Carreau-Yasuda viscosity.
__device__ __forceinline__ void macro(const Params& p, float phx, const float d[Q], float omega_prev, Macro& M) {
  float sd = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) sd += d[i];
  const float mx = (d[1] + d[7] + d[9] + d[11] + d[13]) - (d[2] + d[8] + d[10] + d[12] + d[14]);
  const float my = (d[3] + d[7] + d[10] + d[15] + d[17]) - (d[4] + d[8] + d[9] + d[16] + d[18]);
  const float mz = (d[5] + d[11] + d[14] + d[15] + d[18]) - (d[6] + d[12] + d[13] + d[16] + d[17]);
  const float iphi = fast_rcp(phx);
  const float sumf = phx + sd;                 // phi rho
  const float rm1 = sd * iphi;                 // rho - 1
  const float rho = 1.0f + rm1;
  const float isum = fast_rcp(sumf);
  const float hg = 0.5f * iphi;
  const float vx = mx * isum + p.gx * hg, vy = my * isum + p.gy * hg, vz = mz * isum + p.gz * hg;
  // 1/k = (kc/d^2) (1 - phi)^2 / phi^3
  const float om = 1.0f - phx;
  const float invk = p.kcd * om * om * iphi * iphi * iphi;
  const float dark = phx * p.nu_d * invk;      // phi nu / k
  const float C0 = 0.5f + 0.25f * dark;
  float den, fcoef;
  if (p.forch) {
    const float sik = __builtin_sqrtf(invk);
    const float cf = 1.75f * __builtin_sqrtf(iphi * iphi * iphi * (1.0f / 150.0f));
    const float C1 = 0.5f * phx * phx * cf * sik;
    const float vn = __builtin_sqrtf(vx * vx + vy * vy + vz * vz);
    den = C0 + __builtin_sqrtf(C0 * C0 + C1 * vn);
    fcoef = phx * phx * phx * cf * sik;        // times |u| below
  } else {
    den = 2.0f * C0;
    fcoef = 0.0f;
  }
  const float iden = fast_rcp(den);
  const float ux = vx * iden, uy = vy * iden, uz = vz * iden;
  const float uu = ux * ux + uy * uy + uz * uz;
  const float drag = phx * dark + (p.forch ? fcoef * __builtin_sqrtf(uu) : 0.0f);  // phi^2 nu/k + phi^3 C_F |u|/sqrt(k)
  const float Fx = rho * (p.gx - drag * ux), Fy = rho * (p.gy - drag * uy), Fz = rho * (p.gz - drag * uz);
  // Pi = sum delta c c - [phi (rho-1)/3 I + phi rho u u] + (F u + u F)/2
  const float pr = phx * rho;
  const float iso = phx * rm1 * (1.0f / 3.0f);
  const float Sxx = d[1] + d[2] + d[7] + d[8] + d[9] + d[10] + d[11] + d[12] + d[13] + d[14];
  const float Syy = d[3] + d[4] + d[7] + d[8] + d[9] + d[10] + d[15] + d[16] + d[17] + d[18];
  const float Szz = d[5] + d[6] + d[11] + d[12] + d[13] + d[14] + d[15] + d[16] + d[17] + d[18];
  const float Sxy = (d[7] + d[8]) - (d[9] + d[10]);
  const float Sxz = (d[11] + d[12]) - (d[13] + d[14]);
  const float Syz = (d[15] + d[16]) - (d[17] + d[18]);
  M.P[0] = Sxx - iso - pr * ux * ux + Fx * ux;
  M.P[1] = Syy - iso - pr * uy * uy + Fy * uy;
  M.P[2] = Szz - iso - pr * uz * uz + Fz * uz;
  M.P[3] = Sxy - pr * ux * uy + 0.5f * (Fx * uy + ux * Fy);
  M.P[4] = Sxz - pr * ux * uz + 0.5f * (Fx * uz + ux * Fz);
  M.P[5] = Syz - pr * uy * uz + 0.5f * (Fy * uz + uy * Fz);
  const float pn2 = M.P[0] * M.P[0] + M.P[1] * M.P[1] + M.P[2] * M.P[2] +
                    2.0f * (M.P[3] * M.P[3] + M.P[4] * M.P[4] + M.P[5] * M.P[5]);
  const float irho = fast_rcp(rho);
  const float shear = 3.0f * omega_prev * __builtin_sqrtf(pn2) * irho;
  // Carreau-Yasuda: nu = nu_inf + (nu0 - nu_inf) (1 + (lambda g)^a)^((n-1)/a)
  const float lg = p.lam * shear;
  float la;
  if (p.cy_a2) la = lg * lg;
  else la = lg > 0.0f ? __builtin_amdgcn_exp2f(p.cy_a * __builtin_amdgcn_logf(lg)) : 0.0f;
  const float fac = __builtin_amdgcn_exp2f(p.cy_e * __builtin_amdgcn_logf(1.0f + la));
  const float nu = p.nu_inf + (p.nu0 - p.nu_inf) * fac;
  // omega = 2 rho c_s^2 / (2 mu + rho c_s^2) = 2 rho / (6 nu + rho)
  M.omega = 2.0f * rho * fast_rcp(6.0f * nu + rho);
  M.rho = rho;
  M.rm1 = rm1;
  M.ux = ux; M.uy = uy; M.uz = uz; M.uu = uu;
  M.Fx = Fx; M.Fy = Fy; M.Fz = Fz;
  M.shear = shear;
}

// BGK + Guo + porosity-jump collision, stored as deviations for the consumer.
// Directions come in opposite pairs: with e = c.u and h = c.F the even part
// (omega (A0 + C e^2) - K3 u.F + K9 e h) is shared and the odd part
// (omega B e + K3 h) flips sign.
template <class S, bool SHW>
__device__ __forceinline__ void collide_store(const Params& p, S* __restrict__ B, uint32_t idx, float phx,
                                              const float d[Q], const float pt[Q], const Macro& M) {
  const float om = M.omega;
  const float pr = phx * M.rho;
  const float A0 = phx * M.rm1 - 1.5f * pr * M.uu;
  const float Bc = 3.0f * pr, Cc = 4.5f * pr;
  const float K = 1.0f - 0.5f * om;
  const float K3 = 3.0f * K, K9 = 9.0f * K;
  const float uF = M.ux * M.Fx + M.uy * M.Fy + M.uz * M.Fz;
  const float keep = 1.0f - om;
  const float ev0 = om * A0 - K3 * uF;
  const float shw = phx - 1.0f;
  // rest direction
  {
    float v = wfma(0, ev0 + M.rm1 * (pt[0] - phx), keep * d[0]);
    if (SHW) v += wgt(0) * shw;
    Store<S>::st(B, idx, v, 0);
  }
#define LBM_PAIR(I, EX, HX)                                                              \
  {                                                                                      \
    constexpr int J = Dir<I>::opp;                                                       \
    const float e = (EX), h = (HX);                                                      \
    const float ev = ev0 + om * Cc * e * e + K9 * e * h;                                 \
    const float od = om * Bc * e + K3 * h;                                               \
    float vi = wfma(I, ev + od + M.rm1 * (pt[I] - phx), keep * d[I]);                    \
    float vj = wfma(J, ev - od + M.rm1 * (pt[J] - phx), keep * d[J]);                    \
    if (SHW) { vi += wgt(I) * (pt[I] - 1.0f); vj += wgt(J) * (pt[J] - 1.0f); }           \
    Store<S>::st(B, (uint32_t)I * p.nbox + idx, vi, I);                                  \
    Store<S>::st(B, (uint32_t)J * p.nbox + idx, vj, J);                                  \
  }
  LBM_PAIR(1, M.ux, M.Fx)
  LBM_PAIR(3, M.uy, M.Fy)
  LBM_PAIR(5, M.uz, M.Fz)
  LBM_PAIR(7, M.ux + M.uy, M.Fx + M.Fy)
  LBM_PAIR(9, M.ux - M.uy, M.Fx - M.Fy)
  LBM_PAIR(11, M.ux + M.uz, M.Fx + M.Fz)
  LBM_PAIR(13, M.ux - M.uz, M.Fx - M.Fz)
  LBM_PAIR(15, M.uy + M.uz, M.Fy + M.Fz)
  LBM_PAIR(17, M.uy - M.uz, M.Fy - M.Fz)
#undef LBM_PAIR
  (void)shw;
}

// ---------------------------------------------------------------------------
// Block reduction of FP64 partials: wave64 shuffle, then LDS across the 4 waves.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void block_reduce(double (&v)[N], const int (&op)[N], double* out) {
  __shared__ double sh[BLOCK / 64][N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      double o = __shfl_xor(v[k], m, 64);
      v[k] = op[k] == 0 ? v[k] + o : (op[k] == 1 ? fmax(v[k], o) : fmin(v[k], o));
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) sh[wv][k] = v[k];
  __syncthreads();
  if (threadIdx.x < N) {
    const int k = threadIdx.x;
    double r = sh[0][k];
    for (int w = 1; w < BLOCK / 64; ++w)
      r = op[k] == 0 ? r + sh[w][k] : (op[k] == 1 ? fmax(r, sh[w][k]) : fmin(r, sh[w][k]));
    out[k] = r;
  }
}

// Per-cell diagnostic contributions: mass, momentum, energy, region energy,
// max |u|, min/max omega, non-finite count.
__device__ __forceinline__ void diag_terms(float phx, const float d[Q], const Macro& M, bool reg, bool active,
                                           double (&v)[NDIAGP]) {
  if (!active) {
    v[0] = v[1] = v[2] = v[3] = v[4] = v[5] = v[9] = 0.0;
    v[6] = 0.0; v[7] = 1e300; v[8] = -1e300;
    return;
  }
  float sd = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) sd += d[i];
  v[0] = (double)phx + (double)sd;
  v[1] = (double)((d[1] + d[7] + d[9] + d[11] + d[13]) - (d[2] + d[8] + d[10] + d[12] + d[14]));
  v[2] = (double)((d[3] + d[7] + d[10] + d[15] + d[17]) - (d[4] + d[8] + d[9] + d[16] + d[18]));
  v[3] = (double)((d[5] + d[11] + d[14] + d[15] + d[18]) - (d[6] + d[12] + d[13] + d[16] + d[17]));
  const double ke = 0.5 * (double)M.rho * (double)M.uu;
  v[4] = ke;
  v[5] = reg ? ke : 0.0;
  v[6] = (double)__builtin_sqrtf(M.uu);
  v[7] = (double)M.omega;
  v[8] = (double)M.omega;
  const bool bad = !(__builtin_isfinite(M.rho) && __builtin_isfinite(M.uu) && __builtin_isfinite(M.omega) &&
                     __builtin_isfinite(M.shear));
  v[9] = bad ? 1.0 : 0.0;
  if (bad) { v[6] = 1e300; }
}

// ---------------------------------------------------------------------------
// The step.  DIAG: 0 none, 1 diagnostics of the pre-collision state into
// part[block][NDIAGP], 2 region kinetic energy accumulated into part[block].
// REC: also record the pulled deltas and omega_prev ([20][nf]) and rho (box).
// ---------------------------------------------------------------------------
template <class S, bool SHW, int DIAG, bool REC>
__global__ __launch_bounds__(BLOCK) void k_step(Params p, Bufs b, float amp) {
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t c = blk * BLOCK + threadIdx.x;
  const bool active = c < (uint32_t)p.nf;
  double dv[NDIAGP];
  float ke_reg = 0.0f;
  if (active) {
    int x, y, z;
    bool reg;
    unpack(b.cells[c], x, y, z, reg);
    const uint32_t idx = (uint32_t)x + p.nx * ((uint32_t)y + p.ny * (uint32_t)z);
    const float phx = ldo(b.phi, idx);
    const Nb nb(p, x, y, z);
    float d[Q], pt[Q];
    pull<S, SHW>(p, (const S*)b.A, b.phi, idx, nb, phx, d, pt);
    if (REC) {
#pragma unroll
      for (int i = 0; i < Q; ++i) b.rec[(size_t)i * p.nf + c] = d[i];
    }
    open_fill(p, x, y, z, amp, b.shape, d);
    const float omp = b.omega[c];
    Macro M;
    macro(p, phx, d, omp, M);
    b.omega[c] = M.omega;
    if (REC) {
      b.rec[(size_t)Q * p.nf + c] = omp;
      b.rho_box[idx] = M.rho;
    }
    if (DIAG == 1) diag_terms(phx, d, M, reg, true, dv);
    if (DIAG == 2) ke_reg = reg ? 0.5f * M.rho * M.uu : 0.0f;
    collide_store<S, SHW>(p, (S*)b.B, idx, phx, d, pt, M);
  } else if (DIAG == 1) {
    float d[Q] = {};
    Macro M{};
    diag_terms(0.f, d, M, false, false, dv);
  }
  if (DIAG == 1) {
    const int ops[NDIAGP] = {0, 0, 0, 0, 0, 0, 1, 2, 1, 0};
    block_reduce<NDIAGP>(dv, ops, b.part + (size_t)blockIdx.x * NDIAGP);
  }
  if (DIAG == 2) {
    double v[1] = {(double)ke_reg};
    const int ops[1] = {0};
    __shared__ double tmp[1];
    block_reduce<1>(v, ops, tmp);
    if (threadIdx.x == 0) b.part[blockIdx.x] += tmp[0];
  }
}

// Moments of the current state (no collision): dense outputs (any may be null)
// and optionally the diagnostics partials.
template <class S, bool SHW, bool DIAG>
__global__ __launch_bounds__(BLOCK) void k_moments(Params p, Bufs b, float amp, float* rho_o, float* u_o,
                                                    float* shear_o, float* omega_o, float* sigma_o) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  const bool active = c < (uint32_t)p.nf;
  double dv[NDIAGP];
  if (active) {
    int x, y, z;
    bool reg;
    unpack(b.cells[c], x, y, z, reg);
    const uint32_t idx = (uint32_t)x + p.nx * ((uint32_t)y + p.ny * (uint32_t)z);
    const float phx = ldo(b.phi, idx);
    const Nb nb(p, x, y, z);
    float d[Q], pt[Q];
    pull<S, SHW>(p, (const S*)b.A, b.phi, idx, nb, phx, d, pt);
    open_fill(p, x, y, z, amp, b.shape, d);
    Macro M;
    macro(p, phx, d, b.omega[c], M);
    if (rho_o) rho_o[idx] = M.rho;
    if (u_o) { u_o[idx] = M.ux; u_o[(size_t)p.nbox + idx] = M.uy; u_o[2 * (size_t)p.nbox + idx] = M.uz; }
    if (shear_o) shear_o[idx] = M.shear;
    if (omega_o) omega_o[idx] = M.omega;
    if (sigma_o) {
      const float s = 0.5f * M.omega - 1.0f;
#pragma unroll
      for (int k = 0; k < 6; ++k) sigma_o[(size_t)k * p.nbox + idx] = s * M.P[k];
    }
    if (DIAG) diag_terms(phx, d, M, reg, true, dv);
  } else if (DIAG) {
    float d[Q] = {};
    Macro M{};
    diag_terms(0.f, d, M, false, false, dv);
  }
  if (DIAG) {
    const int ops[NDIAGP] = {0, 0, 0, 0, 0, 0, 1, 2, 1, 0};
    block_reduce<NDIAGP>(dv, ops, b.part + (size_t)blockIdx.x * NDIAGP);
  }
}

// Reduce per-block partials (single workgroup, fixed order: deterministic).
// opmask holds 2 bits per entry: 0 sum, 1 max, 2 min.
__global__ __launch_bounds__(BLOCK) void k_finalize(const double* part, int nblk, int n, uint32_t opmask, double* out) {
  __shared__ double sh[BLOCK];
  for (int k = 0; k < n; ++k) {
    const int op = (int)((opmask >> (2 * k)) & 3u);
    double r = op == 0 ? 0.0 : (op == 1 ? -1e300 : 1e300);
    for (int i = threadIdx.x; i < nblk; i += BLOCK) {
      const double v = part[(size_t)i * n + k];
      r = op == 0 ? r + v : (op == 1 ? fmax(r, v) : fmin(r, v));
    }
    sh[threadIdx.x] = r;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        const double a = sh[threadIdx.x], c2 = sh[threadIdx.x + s];
        sh[threadIdx.x] = op == 0 ? a + c2 : (op == 1 ? fmax(a, c2) : fmin(a, c2));
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sh[0];
    __syncthreads();
  }
}

// Rest state: every consumer reads f_i = w_i phi(x).
template <class S, bool SHW>
__global__ __launch_bounds__(BLOCK) void k_init(Params p, Bufs b, float omega0) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= (uint32_t)p.nf) return;
  int x, y, z;
  bool reg;
  unpack(b.cells[c], x, y, z, reg);
  const uint32_t idx = (uint32_t)x + p.nx * ((uint32_t)y + p.ny * (uint32_t)z);
  const float phx = ldo(b.phi, idx);
  const Nb nb(p, x, y, z);
  float pt[Q];
  pt[0] = phx;
#define LBM_PT(I)                                                               \
  {                                                                             \
    bool out;                                                                   \
    const int o = nb.template off<Dir<I>::cx, Dir<I>::cy, Dir<I>::cz>(out);     \
    const float pn = ldo(b.phi, idx + (uint32_t)o);                             \
    pt[I] = (out || pn == 0.0f) ? phx : pn;                                     \
  }
  LBM_PT(1) LBM_PT(2) LBM_PT(3) LBM_PT(4) LBM_PT(5) LBM_PT(6) LBM_PT(7) LBM_PT(8) LBM_PT(9)
  LBM_PT(10) LBM_PT(11) LBM_PT(12) LBM_PT(13) LBM_PT(14) LBM_PT(15) LBM_PT(16) LBM_PT(17) LBM_PT(18)
#undef LBM_PT
  S* B = (S*)b.B;
#pragma unroll
  for (int i = 0; i < Q; ++i) Store<S>::st(B, (uint32_t)i * p.nbox + idx, SHW ? wgt(i) * (pt[i] - 1.0f) : 0.0f, i);
  b.omega[c] = omega0;
}

// State out: the pulled (pre-collision) stored values as FP32, [19][nf]; the
// host adds the rest value back in FP64.  Open-face unknowns are written as NaN.
template <class S>
__global__ __launch_bounds__(BLOCK) void k_gather_state(Params p, Bufs b, float* out) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= (uint32_t)p.nf) return;
  int x, y, z;
  bool reg;
  unpack(b.cells[c], x, y, z, reg);
  const uint32_t idx = (uint32_t)x + p.nx * ((uint32_t)y + p.ny * (uint32_t)z);
  const Nb nb(p, x, y, z);
  const S* A = (const S*)b.A;
  out[c] = Store<S>::ld(A, idx, 0);
#define LBM_G(I)                                                                          \
  {                                                                                       \
    bool o_;                                                                              \
    const int o = nb.template off<-Dir<I>::cx, -Dir<I>::cy, -Dir<I>::cz>(o_);             \
    const uint32_t src = idx + (uint32_t)o;                                               \
    const bool bb = o_ || ldo(b.phi, src) == 0.0f;                                        \
    const bool unk = nb.template open_only<-Dir<I>::cx, -Dir<I>::cy, -Dir<I>::cz>(p, x);  \
    const uint32_t e = bb ? (uint32_t)Dir<I>::opp * p.nbox + idx : (uint32_t)I * p.nbox + src; \
    out[(size_t)I * p.nf + c] = unk ? __builtin_nanf("") : Store<S>::ld(A, e, I);         \
  }
  LBM_G(1) LBM_G(2) LBM_G(3) LBM_G(4) LBM_G(5) LBM_G(6) LBM_G(7) LBM_G(8) LBM_G(9)
  LBM_G(10) LBM_G(11) LBM_G(12) LBM_G(13) LBM_G(14) LBM_G(15) LBM_G(16) LBM_G(17) LBM_G(18)
#undef LBM_G
}

// State in: inverse of k_gather_state; each stored slot that some consumer
// reads is written exactly once (by that consumer's link).
template <class S>
__global__ __launch_bounds__(BLOCK) void k_scatter_state(Params p, Bufs b, const float* in) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= (uint32_t)p.nf) return;
  int x, y, z;
  bool reg;
  unpack(b.cells[c], x, y, z, reg);
  const uint32_t idx = (uint32_t)x + p.nx * ((uint32_t)y + p.ny * (uint32_t)z);
  const Nb nb(p, x, y, z);
  S* A = (S*)b.B;
  Store<S>::st(A, idx, in[c], 0);
#define LBM_S(I)                                                                          \
  {                                                                                       \
    bool o_;                                                                              \
    const int o = nb.template off<-Dir<I>::cx, -Dir<I>::cy, -Dir<I>::cz>(o_);             \
    const uint32_t src = idx + (uint32_t)o;                                               \
    const bool bb = o_ || ldo(b.phi, src) == 0.0f;                                        \
    const bool unk = nb.template open_only<-Dir<I>::cx, -Dir<I>::cy, -Dir<I>::cz>(p, x);  \
    const uint32_t e = bb ? (uint32_t)Dir<I>::opp * p.nbox + idx : (uint32_t)I * p.nbox + src; \
    if (!unk) Store<S>::st(A, e, in[(size_t)I * p.nf + c], I);                            \
  }
  LBM_S(1) LBM_S(2) LBM_S(3) LBM_S(4) LBM_S(5) LBM_S(6) LBM_S(7) LBM_S(8) LBM_S(9)
  LBM_S(10) LBM_S(11) LBM_S(12) LBM_S(13) LBM_S(14) LBM_S(15) LBM_S(16) LBM_S(17) LBM_S(18)
#undef LBM_S
}

// Plain streaming copy (16-byte vectors), the achievable-bandwidth reference.
__global__ __launch_bounds__(BLOCK) void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
  size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * BLOCK;
  for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace lbm
