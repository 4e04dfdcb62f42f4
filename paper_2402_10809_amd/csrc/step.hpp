// Fused D3Q19 VANSE Carreau-Yasuda stream-collide step and its companions
// (rest-state init, moments/diagnostics, state gather/scatter).
//
// Layout.  Fluid cells are stored row by row: a row is one (y, z) line of the
// box that holds fluid, rows are ordered by z then y, and each row keeps the
// contiguous x range from its first to its last fluid cell (solid cells inside
// that range are "dead" slots that no kernel touches).  Every per-cell array
// and each of the 19 population planes is indexed by this compact index, so
// the touched memory is dense.  A cell's neighbour in the row (y - cy, z - cz)
// sits at x' + delta[row][pair(cy, cz)], where delta = (compact start - first
// x) of that row; periodic y and z wrap inside the delta table, periodic x by
// wrapping x'.
//
// Streaming uses one population buffer in place (the AA pattern): at even
// time t the populations f_i(t, x) sit at slot (i, x); the even step reads
// them there and writes its post-collision q_i(x) to slot (opp i, x).  At odd
// t, f_i(t, x) sits at slot (opp i, x - c_i) (slot (i, x) across a wall); the
// odd step reads there and writes q_i(x) to slot (i, x + c_i) (slot (opp i, x)
// across a wall), which is where the next even step finds it.  Within one
// step every slot is read and written by the same work-item, so no two
// work-items race.  The even step touches only the cell's own slots.
//
// Stored values are scaled deviations from a rest value: with shift mode 0 a
// value consumed as f_i by cell y is stored as U (f_i - w_i phi(y)) (phi(y) is
// the producer's phi~(x + c_i), its own porosity across a wall), so every
// consumer reads v_i = U (f_i - w_i phi(x)).  U = 36 (times 2^10 for FP16)
// makes U w_i an exact integer (12, 2, 1 times 2^k) for every direction, so
// the per-direction arithmetic carries no rounded weight: the collision
// conserves mass and momentum up to unbiased rounding only.  The whole
// collision runs on these deviations:
//   rho - 1 = sum(v) / (U phi),  m = sum(v c) / U,
//   v_eq_i = U w_i phi [(rho - 1) + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)],
//   out_i = v_i - omega (v_i - v_eq_i) + U G_i + U w_i (rho - 1)(phi~_i - phi).
// This is the paper's collide-and-stream update (method section) with f_eq,
// Omega^phi, Guo's Omega^f and Omega^SRT expanded around the rest state, which
// keeps the O(u) signal far above FP32/FP16 rounding of the O(1) rest value.
// Shift mode 1 stores U (f_i - w_i) instead and converts on load and store.
//
// Each cell carries a link word: bit i (1..18) = the pull of direction i
// bounces back (x - c_i is solid or outside a non-periodic face), plus flags
// (dead slot, uniform neighbour porosity, interior, open-face role, region,
// open-face unknowns).  Waves whose cells all have uniform neighbour porosity
// skip the neighbour porosity loads and the porosity-jump arithmetic; on odd
// steps, waves of interior cells also skip the bounce-back address selects.
// Uniform waves of pure fluid (porosity 1 in every lane, no body force) also
// skip the drag and force terms, which vanish there.
#pragma once
#include <type_traits>

#include "fp64math.hpp"
#include "lattice.hpp"

namespace lbm {

constexpr uint32_t LK_DEAD = 1u << 0;   // solid slot inside a row's range
constexpr uint32_t LK_UNI = 1u << 19;   // every fluid neighbour has the cell's porosity
constexpr uint32_t LK_IN = 1u << 20;    // inflow cell (x = 0)
constexpr uint32_t LK_OUT = 1u << 21;   // outflow cell (x = nx - 1)
constexpr uint32_t LK_REG = 1u << 22;   // objective region
constexpr int LK_UNK = 23;              // 5 bits: which x-directed pulls are open-face unknowns
constexpr uint32_t LK_UPS = 1u << 28;   // -x neighbour of an extrapolation-outflow cell
constexpr uint32_t LK_INR = 1u << 29;   // interior: no bounce-back pull, no x wrap
// the x-directed pulls of an inflow (c_x = +1) and an outflow (c_x = -1) cell
constexpr int XIN[5] = {1, 7, 9, 11, 13};
constexpr int XOUT[5] = {2, 8, 10, 12, 14};

// 36 w_i: 12 (rest), 2 (axis), 1 (edge).
__host__ __device__ constexpr float kw(int i) { return i == 0 ? 12.0f : (i < 7 ? 2.0f : 1.0f); }

struct Params {
  int nx, nc;                  // box x extent; compact cells (fluid + dead)
  int nrow;                    // rows of the compact layout
  int px;                      // periodic x
  int inlet, outlet;           // outlet: 1 constant density, 2 extrapolation
  int xbits;                   // code = (row << xbits) | x
  uint32_t plb[27];            // byte offset of population plane i (i * nc * sizeof(storage)), i < Q of the set
  uint32_t abytes;             // byte size of the population buffer
  int cy_a2;                   // a == 2: (lambda g)^a is one multiply
  int forch;                   // Forchheimer drag on
  int an_iters;                // anisotropic permeability: fixed-point iterations
  double in_a0, in_a1, in_period;  // inflow waveform W(s) = a0 (1 + a1 sin(2 pi s / period))
  int in_table;                    // > 0: W is the sampled table of that length over one period
  uint32_t in_ramp;                // pre-run ramp length R (0: none)
  // physical constants in both precisions (the kernels read the one they
  // compute in, straight from the kernel arguments)
  template <class T>
  struct K {
    T U, iU, ks;                 // storage unit, 1/U, U/36
    T nu0, nu_inf, dnu;          // Carreau-Yasuda limits, nu0 - nu_inf
    T lam, cy_e, cy_a;           // lambda, (n-1)/a, a
    T nu_d, kcd;                 // Darcy viscosity, kc/d^2
    T gx, gy, gz;                // body force
    T rho_out;
    T fk2;                       // 1.75 sqrt(kc / (150 d^2)): phi^3 C_F sqrt(1/k) = fk2 (1 - phi)
    T Mi[6], Mh[6];              // anisotropic permeability shape: M^-1, M^-1/2 (xx yy zz xy xz yz)
  };
  K<float> f;
  K<double> d;
  template <class T>
  __device__ __forceinline__ const K<T>& k() const {
    if constexpr (std::is_same<T, double>::value) return d;
    else return f;
  }
};

// Per wave of 64 compact cells (cells 64w .. 64w + 63): the row of its first
// cell, a bit per lane that starts a new row, and flags.  WV_FLUID: every
// lane is a fluid cell without open-face role; WV_UNI: every lane has uniform
// neighbour porosity; WV_INR: every lane is interior.  A plain wave (FLUID and
// UNI) needs neither the position codes nor the link words: even steps touch
// only the cells' own slots, and on odd steps an interior lane's row follows
// from the row starts and its neighbour rows from the per-row offsets rel.
// A FLUID and INR wave without uniform porosity needs them neither: its
// neighbours' porosities are read through the same offsets.
struct WaveInfo {
  uint64_t starts;
  uint32_t row0;
  uint32_t flags;
};
constexpr uint32_t WV_FLUID = 1u;
constexpr uint32_t WV_INR = 2u;
constexpr uint32_t WV_UNI = 4u;

struct Bufs {
  void* A;                // populations, [19][nc], in place
  const uint32_t* code;   // (row << xbits) | x per compact cell
  const uint32_t* links;  // link word per compact cell
  const int* delta;       // [nrow][8]: neighbour-row deltas for pairs 1..8
  const int* rel;         // [nrow][8]: compact index of (x, neighbour row k) minus that of (x, row)
  const WaveInfo* winfo;  // per wave of 64 compact cells
  const float* phi;       // porosity per compact cell
  float* omega;           // per compact cell, previous relaxation rate
  const float* shape;     // inflow profile per row
  const uint32_t* rowbox; // box index of (x = 0) of each row
  double* part;           // per-block partials
  float* rec;             // recompute record: [20][nc] (pulled values, omega_prev)
  float* rho_rec;         // recompute record: rho per compact cell
  uint32_t* tc;           // time counter: the step at parity k reads tc[k] and writes t + 1 to tc[1 - k]
  const double* wave;     // sampled inflow waveform (in_table entries)
  float* side;            // extrapolation outflow: [2][nrow][10] kept values by parity
};

template <int A, int B, class F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (A < B) {
    f(std::integral_constant<int, A>{});
    sfor<A + 1, B>(f);
  }
}

// Hardware reciprocal refined by Newton steps (the raw v_rcp result is biased
// by up to an ulp, which accumulates over thousands of steps).
__device__ __forceinline__ float fast_rcp(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double rsqrt_(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float rfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double rfma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Position of a compact cell and the deltas of its neighbour rows.  xm / xp
// are x - 1 / x + 1, wrapped on a periodic x axis.
struct Pos {
  uint32_t row;
  int x, xm, xp;
  int dl[NPAIR];
  uint32_t bo[NPAIR];  // interior cells: byte offset of (x, neighbour row k) in a plane
};
__device__ __forceinline__ Pos position(const Params& p, uint32_t c, uint32_t code) {
  Pos q;
  q.row = code >> p.xbits;
  q.x = (int)(code & ((1u << p.xbits) - 1u));
  q.xm = q.x - 1 + ((p.px && q.x == 0) ? p.nx : 0);
  q.xp = q.x + 1 - ((p.px && q.x == p.nx - 1) ? p.nx : 0);
  q.dl[0] = (int)c - q.x;
  return q;
}
__device__ __forceinline__ void load_deltas(const int* __restrict__ delta, Pos& q) {
  const int4* d4 = (const int4*)(delta + (size_t)q.row * 8);
  const int4 a = d4[0], b = d4[1];
  q.dl[1] = a.x; q.dl[2] = a.y; q.dl[3] = a.z; q.dl[4] = a.w;
  q.dl[5] = b.x; q.dl[6] = b.y; q.dl[7] = b.z; q.dl[8] = b.w;
}
// Interior cells (every pull source fluid, no x wrap): the sources of a
// neighbour-row pair k are x - c_x in that row, so one byte offset per row,
// (x + delta_k) * SB, serves all of them; the +-1 x shift and the plane go
// into the wave-uniform part.  x + delta_k is itself a fluid cell of that row
// (the pair's c_x = 0 direction pulls from it), hence non-negative.
template <class S>
__device__ __forceinline__ void interior_offsets(Pos& q) {
#pragma unroll
  for (int k = 0; k < NPAIR; ++k) q.bo[k] = (uint32_t)(q.x + q.dl[k]) * (uint32_t)sizeof(S);
}
// Compact index of x - c_I (valid when that cell is fluid).
template <int I>
__device__ __forceinline__ uint32_t src_of(const Params&, const Pos& q) {
  const int xs = CX[I] == 1 ? q.xm : (CX[I] == -1 ? q.xp : q.x);
  return (uint32_t)(xs + q.dl[PK[I]]);
}

// Load through a byte offset from a uniform base.
template <class T>
__device__ __forceinline__ T ldb(const T* base, uint32_t byte_off) {
  return *(const T*)((const char*)base + byte_off);
}

// The population buffer as a raw buffer resource: every access is a 32-bit
// byte offset split into a per-lane part (VGPR) and a wave-uniform part
// (SGPR soffset), so the 19 plane offsets of a local access cost no vector
// instructions.  The resource's size is the buffer's byte size.
template <class S>
struct Pop {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ Pop(const void* base, uint32_t bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000)) {}
  __device__ __forceinline__ float ld(uint32_t voff, uint32_t soff) const {
    if constexpr (std::is_same<S, float>::value) {
      return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    } else {
      const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
      return (float)__builtin_bit_cast(S, h);
    }
  }
  // a 16-bit storage value given as its bits
  __device__ __forceinline__ void st_bits(uint32_t voff, uint32_t soff, unsigned short h) const {
    __builtin_amdgcn_raw_buffer_store_b16(h, r, voff, soff, 0);
  }
  __device__ __forceinline__ void st(uint32_t voff, uint32_t soff, float v) const {
    if constexpr (std::is_same<S, float>::value) {
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
    } else {
      __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (S)v), r, voff, soff, 0);
    }
  }
};

// A slot address: per-lane and wave-uniform byte offsets.
struct Slot {
  uint32_t v, s;
};

// Slot holding f_I(t, x) at parity ODD (INR: the cell is interior, q.bo set;
// the plane offsets are at least nc * SB, so the uniform parts stay >= 0).
template <int I, bool ODD, class S, bool INR = false>
__device__ __forceinline__ Slot slot_in(const Params& p, uint32_t c, uint32_t lk, const Pos& q) {
  constexpr uint32_t SB = sizeof(S);
  if (!ODD || I == 0) return {c * SB, p.plb[I]};
  if (INR) return {q.bo[PK[I]], p.plb[OPP[I]] - (uint32_t)(CX[I] * (int)SB)};
  const bool bb = (lk >> I) & 1u;
  return {bb ? p.plb[I] + c * SB : p.plb[OPP[I]] + src_of<I>(p, q) * SB, 0u};
}
// Slot receiving q_I(x) at parity ODD.
template <int I, bool ODD, class S, bool INR = false>
__device__ __forceinline__ Slot slot_out(const Params& p, uint32_t c, uint32_t lk, const Pos& q) {
  constexpr uint32_t SB = sizeof(S);
  constexpr int J = OPP[I];
  if (!ODD || I == 0) return {c * SB, p.plb[J]};
  if (INR) return {q.bo[PK[J]], p.plb[I] + (uint32_t)(CX[I] * (int)SB)};
  const bool wall = (lk >> J) & 1u;  // x + c_I = x - c_J is not a fluid cell
  return {wall ? p.plb[J] + c * SB : p.plb[I] + src_of<J>(p, q) * SB, 0u};
}

// Pull: v_i(x) = f_i(t, x) (the cell's own opposite output across a wall; the
// open-face unknowns are then replaced by the Zou-He fill).  Unless UNI, also
// pt[j] = porosity of x + c_j (phi(x) across walls) for the producer side.
template <class S, bool SHW, bool UNI, bool ODD, bool INR = false>
__device__ __forceinline__ void pull(const Params& p, const Pop<S>& A, const float* __restrict__ phi, uint32_t c,
                                     uint32_t lk, const Pos& q, float phx, float v[Q], float pt[Q]) {
  auto ld = [&](Slot a) { return A.ld(a.v, a.s); };
  v[0] = ld(slot_in<0, ODD, S, INR>(p, c, lk, q));
  pt[0] = phx;
  sfor<1, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    constexpr int J = OPP[I];
    v[I] = ld(slot_in<I, ODD, S, INR>(p, c, lk, q));
    if (!UNI) {
      if constexpr (INR) {
        // interior: the source x - c_I is fluid, at (x, row k) shifted by -c_x
        pt[J] = ldo(phi, q.bo[PK[I]] / (uint32_t)sizeof(S) - (uint32_t)CX[I]);
      } else {
        const bool bb = (lk >> I) & 1u;
        pt[J] = ldo(phi, bb ? c : src_of<I>(p, q));
      }
    } else {
      pt[J] = phx;
    }
  });
  if (SHW) {
    const float s = p.f.ks * (phx - 1.0f);
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] -= kw(i) * s;
  }
}

// Inflow amplitude at step t, in FP64, rounded once to FP32 (the simulation
// section's pulsatile inflow and its pre-run ramp): A(t) = (t/R) W(0) during
// the ramp, W(t - R) after it; W is the sine waveform or the periodic, linearly
// interpolated sample table.
__device__ __forceinline__ float inflow_amplitude(const Params& p, const double* wave, uint32_t t) {
  double ramp = 1.0, s = 0.0;
  if (t < p.in_ramp) ramp = (double)t / (double)p.in_ramp;
  else s = (double)(t - p.in_ramp);
  double w;
  if (p.in_table > 0) {
    double ph = s / p.in_period;
    ph -= floor(ph);
    const double x = ph * (double)p.in_table;
    int i = (int)x;
    if (i >= p.in_table) i = p.in_table - 1;
    const int j = i + 1 == p.in_table ? 0 : i + 1;
    w = wave[i] + (x - (double)i) * (wave[j] - wave[i]);
  } else {
    w = p.in_a0 * (1.0 + p.in_a1 * sin(6.283185307179586 * s / p.in_period));
  }
  return (float)(ramp * w);
}

// c_s in lattice units
constexpr float CS = 0.57735026918962576f;

// Extrapolation outflow (the simulation section's non-reflecting outflow):
// each unknown population i (c_x = -1) of an outflow cell is carried out at
// the speed of sound, upwind in x and forward in time:
//   f_i(t, x) = (1 - c_s) f_i(t-1, x) + c_s f_i(t-1, x - e_x).
// Both terms are pre-collision values of the previous step, kept per row in
// side[parity of t][row][10] (FP32, relative to w_i): [0, 5) the outflow
// cell's own c_x = -1 populations, [5, 10) those of its -x neighbour (whose
// slots are rewritten during the step, hence the copy).  Without a fluid -x
// neighbour the population keeps its value.  phi = 1 on the outflow cell, so
// its deviations are relative to w_i as well.
__device__ __forceinline__ void extrapolate_out(uint32_t row, uint32_t lk, const float* __restrict__ side_in,
                                                float d[Q]) {
  const float* e = side_in + (size_t)row * 10;
  const bool up = !((lk >> 1) & 1u);  // x - e_x is fluid
#pragma unroll
  for (int k = 0; k < 5; ++k)
    if ((lk >> (LK_UNK + k)) & 1u) d[XOUT[k]] = up ? rfma(CS, e[5 + k] - e[k], e[k]) : e[k];
}

// Keep this step's c_x = -1 pre-collision populations of an outflow cell
// (after the fill) or of its -x neighbour for the next step.
__device__ __forceinline__ void outflow_keep(const Params& p, uint32_t row, uint32_t lk, float phx, const float d[Q],
                                             float* __restrict__ side_out) {
  const float s = p.f.ks * (phx - 1.0f);
  float* e = side_out + (size_t)row * 10 + ((lk & LK_OUT) ? 0 : 5);
#pragma unroll
  for (int k = 0; k < 5; ++k) e[k] = rfma(kw(XOUT[k]), s, d[XOUT[k]]);
}

// Zou-He fill of the unknown populations on the open faces (phi = 1 there, so
// the closures hold for the deviations as for the populations), or the
// extrapolation outflow.
__device__ __forceinline__ void open_fill(const Params& p, uint32_t row, uint32_t lk, uint32_t t,
                                          const float* __restrict__ shape, const double* wave,
                                          const float* __restrict__ side_in, float d[Q]) {
  const bool in = (lk & LK_IN) != 0;
  bool outl = (lk & LK_OUT) != 0;
  if (!(in || outl)) return;
  if (outl && p.outlet == 2) {
    extrapolate_out(row, lk, side_in, d);
    return;
  }
  const float U = p.f.U, iU = p.f.iU;
  const float s0 = d[0] + d[3] + d[4] + d[5] + d[6] + d[15] + d[16] + d[17] + d[18];
  const float ny_ = 0.5f * (d[3] - d[4] + d[15] - d[16] + d[17] - d[18]);
  const float nz_ = 0.5f * (d[5] - d[6] + d[15] - d[16] - d[17] + d[18]);
  // inflow: prescribed u = (ux, 0, 0); density from mass and normal momentum
  float uin = 0.0f;
  if (in) uin = inflow_amplitude(p, wave, t) * shape[row];
  const float sm = d[2] + d[8] + d[10] + d[12] + d[14];
  const float rin = (1.0f + (s0 + 2.0f * sm) * iU) / (1.0f - uin);
  // outflow: prescribed density, normal velocity from mass and the known half
  const float sp = d[1] + d[7] + d[9] + d[11] + d[13];
  const float ro = p.f.rho_out;
  const float uout = (1.0f + (s0 + 2.0f * sp) * iU) / ro - 1.0f;
  const float r3i = U * rin * uin * (1.0f / 3.0f), r6i = U * rin * uin * (1.0f / 6.0f);
  const float r3o = U * ro * uout * (1.0f / 3.0f), r6o = U * ro * uout * (1.0f / 6.0f);
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

// Whether the pull of direction I reads an open-face unknown (flags set on
// the host: source outside the inflow/outflow face, not outside a wall face).
template <int I>
__device__ __forceinline__ bool open_unknown(uint32_t lk) {
  if (CX[I] == 0) return false;
  int k = -1;
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    if ((lk & LK_IN) && XIN[j] == I) k = j;
    if ((lk & LK_OUT) && XOUT[j] == I) k = j;
  }
  return k >= 0 && ((lk >> (LK_UNK + k)) & 1u);
}

// Outer wall normal of a cell (the simulation section's WSS on the voxel
// wall): n = m / |m| with m = sum over the wall links x + c_i of 36 w_i c_i,
// a wall link being a bounce-back pull (of the opposite direction) that is not
// an open-face unknown.  False where the cell has no wall link or its links
// cancel.
__device__ __forceinline__ bool wall_normal(uint32_t lk, float n[3]) {
  int mx = 0, my = 0, mz = 0;
  sfor<1, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;  // link x + c_I, pulled by direction J from x - c_J
    constexpr int J = OPP[I];
    constexpr int k = (int)kw(I);
    if (((lk >> J) & 1u) && !open_unknown<J>(lk)) {
      mx += k * CX[I];
      my += k * CY[I];
      mz += k * CZ[I];
    }
  });
  if ((mx | my | mz) == 0) return false;
  const float il = 1.0f / __builtin_sqrtf((float)(mx * mx + my * my + mz * mz));
  n[0] = (float)mx * il;
  n[1] = (float)my * il;
  n[2] = (float)mz * il;
  return true;
}

// Symmetric 3x3 stored as xx yy zz xy xz yz, times a vector.
template <class R>
__device__ __forceinline__ void sym_mv(const R s[6], R x, R y, R z, R& ox, R& oy, R& oz) {
  ox = s[0] * x + s[3] * y + s[4] * z;
  oy = s[3] * x + s[1] * y + s[5] * z;
  oz = s[4] * x + s[5] * y + s[2] * z;
}

// Moment sums of the 19 values from opposite-pair sums and differences, in
// the arithmetic type R.
template <class R>
struct Sums {
  R s, mx, my, mz, xx, yy, zz, xy, xz, yz;
};
template <class R>
__device__ __forceinline__ Sums<R> moment_sums(const float d[Q]) {
  auto x = [&](int i) { return (R)d[i]; };
  const R P1 = x(1) + x(2), P3 = x(3) + x(4), P5 = x(5) + x(6), P7 = x(7) + x(8), P9 = x(9) + x(10),
          P11 = x(11) + x(12), P13 = x(13) + x(14), P15 = x(15) + x(16), P17 = x(17) + x(18);
  const R M1 = x(1) - x(2), M3 = x(3) - x(4), M5 = x(5) - x(6), M7 = x(7) - x(8), M9 = x(9) - x(10),
          M11 = x(11) - x(12), M13 = x(13) - x(14), M15 = x(15) - x(16), M17 = x(17) - x(18);
  Sums<R> r;
  r.s = x(0) + ((P1 + P3) + (P5 + P7)) + ((P9 + P11) + (P13 + (P15 + P17)));
  r.mx = M1 + M7 + M9 + M11 + M13;
  r.my = M3 + M7 - M9 + M15 + M17;
  r.mz = M5 + M11 - M13 + M15 - M17;
  r.xx = P1 + P7 + P9 + P11 + P13;
  r.yy = P3 + P7 + P9 + P15 + P17;
  r.zz = P5 + P11 + P13 + P15 + P17;
  r.xy = P7 - P9;
  r.xz = P11 - P13;
  r.yz = P15 - P17;
  return r;
}

// Macroscopic state of one cell for one step.
template <class R>
struct Macro {
  R rho, rm1;         // density and rho - 1
  R ux, uy, uz, uu;   // velocity
  R Fx, Fy, Fz;       // force density rho f(u)
  R P[6];             // corrected second moment Pi (xx yy zz xy xz yz)
  float shear;        // shear rate (output)
  R shear_r;          // shear rate in the arithmetic type (FP32 rheology with FP32 arithmetic)
  R cy_la, cy_fac;    // (lambda shear)^a and (1 + (lambda shear)^a)^((n-1)/a)
  R pnorm;            // |Pi|_F
  R omega;
};

// Moments, explicit velocity with drag, force, Pi, shear rate and the new
// relaxation rate from the Carreau-Yasuda viscosity.  R is the arithmetic
// type of everything that feeds the collision's mass and momentum: with FP32
// storage it is FP64, because FP32 rounding of these per-cell scalars is
// common to all 19 directions and acts as a persistent momentum source.
//
// AN: anisotropic permeability K = k M (the method section's Remark): the
// velocity is the fixed point of (A + |u| B) u = v with A = Id + (phi nu/2)
// K^-1 and B = (phi^2 C_F / 2) K^-1/2, iterated an_iters times from u_0 = v
// (each iterate one symmetric 3x3 solve by the adjugate), and the drag is
// the tensor drag -phi^2 nu K^-1 u - phi^3 C_F |u| K^-1/2 u.
// macro_sums takes the moment sums of the cell's values (any velocity set);
// macro forms them from the D3Q19 values.
//
// PF (pure fluid): phi = 1 and no body force.  Then 1/k = 0, so there is no
// drag, C0 = 1/2 and the denominator of the explicit velocity is 1, and the
// force vanishes: u = m / rho and F = 0.  The general expressions reduce to
// these mathematically (their extra terms are products with an exact zero and
// the reciprocals of 1 are 1); the compiler fuses the remaining terms of the
// two forms differently, so an output can differ in its last place.
template <class R, bool AN = false, bool PF = false>
__device__ __forceinline__ void macro_sums(const Params& p, float phx_f, const Sums<R>& s, float omega_prev,
                                           Macro<R>& M) {
  static_assert(!(PF && AN), "the pure-fluid form is the isotropic one");
  const auto& kc = p.k<R>();
  const R phx = PF ? (R)1 : (R)phx_f;
  const R one = (R)1;
  const R iphi = PF ? one : fast_rcp(phx);
  const R rm1 = PF ? s.s * kc.iU : s.s * (kc.iU * iphi);  // rho - 1
  const R rho = one + rm1;
  const R pr = PF ? rho : phx * rho;           // phi rho = sum f
  const R irho = fast_rcp(rho);
  const R iUS = PF ? kc.iU * irho : kc.iU * iphi * irho;  // 1 / (U phi rho)
  R ux, uy, uz, Fx, Fy, Fz;
  if constexpr (PF) {
    ux = s.mx * iUS; uy = s.my * iUS; uz = s.mz * iUS;
    Fx = (R)0; Fy = (R)0; Fz = (R)0;
  } else {
    const R hg = (R)0.5 * iphi;
    const R gx = kc.gx, gy = kc.gy, gz = kc.gz;
    const R vx = s.mx * iUS + gx * hg, vy = s.my * iUS + gy * hg, vz = s.mz * iUS + gz * hg;
    // 1/k = (kc/d^2) (1 - phi)^2 / phi^3
    const R om = one - phx;
    const R invk = kc.kcd * om * om * iphi * iphi * iphi;
    const R dark = phx * kc.nu_d * invk;      // phi nu / k
    if constexpr (AN) {
      const R sik = rsqrt_(invk);
      const R cf = p.forch ? (R)1.75 * rsqrt_(iphi * iphi * iphi * (R)(1.0 / 150.0)) : (R)0;
      const R ha = (R)0.5 * dark, hb = (R)0.5 * phx * phx * cf * sik;
      R Am[6], Bm[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        Am[k] = ha * kc.Mi[k] + (k < 3 ? one : (R)0);
        Bm[k] = hb * kc.Mh[k];
      }
      ux = vx; uy = vy; uz = vz;
      for (int m = 0; m < p.an_iters; ++m) {
        const R un = rsqrt_(ux * ux + uy * uy + uz * uz);
        R X[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) X[k] = rfma(un, Bm[k], Am[k]);
        // adjugate of [[X0 X3 X4] [X3 X1 X5] [X4 X5 X2]]
        const R a00 = X[1] * X[2] - X[5] * X[5], a11 = X[0] * X[2] - X[4] * X[4], a22 = X[0] * X[1] - X[3] * X[3];
        const R a01 = X[4] * X[5] - X[3] * X[2], a02 = X[3] * X[5] - X[4] * X[1], a12 = X[3] * X[4] - X[0] * X[5];
        const R idet = fast_rcp(X[0] * a00 + X[3] * a01 + X[4] * a02);
        ux = (a00 * vx + a01 * vy + a02 * vz) * idet;
        uy = (a01 * vx + a11 * vy + a12 * vz) * idet;
        uz = (a02 * vx + a12 * vy + a22 * vz) * idet;
      }
      R kdx, kdy, kdz, khx, khy, khz;
      sym_mv(kc.Mi, ux, uy, uz, kdx, kdy, kdz);
      sym_mv(kc.Mh, ux, uy, uz, khx, khy, khz);
      const R dd = phx * dark;                                          // phi^2 nu / k
      const R df = phx * phx * phx * cf * sik * rsqrt_(ux * ux + uy * uy + uz * uz);  // phi^3 C_F |u| / sqrt(k)
      Fx = rho * (gx - dd * kdx - df * khx);
      Fy = rho * (gy - dd * kdy - df * khy);
      Fz = rho * (gz - dd * kdz - df * khz);
    } else {
      const R C0 = (R)0.5 + (R)0.25 * dark;
      // drag = phi^2 nu/k + phi^3 C_F |u|/sqrt(k); the Forchheimer part stays
      // inside its branch (evaluated unconditionally it costs every cell the
      // square root's correction sequence)
      R drag = phx * dark;
      if (p.forch) {
        const R sik = rsqrt_(invk);
        const R cf = (R)1.75 * rsqrt_(iphi * iphi * iphi * (R)(1.0 / 150.0));
        const R C1 = (R)0.5 * phx * phx * cf * sik;
        const R vn = rsqrt_(vx * vx + vy * vy + vz * vz);
        const R iden = fast_rcp(C0 + rsqrt_(C0 * C0 + C1 * vn));
        ux = vx * iden; uy = vy * iden; uz = vz * iden;
        drag += phx * phx * phx * cf * sik * rsqrt_(ux * ux + uy * uy + uz * uz);
      } else {
        const R iden = fast_rcp((R)2 * C0);
        ux = vx * iden; uy = vy * iden; uz = vz * iden;
      }
      Fx = rho * (gx - drag * ux); Fy = rho * (gy - drag * uy); Fz = rho * (gz - drag * uz);
    }
  }
  const R uu = ux * ux + uy * uy + uz * uz;
  // Pi = sum (f - f_eq) c c + (F u + u F)/2
  //    = sum(v c c)/U - [phi (rho-1)/3 I + phi rho u u] + (F u + u F)/2
  const R iso = phx * rm1 * (R)(1.0 / 3.0);
  const R iU = kc.iU;
  const R h = (R)0.5;
  if constexpr (PF) {
    M.P[0] = s.xx * iU - iso - pr * ux * ux;
    M.P[1] = s.yy * iU - iso - pr * uy * uy;
    M.P[2] = s.zz * iU - iso - pr * uz * uz;
    M.P[3] = s.xy * iU - pr * ux * uy;
    M.P[4] = s.xz * iU - pr * ux * uz;
    M.P[5] = s.yz * iU - pr * uy * uz;
  } else {
    M.P[0] = s.xx * iU - iso - pr * ux * ux + Fx * ux;
    M.P[1] = s.yy * iU - iso - pr * uy * uy + Fy * uy;
    M.P[2] = s.zz * iU - iso - pr * uz * uz + Fz * uz;
    M.P[3] = s.xy * iU - pr * ux * uy + h * (Fx * uy + ux * Fy);
    M.P[4] = s.xz * iU - pr * ux * uz + h * (Fx * uz + ux * Fz);
    M.P[5] = s.yz * iU - pr * uy * uz + h * (Fy * uz + uy * Fz);
  }
  R nu;
  if constexpr (std::is_same<R, double>::value) {
    // FP64 arithmetic: the shear rate and the Carreau-Yasuda law in FP64 too
    // (the adjoint differentiates this path; FP32 transcendentals would put
    // an error of the same sign into every step's viscosity)
    const double pn = __builtin_sqrt(M.P[0] * M.P[0] + M.P[1] * M.P[1] + M.P[2] * M.P[2] +
                                     2.0 * (M.P[3] * M.P[3] + M.P[4] * M.P[4] + M.P[5] * M.P[5]));
    const double sh = 3.0 * (double)omega_prev * pn * irho;
    M.pnorm = pn;
    const double lg = kc.lam * sh;
    const double la = p.cy_a2 ? lg * lg : (lg > 0.0 ? pow_pos(lg, kc.cy_a) : 0.0);
    const double fac = pow_pos(1.0 + la, kc.cy_e);
    nu = kc.nu_inf + kc.dnu * fac;
    M.shear = (float)sh;
    M.shear_r = sh;
    M.cy_la = la;
    M.cy_fac = fac;
  } else {
    const float pn2 = (float)(M.P[0] * M.P[0] + M.P[1] * M.P[1] + M.P[2] * M.P[2] +
                              (R)2 * (M.P[3] * M.P[3] + M.P[4] * M.P[4] + M.P[5] * M.P[5]));
    // |Pi|_F to one ulp (the hardware square root)
    const float pn = __builtin_amdgcn_sqrtf(pn2);
    const float shear = 3.0f * omega_prev * pn * (float)irho;
    M.pnorm = (R)pn;
    // Carreau-Yasuda: nu = nu_inf + (nu0 - nu_inf) (1 + (lambda g)^a)^((n-1)/a)
    const float lg = p.f.lam * shear;
    float la;
    if (p.cy_a2) la = lg * lg;
    else la = lg > 0.0f ? __builtin_amdgcn_exp2f(p.f.cy_a * __builtin_amdgcn_logf(lg)) : 0.0f;
    const float fac = __builtin_amdgcn_exp2f(p.f.cy_e * __builtin_amdgcn_logf(1.0f + la));
    nu = kc.nu_inf + kc.dnu * (R)fac;
    M.shear = shear;
    M.shear_r = (R)shear;
    M.cy_la = (R)la;
    M.cy_fac = (R)fac;
  }
  // omega = 2 rho c_s^2 / (2 mu + rho c_s^2) = 2 rho / (6 nu + rho)
  M.omega = (R)2 * rho * fast_rcp((R)6 * nu + rho);
  M.rho = rho;
  M.rm1 = rm1;
  M.ux = ux; M.uy = uy; M.uz = uz; M.uu = uu;
  M.Fx = Fx; M.Fy = Fy; M.Fz = Fz;
}
template <class R, bool AN = false, bool PF = false>
__device__ __forceinline__ void macro(const Params& p, float phx_f, const float d[Q], float omega_prev, Macro<R>& M) {
  macro_sums<R, AN, PF>(p, phx_f, moment_sums<R>(d), omega_prev, M);
}

// Wall shear stress tau = sigma n - (n . sigma n) n of a wall cell, with the
// deviatoric stress sigma = (omega/2 - 1) Pi of this step; returns |tau|.
template <class R>
__device__ __forceinline__ R wall_tau(const Macro<R>& M, const float n[3], R tau[3]) {
  const R s = (R)0.5 * M.omega - (R)1;
  const R nx = (R)n[0], ny = (R)n[1], nz = (R)n[2];
  R sx, sy, sz;
  sym_mv(M.P, nx, ny, nz, sx, sy, sz);
  sx *= s; sy *= s; sz *= s;
  const R nsn = sx * nx + sy * ny + sz * nz;
  tau[0] = sx - nsn * nx;
  tau[1] = sy - nsn * ny;
  tau[2] = sz - nsn * nz;
  return rsqrt_(tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2]);
}

// |tau| of a region wall cell, 0 elsewhere (the WSS objective's cell term).
template <class R>
__device__ __forceinline__ R region_wss(uint32_t lk, const Macro<R>& M) {
  float n[3];
  if (!(lk & LK_REG) || !wall_normal(lk, n)) return (R)0;
  R tau[3];
  return wall_tau(M, n, tau);
}

// Rounding of the 16-bit storage forms (RM):
//   0 nearest: every value rounds to nearest even on its own;
//   1 conserving: every value is rounded to nearest except that the rounding
//     residuals of the cell's mass and momentum are carried.  The non-axis
//     values (directions 7.. in opposite pairs) are rounded first; their
//     momentum residual moves onto the three axis pairs (as pair differences,
//     which carry no mass) before those are rounded; the whole mass residual
//     moves onto the rest value, rounded last.  The cell's stored mass and
//     momentum each carry one rounding instead of the sum of all of them;
//   2 stochastic: every value rounds up or down with probabilities given by
//     its distance to the two neighbours (the hardware's stochastic-rounding
//     conversion, v_cvt_sr), so every rounding error has mean zero.
// Deterministic rounding of a smooth, nearly periodic flow makes the same
// error at the same place step after step: a steady forcing, which the slowly
// damped modes at an open face integrate (the staggered velocity mode next to
// a constant-density outflow grows to ~1e-4 of u in 20 000 steps).  Stochastic
// rounding turns that forcing into zero-mean noise.  Works for any velocity set
// ordered rest, axis pairs, then opposite pairs.
//
// Random bits: a per-(cell, step) word A from an integer hash (the "lowbias32"
// finaliser of C. Wellons' hash-prospector) and B, one step of Marsaglia's
// xorshift32 from A.  Opposite pair k takes the word A ^ rotr(B, SR_ROT[k]),
// the rest value the word after the last pair (the conversion reads the top 13
// bits for FP16, the top 16 for BF16, so the word shifted left by 13 or 16
// serves the pair's second value): two instructions a word.  All the words are
// GF(2)-linear in A; the rotations are chosen so that every two FP16 windows
// of a cell (13 bits each, 19 or 27 of them) are jointly of full rank 26,
// i.e. pairwise independent and uniform, which is what the variance of the
// cell's summed rounding errors depends on.  (Two 16-bit BF16 windows would
// need all 32 bits; some pairs share a linear relation, as they do along the
// xorshift sequence itself.)
__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
__device__ __forceinline__ uint32_t xorshift32(uint32_t x) {
  x ^= x << 13;
  x ^= x >> 17;
  x ^= x << 5;
  return x;
}
// The word A of cell c at step t.
__device__ __forceinline__ uint32_t round_seed(uint32_t c, uint32_t t) {
  return hash32(c ^ hash32(t * 0x9e3779b9u + 0x632be5abu));
}
constexpr int SR_ROT[14] = {3, 8, 18, 7, 21, 31, 24, 16, 4, 15, 23, 12, 20, 5};
__device__ __forceinline__ uint32_t rotr32(uint32_t x, int r) { return r ? (x >> r) | (x << (32 - r)) : x; }
// v rounded stochastically to S (FP16 or BF16) with the random word r.
template <class S>
__device__ __forceinline__ unsigned short round_sr(float v, uint32_t r) {
  // the conversion writes one half of a register and keeps the other; only
  // the low half is used, so the conversion overwrites the input's own
  // register rather than a cleared one (no move)
  if constexpr (std::is_same<S, _Float16>::value) {
    typedef _Float16 v2 __attribute__((ext_vector_type(2)));
    v2 a = __builtin_bit_cast(v2, v);
    a = __builtin_amdgcn_cvt_sr_f16_f32(a, v, r, false);
    return __builtin_bit_cast(unsigned short, a[0]);
  } else {
    typedef __bf16 v2 __attribute__((ext_vector_type(2)));
    v2 a = __builtin_bit_cast(v2, v);
    a = __builtin_amdgcn_cvt_sr_bf16_f32(a, v, r, false);
    return __builtin_bit_cast(unsigned short, a[0]);
  }
}
template <class S, int NQ, int RM>
__device__ __forceinline__ void round16(const int (&cx)[NQ], const int (&cy)[NQ], const int (&cz)[NQ],
                                        const float o[NQ], unsigned short hb[NQ], uint32_t seed) {
  constexpr bool SR = RM == 2;
  constexpr int SH = std::is_same<S, _Float16>::value ? 13 : 16;  // second window of a random word
  const uint32_t sb = SR ? xorshift32(seed) : 0u;
  int iw = 0;
  // the next random word (unused without stochastic rounding)
  auto word = [&]() -> uint32_t {
    if constexpr (SR) {
      return seed ^ rotr32(sb, SR_ROT[iw++]);
    } else {
      return 0u;
    }
  };
  // hb[i] = v rounded in S; returns the residual (exact in FP32)
  auto rn = [&](int i, float v, uint32_t r) {
    unsigned short h;
    if constexpr (SR) h = round_sr<S>(v, r);
    else h = __builtin_bit_cast(unsigned short, (S)v);
    hb[i] = h;
    return v - (float)__builtin_bit_cast(S, h);
  };
  if constexpr (RM != 1) {
    sfor<0, (NQ - 1) / 2>([&](auto kc) {
      constexpr int I = 1 + 2 * decltype(kc)::value;
      const uint32_t r = word();
      rn(I, o[I], r);
      rn(I + 1, o[I + 1], r << SH);
    });
    rn(0, o[0], word());
    return;
  }
  float m = 0.0f, rx = 0.0f, ry = 0.0f, rz = 0.0f;
  // the pair sum carries mass, the difference momentum along c_I
  sfor<0, (NQ - 7) / 2>([&](auto kc) {
    constexpr int I = 7 + 2 * decltype(kc)::value;
    const uint32_t r = word();
    const float a = rn(I, o[I], r), b = rn(I + 1, o[I + 1], r << SH);
    m += a + b;
    const float d = a - b;
    if (cx[I]) rx += cx[I] > 0 ? d : -d;
    if (cy[I]) ry += cy[I] > 0 ? d : -d;
    if (cz[I]) rz += cz[I] > 0 ? d : -d;
  });
  uint32_t r = word();
  m += rn(1, o[1] + 0.5f * rx, r);
  m += rn(2, o[2] - 0.5f * rx, r << SH);
  r = word();
  m += rn(3, o[3] + 0.5f * ry, r);
  m += rn(4, o[4] - 0.5f * ry, r << SH);
  r = word();
  m += rn(5, o[5] + 0.5f * rz, r);
  m += rn(6, o[6] - 0.5f * rz, r << SH);
  rn(0, o[0] + m, word());
}

// BGK + Guo + porosity-jump collision, stored as deviations for the consumer.
// Directions come in opposite pairs: with e = c.u and h = c.F the even part
// (omega (A0 + C e^2) - K3 u.F + K9 e h) is shared and the odd part
// (omega B e + K3 h) flips sign; both are per unit weight, scaled by the exact
// U w_i.
//
// PROJ (FP32 arithmetic with FP32 storage): rounding of the per-cell scalars
// (u, omega, ...) is common to all 19 directions, so the collision's momentum
// change picks up a small relative error that repeats every step and
// accumulates in slowly evolving flows.  The projection evaluates, in FP64 on
// the FP32 values, the momentum the outputs actually carry and moves the
// difference to the intended momentum (input momentum + force + porosity-jump
// momentum) onto the three axis pairs, leaving only the final rounding of
// each stored value.
// collide_values: the outputs, in place of the pulled values d; collide_store
// also rounds and stores them.
// PF (pure fluid, see macro_sums; implies UNI): F = 0 and phi = 1, so the Guo
// term and the terms in u.F and c.F vanish exactly.
template <bool SHW, bool UNI, class R, bool PROJ, bool PF = false>
__device__ __forceinline__ void collide_values(const Params& p, float phx_f, float d[Q], const float pt[Q],
                                               const Macro<R>& M) {
  static_assert(!PF || UNI, "a pure-fluid wave has uniform porosity");
  const R phx = PF ? (R)1 : (R)phx_f;
  const R om = M.omega;
  const R pr = phx * M.rho;
  const R A0 = phx * M.rm1 - (R)1.5 * pr * M.uu;
  const R Bc = (R)3 * pr, Cc = (R)4.5 * pr;
  const R K = (R)1 - (R)0.5 * om;
  const R K3 = (R)3 * K, K9 = (R)9 * K;
  const R uF = M.ux * M.Fx + M.uy * M.Fy + M.uz * M.Fz;
  const R keep = (R)1 - om;
  const R ev0 = PF ? om * A0 : om * A0 - K3 * uF;
  const R ks = p.k<R>().ks;
  // U w_i = ks kw(i) takes two values on the moving directions (axis 2 ks,
  // edge ks): fold it into the per-pair constants once
  const R ka = ks * (R)kw(1), ke = ks * (R)kw(7);
  const R omC = om * Cc, omB = om * Bc;
  const R ev0a = ka * ev0, omCa = ka * omC, K9a = ka * K9, omBa = ka * omB, K3a = ka * K3;
  const R ev0e = ke * ev0, omCe = ke * omC, K9e = ke * K9, omBe = ke * omB, K3e = ke * K3;
  // porosity-jump term per unit weight: (rho - 1)(phi~_i - phi)
  auto jump = [&](int i) -> R { return UNI ? (R)0 : M.rm1 * ((R)pt[i] - phx); };
  // the projection's input momentum, taken before the outputs overwrite d[]
  double tmx = 0.0, tmy = 0.0, tmz = 0.0;
  if constexpr (PROJ) {
    const Sums<double> si = moment_sums<double>(d);
    tmx = si.mx; tmy = si.my; tmz = si.mz;
  }
  float* o = d;
  o[0] = (float)rfma(ks * (R)kw(0), ev0 + jump(0), keep * (R)d[0]);
  auto pair = [&](auto ic, R e, R h) {
    constexpr int I = decltype(ic)::value;
    constexpr int J = OPP[I];
    constexpr bool AX = I < 7;
    const R kk = AX ? ka : ke;
    const R ev = PF ? rfma(AX ? omCa : omCe, e * e, AX ? ev0a : ev0e)
                    : rfma(AX ? omCa : omCe, e * e, rfma(AX ? K9a : K9e, e * h, AX ? ev0a : ev0e));
    const R od = PF ? (AX ? omBa : omBe) * e : rfma(AX ? omBa : omBe, e, (AX ? K3a : K3e) * h);
    if (UNI) {
      o[I] = (float)rfma(keep, (R)d[I], ev + od);
      o[J] = (float)rfma(keep, (R)d[J], ev - od);
    } else {
      o[I] = (float)rfma(keep, (R)d[I], ev + od + kk * jump(I));
      o[J] = (float)rfma(keep, (R)d[J], ev - od + kk * jump(J));
    }
  };
  pair(std::integral_constant<int, 1>{}, M.ux, M.Fx);
  pair(std::integral_constant<int, 3>{}, M.uy, M.Fy);
  pair(std::integral_constant<int, 5>{}, M.uz, M.Fz);
  pair(std::integral_constant<int, 7>{}, M.ux + M.uy, PF ? (R)0 : M.Fx + M.Fy);
  pair(std::integral_constant<int, 9>{}, M.ux - M.uy, PF ? (R)0 : M.Fx - M.Fy);
  pair(std::integral_constant<int, 11>{}, M.ux + M.uz, PF ? (R)0 : M.Fx + M.Fz);
  pair(std::integral_constant<int, 13>{}, M.ux - M.uz, PF ? (R)0 : M.Fx - M.Fz);
  pair(std::integral_constant<int, 15>{}, M.uy + M.uz, PF ? (R)0 : M.Fy + M.Fz);
  pair(std::integral_constant<int, 17>{}, M.uy - M.uz, PF ? (R)0 : M.Fy - M.Fz);
  if constexpr (PROJ) {
    // momentum in and out (pair differences are exact in FP64)
    const Sums<double> so = moment_sums<double>(o);
    const double U = p.d.U;
    double tx = tmx, ty = tmy, tz = tmz;
    if (!PF) {
      tx += U * (double)M.Fx; ty += U * (double)M.Fy; tz += U * (double)M.Fz;
    }
    if (!UNI) {
      const double rm1 = (double)M.rm1, ph = (double)phx_f;
      double jx = 0.0, jy = 0.0, jz = 0.0;
      sfor<1, Q>([&](auto ic) {
        constexpr int I = decltype(ic)::value;
        const double jt = (double)kw(I) * ((double)pt[I] - ph);
        if (CX[I]) jx += CX[I] * jt;
        if (CY[I]) jy += CY[I] * jt;
        if (CZ[I]) jz += CZ[I] * jt;
      });
      const double kr = p.d.ks * rm1;
      tx += kr * jx; ty += kr * jy; tz += kr * jz;
    }
    // the axis pairs carry 2 (U w) = 2 ks * 2 per unit change of f_i - f_opp
    const double rx = 0.5 * (tx - so.mx), ry = 0.5 * (ty - so.my), rz = 0.5 * (tz - so.mz);
    o[1] = (float)((double)o[1] + rx); o[2] = (float)((double)o[2] - rx);
    o[3] = (float)((double)o[3] + ry); o[4] = (float)((double)o[4] - ry);
    o[5] = (float)((double)o[5] + rz); o[6] = (float)((double)o[6] - rz);
  }
  if (SHW && !PF) {
    // stored relative to w_i instead of w_i phi~_i (phi = 1: no change)
    const float ksf = p.f.ks;
#pragma unroll
    for (int i = 0; i < Q; ++i) o[i] += ksf * kw(i) * ((UNI ? phx_f : pt[i]) - 1.0f);
  }
}

template <class S, bool SHW, bool UNI, bool ODD, class R, bool PROJ, bool INR = false, int RM = 0, bool PF = false>
__device__ __forceinline__ void collide_store(const Params& p, const Pop<S>& A, uint32_t c, uint32_t lk, const Pos& q,
                                              float phx_f, float d[Q], const float pt[Q], const Macro<R>& M,
                                              uint32_t seed = 0u) {
  collide_values<SHW, UNI, R, PROJ, PF>(p, phx_f, d, pt, M);
  const float* o = d;
  if constexpr (!std::is_same<S, float>::value && RM != 0) {
    unsigned short hb[Q];
    round16<S, Q, RM>(CX, CY, CZ, o, hb, seed);
    sfor<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      const Slot a = slot_out<I, ODD, S, INR>(p, c, lk, q);
      A.st_bits(a.v, a.s, hb[I]);
    });
  } else {
    sfor<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      const Slot a = slot_out<I, ODD, S, INR>(p, c, lk, q);
      A.st(a.v, a.s, o[I]);
    });
  }
}

// ---------------------------------------------------------------------------
// Block reduction of FP64 partials: wave64 shuffle, then LDS across the 4 waves.
// ---------------------------------------------------------------------------
template <int N, int NT = BLOCK>
__device__ __forceinline__ void block_reduce(double (&v)[N], const int (&op)[N], double* out) {
  __shared__ double sh[NT / 64][N];
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
    for (int w = 1; w < NT / 64; ++w)
      r = op[k] == 0 ? r + sh[w][k] : (op[k] == 1 ? fmax(r, sh[w][k]) : fmin(r, sh[w][k]));
    out[k] = r;
  }
}

// Per-cell diagnostic contributions: mass, momentum, energy, region energy,
// max |u|, min/max omega, non-finite count, region wall shear stress |tau|.
template <class R>
__device__ __forceinline__ void diag_terms(const Params& p, float phx, const float d[Q], const Macro<R>& M, uint32_t lk,
                                           bool active, double (&v)[NDIAGP]) {
  const bool reg = (lk & LK_REG) != 0;
  if (!active) {
    v[0] = v[1] = v[2] = v[3] = v[4] = v[5] = v[9] = v[10] = 0.0;
    v[6] = 0.0; v[7] = 1e300; v[8] = -1e300;
    return;
  }
  const Sums<double> s = moment_sums<double>(d);
  v[0] = (double)phx + s.s * p.d.iU;
  v[1] = s.mx * p.d.iU;
  v[2] = s.my * p.d.iU;
  v[3] = s.mz * p.d.iU;
  const double ke = 0.5 * (double)M.rho * (double)M.uu;
  v[4] = ke;
  v[5] = reg ? ke : 0.0;
  v[6] = __builtin_sqrt((double)M.uu);
  v[7] = (double)M.omega;
  v[8] = (double)M.omega;
  const bool bad = !(__builtin_isfinite((double)M.rho) && __builtin_isfinite((double)M.uu) &&
                     __builtin_isfinite((double)M.omega) && __builtin_isfinite(M.shear));
  v[9] = bad ? 1.0 : 0.0;
  if (bad) { v[6] = 1e300; }
  v[10] = (double)region_wss<R>(lk, M);
}

// Body of the step for one cell (UNI: the whole wave has uniform neighbour
// porosity; INR: every cell of the wave is interior; RM: rounding of 16-bit
// storage, see round16).
template <class S, bool SHW, bool UNI, bool ODD, int DIAG, bool REC, class R, bool PROJ, bool AN, bool INR, int RM,
          bool PL = false, bool PF = false>
__device__ __forceinline__ void step_cell(const Params& p, const Bufs& b, uint32_t c, uint32_t lk, uint32_t t,
                                          float phx, double (&dv)[NDIAGP], float& ke_reg, uint32_t row = 0u) {
  Pos q;
  if constexpr (PL) {
    // a plain wave (lk synthesised: uniform, interior on odd steps) or a
    // non-uniform interior one; row given
    q.row = row;
    if constexpr (ODD || !UNI) {
      const int4* r4 = (const int4*)(b.rel + (size_t)row * 8);
      const int4 a = r4[0], e = r4[1];
      const int rl[NPAIR] = {0, a.x, a.y, a.z, a.w, e.x, e.y, e.z, e.w};
#pragma unroll
      for (int k = 0; k < NPAIR; ++k) q.bo[k] = (c + (uint32_t)rl[k]) * (uint32_t)sizeof(S);
    }
  } else {
    // an even step of a uniform-porosity cell touches only its own slots: its
    // position is needed only for an open-face row's data
    const bool where = ODD || !UNI || (lk & (LK_IN | LK_OUT | LK_UPS));
    q = position(p, c, where ? b.code[c] : 0u);
    if (ODD || !UNI) load_deltas(b.delta, q);
    if (INR) interior_offsets<S>(q);
  }
  float d[Q], pt[Q];
  const Pop<S> A(b.A, p.abytes);
  pull<S, SHW, UNI, ODD, INR>(p, A, b.phi, c, lk, q, phx, d, pt);
  const size_t half = (size_t)p.nrow * 10;
  open_fill(p, q.row, lk, t, b.shape, b.wave, b.side + (ODD ? half : 0), d);
  if (REC) {
    // the segment record (after the open-face fill, so that it holds the
    // extrapolation outflow's unknowns) is read once, by the reverse step:
    // stream it past the caches
#pragma unroll
    for (int i = 0; i < Q; ++i) __builtin_nontemporal_store(d[i], &b.rec[(size_t)i * p.nc + c]);
  }
  if (p.outlet == 2 && (lk & (LK_OUT | LK_UPS))) outflow_keep(p, q.row, lk, phx, d, b.side + (ODD ? 0 : half));
  const float omp = b.omega[c];
  Macro<R> M;
  macro<R, AN, PF>(p, phx, d, omp, M);
  b.omega[c] = (float)M.omega;
  if (REC) {
    __builtin_nontemporal_store(omp, &b.rec[(size_t)Q * p.nc + c]);
    __builtin_nontemporal_store((float)M.rho, &b.rho_rec[c]);
  }
  const bool reg = (lk & LK_REG) != 0;
  if (DIAG == 1) diag_terms<R>(p, phx, d, M, lk, true, dv);
  if (DIAG == 2) ke_reg = reg ? (float)((R)0.5 * M.rho * M.uu) : 0.0f;
  if (DIAG == 3) ke_reg = (float)region_wss<R>(lk, M);
  collide_store<S, SHW, UNI, ODD, R, PROJ, INR, RM, PF>(p, A, c, lk, q, phx, d, pt, M,
                                                        RM == 2 ? round_seed(c, t) : 0u);
}

// Whether the pure-fluid form serves this wave: the plain step (FP32
// arithmetic, isotropic, no diagnostics or record), no body force, and
// porosity 1 at every active lane.
template <int DIAG, bool REC, class R, bool AN>
constexpr bool pure_form() {
  return DIAG == 0 && !REC && !AN && std::is_same<R, float>::value;
}
template <int DIAG, bool REC, class R, bool AN>
__device__ __forceinline__ bool pure_wave(const Params& p, bool active, float phx) {
  if constexpr (!pure_form<DIAG, REC, R, AN>()) {
    return false;
  } else {
    return p.f.gx == 0.0f && p.f.gy == 0.0f && p.f.gz == 0.0f && __all(!active || phx == 1.0f);
  }
}

// The step of cell c (any cell of the compact range or past it) through its
// link word, with the wave-uniform choice of the uniform-porosity and
// interior forms; returns whether c is a fluid cell.  Every lane of the wave
// takes part.
template <class S, bool SHW, bool ODD, int DIAG, bool REC, class R, bool PROJ, bool AN, int RM>
__device__ __forceinline__ bool step_any(const Params& p, const Bufs& b, uint32_t c, uint32_t t,
                                         double (&dv)[NDIAGP], float& ke_reg) {
  const uint32_t lk = c < (uint32_t)p.nc ? b.links[c] : LK_DEAD;
  const bool active = !(lk & LK_DEAD);
  const bool uni = !active || (lk & LK_UNI);
  const float phx = active ? ldo(b.phi, c) : 1.0f;
  if (__all(uni)) {
    // odd steps address the neighbours: interior waves (most of a vessel's
    // waves) need no per-direction bounce-back selects
    constexpr bool PFK = pure_form<DIAG, REC, R, AN>();
    const bool pf = pure_wave<DIAG, REC, R, AN>(p, active, phx);
    if (ODD && __all(!active || (lk & LK_INR))) {
      if (pf) {
        if (active)
          step_cell<S, SHW, true, ODD, DIAG, REC, R, PROJ, AN, true, RM, false, PFK>(p, b, c, lk, t, phx, dv, ke_reg);
      } else {
        if (active) step_cell<S, SHW, true, ODD, DIAG, REC, R, PROJ, AN, true, RM>(p, b, c, lk, t, phx, dv, ke_reg);
      }
    } else {
      if (pf) {
        if (active)
          step_cell<S, SHW, true, ODD, DIAG, REC, R, PROJ, AN, false, RM, false, PFK>(p, b, c, lk, t, phx, dv,
                                                                                      ke_reg);
      } else {
        if (active) step_cell<S, SHW, true, ODD, DIAG, REC, R, PROJ, AN, false, RM>(p, b, c, lk, t, phx, dv, ke_reg);
      }
    }
  } else {
    if (active) step_cell<S, SHW, false, ODD, DIAG, REC, R, PROJ, AN, false, RM>(p, b, c, lk, t, phx, dv, ke_reg);
  }
  return active;
}

// ---------------------------------------------------------------------------
// The step at parity ODD (t odd), NT work-items per workgroup.  DIAG: 0 none,
// 1 diagnostics of the pre-collision state into part[block][NDIAGP], 2 region
// kinetic energy, 3 region wall shear stress |tau|, accumulated into
// part[block].  REC: also record the pulled
// values and omega_prev ([20][nc]) and rho.
// ---------------------------------------------------------------------------
// The 16-bit odd step needs 97 VGPRs as compiled freely (4 waves per SIMD);
// asked for 5 waves the compiler fits it in 96 without scratch, and the step
// runs 1-2 % faster.  The FP32-arithmetic step is asked for 4 waves: compiled
// freely its odd step spills 20 bytes per lane.  Other instantiations would
// spill at these targets and keep the default.
// WR: the wave records are used (always with FP32 storage; the 16-bit steps
// take them only when the state exceeds the Infinity Cache: on a cache-resident
// state the record lookup in front of their loads costs more than the bytes it
// saves).
template <class S, bool SHW, bool ODD, int DIAG, bool REC, class R, bool PROJ, int NT, bool AN = false, int RM = 0,
          bool WR = sizeof(S) == 4>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu((ODD && sizeof(S) == 2 && DIAG == 0 && !REC) ? 5 : (sizeof(S) == 4 && DIAG == 0 && !REC && std::is_same<R, float>::value && !AN ? 4 : 1))))
void k_step(Params p, Bufs b) {
  const uint32_t c = xcd_block(blockIdx.x, gridDim.x) * NT + threadIdx.x;
  const uint32_t t = b.tc[ODD ? 1 : 0];
  double dv[NDIAGP];
  float ke_reg = 0.0f;
  if constexpr (DIAG == 0 && WR) {
    const WaveInfo wi = b.winfo[__builtin_amdgcn_readfirstlane(c >> 6)];
    if (wi.flags & WV_FLUID) {
      const bool uni = (wi.flags & WV_UNI) != 0, inr = (wi.flags & WV_INR) != 0;
      if (uni ? (!ODD || inr) : inr) {
        const uint32_t lane = threadIdx.x & 63u;
        const uint32_t row = wi.row0 + (uint32_t)__popcll(wi.starts & ((2ull << lane) - 2ull));
        const float phx = ldo(b.phi, c);
        constexpr uint32_t LKU = LK_UNI | (ODD ? LK_INR : 0u);
        constexpr bool PFK = pure_form<DIAG, REC, R, AN>();
        if (uni && pure_wave<DIAG, REC, R, AN>(p, true, phx))
          step_cell<S, SHW, true, ODD, DIAG, REC, R, PROJ, AN, ODD, RM, true, PFK>(p, b, c, LKU, t, phx, dv, ke_reg,
                                                                                     row);
        else if (uni)
          step_cell<S, SHW, true, ODD, DIAG, REC, R, PROJ, AN, ODD, RM, true>(p, b, c, LKU, t, phx, dv, ke_reg, row);
        else
          step_cell<S, SHW, false, ODD, DIAG, REC, R, PROJ, AN, true, RM, true>(p, b, c, LK_INR, t, phx, dv, ke_reg,
                                                                                row);
        if (blockIdx.x == 0 && threadIdx.x == 0) b.tc[ODD ? 0 : 1] = t + 1u;
        return;
      }
    }
  }
  const bool active = step_any<S, SHW, ODD, DIAG, REC, R, PROJ, AN, RM>(p, b, c, t, dv, ke_reg);
  if (DIAG == 1) {
    if (!active) {
      float d[Q] = {};
      Macro<R> M{};
      diag_terms<R>(p, 0.f, d, M, 0u, false, dv);
    }
    const int ops[NDIAGP] = {0, 0, 0, 0, 0, 0, 1, 2, 1, 0, 0};
    block_reduce<NDIAGP, NT>(dv, ops, b.part + (size_t)blockIdx.x * NDIAGP);
  }
  if (DIAG >= 2) {
    double v[1] = {(double)ke_reg};
    const int ops[1] = {0};
    __shared__ double tmp[1];
    block_reduce<1, NT>(v, ops, tmp);
    if (threadIdx.x == 0) b.part[blockIdx.x] += tmp[0];
  }
  // the next step (the other parity) reads t + 1 from the other slot
  if (blockIdx.x == 0 && threadIdx.x == 0) b.tc[ODD ? 0 : 1] = t + 1u;
}

// Moments of the current state (no collision): dense box outputs (any may be
// null) and optionally the diagnostics partials.
template <class S, bool SHW, bool ODD, bool DIAG, class R, bool AN = false>
__global__ __launch_bounds__(BLOCK) void k_moments(Params p, Bufs b, uint32_t t, size_t nbox, float* rho_o,
                                                    float* u_o, float* shear_o, float* omega_o, float* sigma_o,
                                                    float* tau_o) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  const uint32_t lk = c < (uint32_t)p.nc ? b.links[c] : LK_DEAD;
  const bool active = !(lk & LK_DEAD);
  double dv[NDIAGP];
  if (active) {
    Pos q = position(p, c, b.code[c]);
    if (ODD) load_deltas(b.delta, q);
    const float phx = ldo(b.phi, c);
    float d[Q], pt[Q];
    pull<S, SHW, true, ODD>(p, Pop<S>(b.A, p.abytes), b.phi, c, lk, q, phx, d, pt);
    open_fill(p, q.row, lk, t, b.shape, b.wave, b.side + (ODD ? (size_t)p.nrow * 10 : 0), d);
    Macro<R> M;
    macro<R, AN>(p, phx, d, b.omega[c], M);
    const size_t idx = (size_t)b.rowbox[q.row] + (size_t)q.x;
    if (rho_o) rho_o[idx] = (float)M.rho;
    if (u_o) {
      u_o[idx] = (float)M.ux;
      u_o[nbox + idx] = (float)M.uy;
      u_o[2 * nbox + idx] = (float)M.uz;
    }
    if (shear_o) shear_o[idx] = M.shear;
    if (omega_o) omega_o[idx] = (float)M.omega;
    if (sigma_o) {
      const R s = (R)0.5 * M.omega - (R)1;
#pragma unroll
      for (int k = 0; k < 6; ++k) sigma_o[(size_t)k * nbox + idx] = (float)(s * M.P[k]);
    }
    if (tau_o) {
      float n[3];
      R tw[3] = {(R)0, (R)0, (R)0};
      if (wall_normal(lk, n)) wall_tau(M, n, tw);
#pragma unroll
      for (int a = 0; a < 3; ++a) tau_o[(size_t)a * nbox + idx] = (float)tw[a];
    }
    if (DIAG) diag_terms<R>(p, phx, d, M, lk, true, dv);
  } else if (DIAG) {
    float d[Q] = {};
    Macro<R> M{};
    diag_terms<R>(p, 0.f, d, M, 0u, false, dv);
  }
  if (DIAG) {
    const int ops[NDIAGP] = {0, 0, 0, 0, 0, 0, 1, 2, 1, 0, 0};
    block_reduce<NDIAGP>(dv, ops, b.part + (size_t)blockIdx.x * NDIAGP);
  }
}

// Rest state at even parity: slot (i, x) holds f_i(x) = w_i phi(x), which is
// 0 in shift mode 0 and U w_i (phi(x) - 1) in shift mode 1.
template <class S, bool SHW>
__global__ __launch_bounds__(BLOCK) void k_init(Params p, Bufs b, float omega0) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= (uint32_t)p.nc) return;
  if (b.links[c] & LK_DEAD) return;
  const float phx = ldo(b.phi, c);
  const Pop<S> A(b.A, p.abytes);
  const float ks = p.f.ks;
#pragma unroll
  for (int i = 0; i < Q; ++i) A.st(c * (uint32_t)sizeof(S), p.plb[i], SHW ? ks * kw(i) * (phx - 1.0f) : 0.0f);
  b.omega[c] = omega0;
  if (c == 0) b.tc[0] = 0u;
}

// Whether the state keeps the open-face unknown I: the extrapolation outflow's.
template <int I>
__device__ __forceinline__ bool kept_unknown(const Params& p, uint32_t lk) {
  return CX[I] == -1 && (lk & LK_OUT) && p.outlet == 2;
}

// State out: the pulled (pre-collision) stored values as FP32, [19][nc]; the
// host converts them back to populations in FP64.  Open-face unknowns are NaN,
// except the extrapolation outflow's, which are part of the state: their
// value at time t is extrapolated as the next step would.
template <class S, bool ODD>
__global__ __launch_bounds__(BLOCK) void k_gather_state(Params p, Bufs b, float* out) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= (uint32_t)p.nc) return;
  const uint32_t lk = b.links[c];
  if (lk & LK_DEAD) return;
  Pos q = position(p, c, b.code[c]);
  if (ODD) load_deltas(b.delta, q);
  const Pop<S> A(b.A, p.abytes);
  float d[Q];
  sfor<0, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    const Slot a = slot_in<I, ODD, S>(p, c, lk, q);
    d[I] = A.ld(a.v, a.s);
  });
  if ((lk & LK_OUT) && p.outlet == 2) extrapolate_out(q.row, lk, b.side + (ODD ? (size_t)p.nrow * 10 : 0), d);
  sfor<0, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    const bool unk = open_unknown<I>(lk) && !kept_unknown<I>(p, lk);
    out[(size_t)I * p.nc + c] = unk ? __builtin_nanf("") : d[I];
  });
}

// State in: inverse of k_gather_state; each slot that some consumer reads is
// written exactly once (by that consumer's link).  A kept unknown of the
// extrapolation outflow goes to both side values, so that the next step's
// extrapolation returns it.
template <class S, bool ODD>
__global__ __launch_bounds__(BLOCK) void k_scatter_state(Params p, Bufs b, const float* in) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= (uint32_t)p.nc) return;
  const uint32_t lk = b.links[c];
  if (lk & LK_DEAD) return;
  Pos q = position(p, c, b.code[c]);
  if (ODD) load_deltas(b.delta, q);
  const Pop<S> A(b.A, p.abytes);
  sfor<0, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    const Slot a = slot_in<I, ODD, S>(p, c, lk, q);
    const float v = in[(size_t)I * p.nc + c];
    if (kept_unknown<I>(p, lk) && open_unknown<I>(lk)) {
      int k = 0;
#pragma unroll
      for (int j = 0; j < 5; ++j) k = XOUT[j] == I ? j : k;
      float* e = b.side + (ODD ? (size_t)p.nrow * 10 : 0) + (size_t)q.row * 10;
      e[k] = v;
      e[5 + k] = v;
    } else if (!open_unknown<I>(lk)) {
      A.st(a.v, a.s, v);
    }
  });
}

}  // namespace lbm
