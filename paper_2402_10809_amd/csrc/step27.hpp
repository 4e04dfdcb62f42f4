// The step on the D3Q27 velocity set (the method section's lattice): the same
// scheme as step.hpp (compact rows, in-place AA streaming, stored scaled
// deviations, BGK + Guo + porosity-jump collision, Carreau-Yasuda relaxation,
// open faces), written once for 27 directions with loops over the directions
// and over the 13 opposite pairs that the compiler unrolls.  The
// moments-to-relaxation part (macro_sums) is shared with the D3Q19 kernels.
//
// Differences from D3Q19:
//   - weights 8/27, 2/27, 1/54, 1/216; the storage unit U is a multiple of
//     216, so U w_i is an exact integer (64, 16, 4, 1 times U/216);
//   - the link word is 64 bits: bit 0 dead slot, bits 1..26 bounce-back of the
//     pull of direction i, 27 uniform neighbour porosity, 28 inflow, 29
//     outflow, 30 region, 31 -x neighbour of an extrapolation-outflow cell,
//     bits 32..40 which of the nine x-directed pulls are open-face unknowns;
//   - the Zou-He faces fill nine unknowns with a weight-proportional
//     transverse correction: d_i = d_opp(i) + 6 U w_i rho c_i.u
//     - 18 U w_i (c_iy N_y + c_iz N_z), N_a = sum_{c_x = 0} f c_a - (2/3) rho u_a,
//     which imposes the density and the whole velocity.
#pragma once
#include "step.hpp"

namespace lbm {
namespace q27 {

constexpr int Q = 27;
// rest; axes; xy, xz, yz edges; corners; each odd direction followed by its opposite
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, -1, 1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, 1, -1};
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
// 216 w_i
__host__ __device__ constexpr int kw(int i) {
  return (CX[i] != 0) + (CY[i] != 0) + (CZ[i] != 0) == 0 ? 64
         : (CX[i] != 0) + (CY[i] != 0) + (CZ[i] != 0) == 1 ? 16
         : (CX[i] != 0) + (CY[i] != 0) + (CZ[i] != 0) == 2 ? 4 : 1;
}
__host__ __device__ constexpr int pk(int i) { return pair_of(CY[i], CZ[i]); }
// the collision's pairing: every odd direction's opposite follows it, with the same weight
static_assert([] {
  for (int i = 1; i < Q; i += 2)
    if (opp(i) != i + 1 || kw(i) != kw(i + 1) || CX[i] != -CX[i + 1] || CY[i] != -CY[i + 1] || CZ[i] != -CZ[i + 1])
      return false;
  return true;
}(), "D3Q27 directions must come in opposite pairs");

constexpr uint64_t L_DEAD = 1ull << 0;
constexpr uint64_t L_UNI = 1ull << 27;
constexpr uint64_t L_IN = 1ull << 28;
constexpr uint64_t L_OUT = 1ull << 29;
constexpr uint64_t L_REG = 1ull << 30;
constexpr uint64_t L_UPS = 1ull << 31;
constexpr int L_UNK = 32;
constexpr int NX = 9;  // populations per open face
constexpr int XIN[NX] = {1, 7, 9, 11, 13, 19, 21, 23, 26};
constexpr int XOUT[NX] = {2, 8, 10, 12, 14, 20, 22, 24, 25};

struct Bufs27 {
  void* A;                // populations, [27][nc], in place
  const uint32_t* code;   // (row << xbits) | x
  const uint64_t* links;  // link word per compact cell
  const int* delta;       // [nrow][8] neighbour-row deltas
  const float* phi;
  float* omega;
  const float* shape;
  const uint32_t* rowbox;
  double* part;
  uint32_t* tc;
  const double* wave;
  float* side;            // extrapolation outflow: [2][nrow][18] kept values by parity
};

template <int I>
__device__ __forceinline__ uint32_t src_of(const Pos& q) {
  const int xs = CX[I] == 1 ? q.xm : (CX[I] == -1 ? q.xp : q.x);
  return (uint32_t)(xs + q.dl[pk(I)]);
}
template <int I, bool ODD, class S>
__device__ __forceinline__ Slot slot_in(const Params& p, uint32_t c, uint64_t lk, const Pos& q) {
  constexpr uint32_t SB = sizeof(S);
  if (!ODD || I == 0) return {c * SB, p.plb[I]};
  const bool bb = (lk >> I) & 1u;
  return {bb ? p.plb[I] + c * SB : p.plb[opp(I)] + src_of<I>(q) * SB, 0u};
}
template <int I, bool ODD, class S>
__device__ __forceinline__ Slot slot_out(const Params& p, uint32_t c, uint64_t lk, const Pos& q) {
  constexpr uint32_t SB = sizeof(S);
  constexpr int J = opp(I);
  if (!ODD || I == 0) return {c * SB, p.plb[J]};
  const bool wall = (lk >> J) & 1u;
  return {wall ? p.plb[J] + c * SB : p.plb[I] + src_of<J>(q) * SB, 0u};
}

template <int I>
__device__ __forceinline__ int unk_index(uint64_t lk) {
  int k = -1;
#pragma unroll
  for (int j = 0; j < NX; ++j) {
    if ((lk & L_IN) && XIN[j] == I) k = j;
    if ((lk & L_OUT) && XOUT[j] == I) k = j;
  }
  return k;
}
template <int I>
__device__ __forceinline__ bool open_unknown(uint64_t lk) {
  if (CX[I] == 0) return false;
  const int k = unk_index<I>(lk);
  return k >= 0 && ((lk >> (L_UNK + k)) & 1u);
}

template <class S, bool SHW, bool UNI, bool ODD>
__device__ __forceinline__ void pull(const Params& p, const Pop<S>& A, const float* __restrict__ phi, uint32_t c,
                                     uint64_t lk, const Pos& q, float phx, float v[Q], float pt[Q]) {
  v[0] = A.ld(slot_in<0, ODD, S>(p, c, lk, q).v, slot_in<0, ODD, S>(p, c, lk, q).s);
  pt[0] = phx;
  sfor<1, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    constexpr int J = opp(I);
    const Slot a = slot_in<I, ODD, S>(p, c, lk, q);
    v[I] = A.ld(a.v, a.s);
    if (!UNI) {
      const bool bb = (lk >> I) & 1u;
      pt[J] = ldo(phi, bb ? c : src_of<I>(q));
    } else {
      pt[J] = phx;
    }
  });
  if (SHW) {
    const float s = p.f.ks * (phx - 1.0f);
#pragma unroll
    for (int i = 0; i < Q; ++i) v[i] -= (float)kw(i) * s;
  }
}

// Moment sums of the 27 values, from the opposite-pair sums P = x_I + x_J
// (even moments) and differences M = x_I - x_J (odd moments), as on D3Q19.
template <class R>
__device__ __forceinline__ Sums<R> moment_sums(const float d[Q]) {
  Sums<R> r{};
  r.s = (R)d[0];
  sfor<0, (Q - 1) / 2>([&](auto kc) {
    constexpr int I = 1 + 2 * decltype(kc)::value;
    const R a = (R)d[I], b = (R)d[I + 1];
    const R P = a + b, M = a - b;
    r.s += P;
    if (CX[I]) r.mx = CX[I] > 0 ? r.mx + M : r.mx - M;
    if (CY[I]) r.my = CY[I] > 0 ? r.my + M : r.my - M;
    if (CZ[I]) r.mz = CZ[I] > 0 ? r.mz + M : r.mz - M;
    if (CX[I]) r.xx += P;
    if (CY[I]) r.yy += P;
    if (CZ[I]) r.zz += P;
    if (CX[I] * CY[I]) r.xy = CX[I] * CY[I] > 0 ? r.xy + P : r.xy - P;
    if (CX[I] * CZ[I]) r.xz = CX[I] * CZ[I] > 0 ? r.xz + P : r.xz - P;
    if (CY[I] * CZ[I]) r.yz = CY[I] * CZ[I] > 0 ? r.yz + P : r.yz - P;
  });
  return r;
}

// Momentum sum(x c) of the 27 values in FP64, from the opposite-pair
// differences (exact in FP64): the FP64 projection needs only this moment.
__device__ __forceinline__ void pair_momentum(const float d[Q], double& mx, double& my, double& mz) {
  mx = 0.0; my = 0.0; mz = 0.0;
  sfor<0, (Q - 1) / 2>([&](auto kc) {
    constexpr int I = 1 + 2 * decltype(kc)::value;
    const double m = (double)d[I] - (double)d[I + 1];
    if (CX[I]) mx = CX[I] > 0 ? mx + m : mx - m;
    if (CY[I]) my = CY[I] > 0 ? my + m : my - m;
    if (CZ[I]) mz = CZ[I] > 0 ? mz + m : mz - m;
  });
}

// Open faces (phi = 1 there): Zou-He inflow / density outflow on nine
// unknowns, or the extrapolation outflow (side[parity][row][0..8] the cell's
// own c_x = -1 values of the previous step, [9..17] its -x neighbour's).
__device__ __forceinline__ void open_fill(const Params& p, uint32_t row, uint64_t lk, uint32_t t,
                                          const float* __restrict__ shape, const double* wave,
                                          const float* __restrict__ side_in, float d[Q]) {
  const bool in = (lk & L_IN) != 0;
  const bool outl = (lk & L_OUT) != 0;
  if (!(in || outl)) return;
  // One path for every open-face cell, with selects instead of conditional
  // stores: branches that store to different elements of d[] make the
  // compiler move d[] to scratch memory.
  const float iU = p.f.iU, ks = p.f.ks;
  float s0 = 0.0f, sp = 0.0f, sm = 0.0f, ty = 0.0f, tz = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (CX[i] == 0) {
      s0 += d[i];
      if (CY[i]) ty += CY[i] * d[i];
      if (CZ[i]) tz += CZ[i] * d[i];
    } else if (CX[i] == 1) {
      sp += d[i];
    } else {
      sm += d[i];
    }
  }
  // inflow: rho from mass and normal momentum, u = (uin, 0, 0); outflow:
  // rho_out and u_x from mass and the known half
  const float uin = in ? inflow_amplitude(p, wave, t) * shape[row] : 0.0f;
  const float rin = (1.0f + (s0 + 2.0f * sm) * iU) / (1.0f - uin);
  const float ro = p.f.rho_out;
  const float uout = (1.0f + (s0 + 2.0f * sp) * iU) / ro - 1.0f;
  // 6 U w_i rho c_ix u_x per unit 216 w_i, and 18 U w_i N_a / U per unit 216 w_i
  const float ain = 6.0f * ks * rin * uin, aout = -6.0f * ks * ro * uout;
  const float b = 18.0f / 216.0f;
  // extrapolation outflow: the cell's and its -x neighbour's kept values
  const bool ext = outl && p.outlet == 2;
  const float* e = side_in + (size_t)row * 18;
  const bool up = !((lk >> 1) & 1u);
  float dn[2 * NX];
#pragma unroll
  for (int k = 0; k < NX; ++k) {
    const float kwi = (float)kw(XIN[k]), kwo = (float)kw(XOUT[k]);
    dn[k] = d[XOUT[k]] + kwi * ain - kwi * b * ((float)CY[XIN[k]] * ty + (float)CZ[XIN[k]] * tz);
    float vo = d[XIN[k]] + kwo * aout - kwo * b * ((float)CY[XOUT[k]] * ty + (float)CZ[XOUT[k]] * tz);
    if (p.outlet == 2) {
      // the extrapolation replaces only the populations that come from
      // outside the face; Zou-He closes all nine (as on D3Q19)
      const bool u = (lk >> (L_UNK + k)) & 1u;
      const float own = ext ? e[k] : 0.0f, ups = ext ? e[NX + k] : 0.0f;
      const float ve = up ? rfma(CS, ups - own, own) : own;
      vo = ext ? (u ? ve : d[XOUT[k]]) : vo;
    }
    dn[NX + k] = vo;
  }
#pragma unroll
  for (int k = 0; k < NX; ++k) {
    d[XIN[k]] = in ? dn[k] : d[XIN[k]];
    d[XOUT[k]] = outl ? dn[NX + k] : d[XOUT[k]];
  }
}

// Keep the c_x = -1 pre-collision values of an extrapolation-outflow cell or
// of its -x neighbour for the next step.
__device__ __forceinline__ void outflow_keep(const Params& p, uint32_t row, uint64_t lk, float phx, const float d[Q],
                                             float* __restrict__ side_out) {
  const float s = p.f.ks * (phx - 1.0f);
  float* e = side_out + (size_t)row * 18 + ((lk & L_OUT) ? 0 : NX);
#pragma unroll
  for (int k = 0; k < NX; ++k) e[k] = rfma((float)kw(XOUT[k]), s, d[XOUT[k]]);
}

// Outer wall normal from the wall links (see step.hpp), 27 directions.
__device__ __forceinline__ bool wall_normal(uint64_t lk, float n[3]) {
  int mx = 0, my = 0, mz = 0;
  sfor<1, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    constexpr int J = opp(I);
    constexpr int k = kw(I);
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

// c_I . (x, y, z) summed over the nonzero components of c_I, in x, y, z order.
template <int I, class R>
__device__ __forceinline__ R cdot(R x, R y, R z) {
  R r = (R)0;
  bool any = false;
  auto add = [&](int ci, R v) {
    if (ci != 0) {
      r = any ? (ci > 0 ? r + v : r - v) : (ci > 0 ? v : -v);
      any = true;
    }
  };
  add(CX[I], x);
  add(CY[I], y);
  add(CZ[I], z);
  return r;
}

// Collision and store, as in step.hpp (deviation form, optional FP64 momentum
// projection onto the axis pairs, shift mode 1 conversion).
template <class S, bool SHW, bool UNI, bool ODD, class R, bool PROJ, int RM>
__device__ __forceinline__ void collide_store(const Params& p, const Pop<S>& A, uint32_t c, uint64_t lk, const Pos& q,
                                              float phx_f, float d[Q], const float pt[Q], const Macro<R>& M,
                                              uint32_t seed) {
  const R phx = (R)phx_f;
  const R om = M.omega;
  const R pr = phx * M.rho;
  const R A0 = phx * M.rm1 - (R)1.5 * pr * M.uu;
  const R K = (R)1 - (R)0.5 * om;
  const R K3 = (R)3 * K, K9 = (R)9 * K;
  const R uF = M.ux * M.Fx + M.uy * M.Fy + M.uz * M.Fz;
  const R keep = (R)1 - om;
  const R ev0 = om * A0 - K3 * uF;
  const R omB = om * (R)3 * pr, omC = om * (R)4.5 * pr;
  const R ks = p.k<R>().ks;
  // the input momentum for the projection, before d[] is overwritten by the
  // outputs (27 values kept once, not twice)
  double tx = 0.0, ty = 0.0, tz = 0.0;
  if constexpr (PROJ) pair_momentum(d, tx, ty, tz);
  float* o = d;
  // Directions come in opposite pairs (I odd, I + 1 its opposite): with
  // e = c_I.u and h = c_I.F the part omega C e^2 + K9 e h + ev0 is shared by
  // the pair and omega B e + K3 h flips sign, so each pair costs one
  // evaluation; c.u and c.F take only the nonzero components of c_I.
  o[0] = (float)rfma(ks * (R)kw(0), UNI ? ev0 : ev0 + M.rm1 * ((R)pt[0] - phx), keep * (R)d[0]);
  sfor<0, (Q - 1) / 2>([&](auto kc) {
    constexpr int I = 1 + 2 * decltype(kc)::value;
    constexpr int J = I + 1;
    const R e = cdot<I>(M.ux, M.uy, M.uz);
    const R h = cdot<I>(M.Fx, M.Fy, M.Fz);
    const R ev = rfma(omC, e * e, rfma(K9, e * h, ev0));
    const R od = rfma(omB, e, K3 * h);
    R gi = ev + od, gj = ev - od;
    if (!UNI) {
      gi += M.rm1 * ((R)pt[I] - phx);
      gj += M.rm1 * ((R)pt[J] - phx);
    }
    const R kk = ks * (R)kw(I);
    o[I] = (float)rfma(kk, gi, keep * (R)d[I]);
    o[J] = (float)rfma(kk, gj, keep * (R)d[J]);
  });
  if constexpr (PROJ) {
    double smx, smy, smz;
    pair_momentum(o, smx, smy, smz);
    const double U = p.d.U;
    tx += U * (double)M.Fx; ty += U * (double)M.Fy; tz += U * (double)M.Fz;
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
    const double rx = 0.5 * (tx - smx), ry = 0.5 * (ty - smy), rz = 0.5 * (tz - smz);
    o[1] = (float)((double)o[1] + rx); o[2] = (float)((double)o[2] - rx);
    o[3] = (float)((double)o[3] + ry); o[4] = (float)((double)o[4] - ry);
    o[5] = (float)((double)o[5] + rz); o[6] = (float)((double)o[6] - rz);
  }
  if (SHW) {
    const float ksf = p.f.ks;
#pragma unroll
    for (int i = 0; i < Q; ++i) o[i] += ksf * (float)kw(i) * ((UNI ? phx_f : pt[i]) - 1.0f);
  }
  if constexpr (!std::is_same<S, float>::value && RM != 0) {
    unsigned short hb[Q];
    round16<S, Q, RM>(CX, CY, CZ, o, hb, seed);
    sfor<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      const Slot a = slot_out<I, ODD, S>(p, c, lk, q);
      A.st_bits(a.v, a.s, hb[I]);
    });
  } else {
    sfor<0, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      const Slot a = slot_out<I, ODD, S>(p, c, lk, q);
      A.st(a.v, a.s, o[I]);
    });
  }
}

template <class R>
__device__ __forceinline__ void diag_terms(const Params& p, float phx, const float d[Q], const Macro<R>& M, uint64_t lk,
                                           bool active, double (&v)[NDIAGP]) {
  if (!active) {
    v[0] = v[1] = v[2] = v[3] = v[4] = v[5] = v[9] = v[10] = 0.0;
    v[6] = 0.0; v[7] = 1e300; v[8] = -1e300;
    return;
  }
  const bool reg = (lk & L_REG) != 0;
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
  if (bad) v[6] = 1e300;
  float n[3];
  R tau[3];
  v[10] = (reg && wall_normal(lk, n)) ? (double)wall_tau(M, n, tau) : 0.0;
}

template <class S, bool SHW, bool UNI, bool ODD, int DIAG, class R, bool PROJ, int RM>
__device__ __forceinline__ void step_cell(const Params& p, const Bufs27& b, uint32_t c, uint64_t lk, uint32_t t,
                                          double (&dv)[NDIAGP]) {
  // an even step of a uniform-porosity cell touches only its own slots: its
  // position is needed only for an open-face row's data
  const bool where = ODD || !UNI || (lk & (L_IN | L_OUT | L_UPS));
  Pos q = position(p, c, where ? b.code[c] : 0u);
  if (ODD || !UNI) load_deltas(b.delta, q);
  const float phx = ldo(b.phi, c);
  float d[Q], pt[Q];
  const Pop<S> A(b.A, p.abytes);
  pull<S, SHW, UNI, ODD>(p, A, b.phi, c, lk, q, phx, d, pt);
  const size_t half = (size_t)p.nrow * 18;
  open_fill(p, q.row, lk, t, b.shape, b.wave, b.side + (ODD ? half : 0), d);
  if (p.outlet == 2 && (lk & (L_OUT | L_UPS))) outflow_keep(p, q.row, lk, phx, d, b.side + (ODD ? 0 : half));
  const float omp = b.omega[c];
  Macro<R> M;
  macro_sums<R>(p, phx, moment_sums<R>(d), omp, M);
  b.omega[c] = (float)M.omega;
  if (DIAG == 1) diag_terms<R>(p, phx, d, M, lk, true, dv);
  collide_store<S, SHW, UNI, ODD, R, PROJ, RM>(p, A, c, lk, q, phx, d, pt, M, RM == 2 ? round_seed(c, t) : 0u);
}

// One D3Q27 step at parity ODD.  DIAG: 0 none, 1 diagnostics partials.
template <class S, bool SHW, bool ODD, int DIAG, class R, bool PROJ, int NT, int RM = 0>
__global__ __launch_bounds__(NT) void k_step(Params p, Bufs27 b) {
  const uint32_t c = xcd_block(blockIdx.x, gridDim.x) * NT + threadIdx.x;
  const uint32_t t = b.tc[ODD ? 1 : 0];
  const uint64_t lk = c < (uint32_t)p.nc ? b.links[c] : L_DEAD;
  const bool active = !(lk & L_DEAD);
  double dv[NDIAGP];
  const bool uni = !active || (lk & L_UNI);
  if (__all(uni)) {
    if (active) step_cell<S, SHW, true, ODD, DIAG, R, PROJ, RM>(p, b, c, lk, t, dv);
  } else {
    if (active) step_cell<S, SHW, false, ODD, DIAG, R, PROJ, RM>(p, b, c, lk, t, dv);
  }
  if (DIAG == 1) {
    if (!active) {
      float d[Q] = {};
      Macro<R> M{};
      diag_terms<R>(p, 0.f, d, M, uint64_t(0), false, dv);
    }
    const int ops[NDIAGP] = {0, 0, 0, 0, 0, 0, 1, 2, 1, 0, 0};
    block_reduce<NDIAGP, NT>(dv, ops, b.part + (size_t)blockIdx.x * NDIAGP);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) b.tc[ODD ? 0 : 1] = t + 1u;
}

// Moments of the current state (dense box outputs, any may be null) and
// optionally the diagnostics partials.
template <class S, bool SHW, bool ODD, bool DIAG, class R>
__global__ __launch_bounds__(BLOCK) void k_moments(Params p, Bufs27 b, uint32_t t, size_t nbox, float* rho_o,
                                                    float* u_o, float* shear_o, float* omega_o, float* sigma_o,
                                                    float* tau_o) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  const uint64_t lk = c < (uint32_t)p.nc ? b.links[c] : L_DEAD;
  const bool active = !(lk & L_DEAD);
  double dv[NDIAGP];
  if (active) {
    Pos q = position(p, c, b.code[c]);
    if (ODD) load_deltas(b.delta, q);
    const float phx = ldo(b.phi, c);
    float d[Q], pt[Q];
    pull<S, SHW, true, ODD>(p, Pop<S>(b.A, p.abytes), b.phi, c, lk, q, phx, d, pt);
    open_fill(p, q.row, lk, t, b.shape, b.wave, b.side + (ODD ? (size_t)p.nrow * 18 : 0), d);
    Macro<R> M;
    macro_sums<R>(p, phx, moment_sums<R>(d), b.omega[c], M);
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
    diag_terms<R>(p, 0.f, d, M, uint64_t(0), false, dv);
  }
  if (DIAG) {
    const int ops[NDIAGP] = {0, 0, 0, 0, 0, 0, 1, 2, 1, 0, 0};
    block_reduce<NDIAGP>(dv, ops, b.part + (size_t)blockIdx.x * NDIAGP);
  }
}

// Rest state at even parity (see step.hpp's k_init).
template <class S, bool SHW>
__global__ __launch_bounds__(BLOCK) void k_init(Params p, Bufs27 b, float omega0) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= (uint32_t)p.nc) return;
  if (b.links[c] & L_DEAD) return;
  const float phx = ldo(b.phi, c);
  const Pop<S> A(b.A, p.abytes);
  const float ks = p.f.ks;
#pragma unroll
  for (int i = 0; i < Q; ++i)
    A.st(c * (uint32_t)sizeof(S), p.plb[i], SHW ? ks * (float)kw(i) * (phx - 1.0f) : 0.0f);
  b.omega[c] = omega0;
  if (c == 0) b.tc[0] = 0u;
}

template <int I>
__device__ __forceinline__ bool kept_unknown(const Params& p, uint64_t lk) {
  return CX[I] == -1 && (lk & L_OUT) && p.outlet == 2;
}

// State out / in, as in step.hpp.
template <class S, bool ODD>
__global__ __launch_bounds__(BLOCK) void k_gather_state(Params p, Bufs27 b, float* out) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= (uint32_t)p.nc) return;
  const uint64_t lk = b.links[c];
  if (lk & L_DEAD) return;
  Pos q = position(p, c, b.code[c]);
  if (ODD) load_deltas(b.delta, q);
  const Pop<S> A(b.A, p.abytes);
  float d[Q];
  sfor<0, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    const Slot a = slot_in<I, ODD, S>(p, c, lk, q);
    d[I] = A.ld(a.v, a.s);
  });
  if ((lk & L_OUT) && p.outlet == 2) {
    const float* e = b.side + (ODD ? (size_t)p.nrow * 18 : 0) + (size_t)q.row * 18;
    const bool up = !((lk >> 1) & 1u);
#pragma unroll
    for (int k = 0; k < NX; ++k)
      if ((lk >> (L_UNK + k)) & 1u) d[XOUT[k]] = up ? rfma(CS, e[NX + k] - e[k], e[k]) : e[k];
  }
  sfor<0, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    const bool unk = open_unknown<I>(lk) && !kept_unknown<I>(p, lk);
    out[(size_t)I * p.nc + c] = unk ? __builtin_nanf("") : d[I];
  });
}

template <class S, bool ODD>
__global__ __launch_bounds__(BLOCK) void k_scatter_state(Params p, Bufs27 b, const float* in) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= (uint32_t)p.nc) return;
  const uint64_t lk = b.links[c];
  if (lk & L_DEAD) return;
  Pos q = position(p, c, b.code[c]);
  if (ODD) load_deltas(b.delta, q);
  const Pop<S> A(b.A, p.abytes);
  sfor<0, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    const Slot a = slot_in<I, ODD, S>(p, c, lk, q);
    const float v = in[(size_t)I * p.nc + c];
    if (kept_unknown<I>(p, lk) && open_unknown<I>(lk)) {
      const int k = unk_index<I>(lk);
      float* e = b.side + (ODD ? (size_t)p.nrow * 18 : 0) + (size_t)q.row * 18;
      e[k] = v;
      e[NX + k] = v;
    } else if (!open_unknown<I>(lk)) {
      A.st(a.v, a.s, v);
    }
  });
}

}  // namespace q27
}  // namespace lbm
