// Reverse-time (adjoint) step of the VANSE Carreau-Yasuda collide-and-stream
// map, for the gradient of a region kinetic-energy objective with respect to
// the porosity field.
//
// The per-cell forward map of step n is
//   (pulled f_i, omega_prev, phi(x), phi~(x + c_i)) -> (q_i, omega, e)
// with the open-face fill, moments, explicit velocity with Darcy drag, force,
// equilibrium, corrected second moment Pi, semi-explicit shear rate,
// Carreau-Yasuda viscosity, relaxation rate and the BGK + Guo + porosity-jump
// collision (the paper's method section).  Its transpose is written out by hand
// below in terms of the weighted output adjoint a_i = w_i qhat_i and its
// moments s0 = sum a_i, s1 = sum a_i c_i, s2 = sum a_i c_i c_i, so the sweep
// stays in registers.  The streaming transpose gathers qhat_i(x) from the
// consumer's pulled-value adjoint at x + c_i (or the cell's own opposite slot
// across a wall).  The porosity-jump term couples q_i(x) to phi(x + c_i); that
// contribution is gathered by the consumer cell from the producer's recorded
// density of the previous step, so no atomics are needed.
//
// Supported: FP32 storage, shift mode 0, no Forchheimer drag.
#pragma once
#include "step.hpp"

namespace lbm {

struct AdjBufs {
  const uint32_t* cells;
  const float* phi;       // dense box porosity
  const float* shape;     // inflow profile
  const float* rec;       // record of step n: [19][nf] pulled deltas (before the fill), [nf] omega_prev
  const float* rho_prev;  // dense density of step n-1 (null for n = 0)
  const float* ph_next;   // adjoint of the pulled populations of step n+1, [19][nbox]
  float* ph_out;          // adjoint of the pulled populations of step n, [19][nbox]
  float* omh;             // per cell: in adjoint of omega_n, out adjoint of omega_{n-1}
  float* phih;            // per cell: porosity adjoint accumulator (FP32, flushed per segment)
};

// Symmetric 3x3 stored as xx yy zz xy xz yz.
__device__ __forceinline__ void sym_mv(const float s[6], float x, float y, float z, float& ox, float& oy, float& oz) {
  ox = s[0] * x + s[3] * y + s[4] * z;
  oy = s[3] * x + s[1] * y + s[5] * z;
  oz = s[4] * x + s[5] * y + s[2] * z;
}

__global__ __launch_bounds__(BLOCK) void k_adjoint(Params p, AdjBufs a, float amp, float ew) {
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t c = blk * BLOCK + threadIdx.x;
  if (c >= (uint32_t)p.nf) return;
  int x, y, z;
  bool reg;
  unpack(a.cells[c], x, y, z, reg);
  const uint32_t idx = (uint32_t)x + p.nx * ((uint32_t)y + p.ny * (uint32_t)z);
  const float phx = ldo(a.phi, idx);
  const Nb nb(p, x, y, z);

  // ---- forward recompute from the record --------------------------------
  float d[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) d[i] = a.rec[(size_t)i * p.nf + c];
  const float omp = a.rec[(size_t)Q * p.nf + c];
  open_fill(p, x, y, z, amp, a.shape, d);
  Macro M;
  macro(p, phx, d, omp, M);
  const float iphi = fast_rcp(phx);
  float sd = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) sd += d[i];
  const float S = phx + sd;  // sum f = phi rho
  const float mx = (d[1] + d[7] + d[9] + d[11] + d[13]) - (d[2] + d[8] + d[10] + d[12] + d[14]);
  const float my = (d[3] + d[7] + d[10] + d[15] + d[17]) - (d[4] + d[8] + d[9] + d[16] + d[18]);
  const float mz = (d[5] + d[11] + d[14] + d[15] + d[18]) - (d[6] + d[12] + d[13] + d[16] + d[17]);
  const float om1 = 1.0f - phx;
  const float kn = p.kcd * p.nu_d;
  const float dark = kn * om1 * om1 * iphi * iphi;  // phi nu / k
  const float C0 = 0.5f + 0.25f * dark;
  const float D = phx * dark;                       // phi^2 nu / k
  const float rho = M.rho, ux = M.ux, uy = M.uy, uz = M.uz, uu = M.uu;
  const float Fx = M.Fx, Fy = M.Fy, Fz = M.Fz;
  const float om = M.omega;
  const float pn2 = M.P[0] * M.P[0] + M.P[1] * M.P[1] + M.P[2] * M.P[2] +
                    2.0f * (M.P[3] * M.P[3] + M.P[4] * M.P[4] + M.P[5] * M.P[5]);
  const float Nn = __builtin_sqrtf(pn2);
  const float shear = M.shear;
  const float lg = p.lam * shear;
  float la, dla;  // (lambda g)^a and its derivative in g
  if (p.cy_a2) { la = lg * lg; dla = 2.0f * p.lam * lg; }
  else {
    la = lg > 0.0f ? __builtin_amdgcn_exp2f(p.cy_a * __builtin_amdgcn_logf(lg)) : 0.0f;
    dla = (lg > 0.0f && shear > 0.0f) ? p.cy_a * la / shear : 0.0f;
  }
  const float h = 1.0f + la;
  const float fac = __builtin_amdgcn_exp2f(p.cy_e * __builtin_amdgcn_logf(h));
  const float nu = p.nu_inf + (p.nu0 - p.nu_inf) * fac;
  const float dnu = (p.nu0 - p.nu_inf) * p.cy_e * fac * fast_rcp(h) * dla;

  // ---- gather the adjoint of the post-collision populations --------------
  float qh[Q];
  qh[0] = ldo(a.ph_next, idx);
  uint32_t fmask = 0;
  float sfl = 0.f, sjump = 0.f;
#define LBM_QH(I)                                                                        \
  {                                                                                      \
    bool out;                                                                            \
    const int o = nb.template off<Dir<I>::cx, Dir<I>::cy, Dir<I>::cz>(out);              \
    const uint32_t tgt = idx + (uint32_t)o;                                              \
    const float pn = ldo(a.phi, tgt);                                                    \
    const bool fl = !out && (pn != 0.0f);                                                \
    const uint32_t e = fl ? (uint32_t)I * p.nbox + tgt : (uint32_t)Dir<I>::opp * p.nbox + idx; \
    qh[I] = ldo(a.ph_next, e);                                                           \
    const float ai = wgt(I) * qh[I];                                                     \
    sfl += fl ? ai : 0.0f;                                                               \
    sjump += fl ? ai * (pn - phx) : 0.0f;                                                \
    fmask |= fl ? (1u << I) : 0u;                                                        \
  }
  LBM_QH(1) LBM_QH(2) LBM_QH(3) LBM_QH(4) LBM_QH(5) LBM_QH(6) LBM_QH(7) LBM_QH(8) LBM_QH(9)
  LBM_QH(10) LBM_QH(11) LBM_QH(12) LBM_QH(13) LBM_QH(14) LBM_QH(15) LBM_QH(16) LBM_QH(17) LBM_QH(18)
#undef LBM_QH

  // moments of a_i = w_i qhat_i
  float av[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) av[i] = wgt(i) * qh[i];
  float s0 = 0.f, qd = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) { s0 += av[i]; qd += qh[i] * d[i]; }
  const float s1x = (av[1] + av[7] + av[9] + av[11] + av[13]) - (av[2] + av[8] + av[10] + av[12] + av[14]);
  const float s1y = (av[3] + av[7] + av[10] + av[15] + av[17]) - (av[4] + av[8] + av[9] + av[16] + av[18]);
  const float s1z = (av[5] + av[11] + av[14] + av[15] + av[18]) - (av[6] + av[12] + av[13] + av[16] + av[17]);
  float s2[6];
  s2[0] = av[1] + av[2] + av[7] + av[8] + av[9] + av[10] + av[11] + av[12] + av[13] + av[14];
  s2[1] = av[3] + av[4] + av[7] + av[8] + av[9] + av[10] + av[15] + av[16] + av[17] + av[18];
  s2[2] = av[5] + av[6] + av[11] + av[12] + av[13] + av[14] + av[15] + av[16] + av[17] + av[18];
  s2[3] = (av[7] + av[8]) - (av[9] + av[10]);
  s2[4] = (av[11] + av[12]) - (av[13] + av[14]);
  s2[5] = (av[15] + av[16]) - (av[17] + av[18]);

  const float pr = phx * rho;
  const float K = 1.0f - 0.5f * om, keep = 1.0f - om;
  const float uF = ux * Fx + uy * Fy + uz * Fz;
  float s2ux, s2uy, s2uz, s2Fx, s2Fy, s2Fz;
  sym_mv(s2, ux, uy, uz, s2ux, s2uy, s2uz);
  sym_mv(s2, Fx, Fy, Fz, s2Fx, s2Fy, s2Fz);
  const float s1u = s1x * ux + s1y * uy + s1z * uz;
  const float s1F = s1x * Fx + s1y * Fy + s1z * Fz;
  const float us2u = ux * s2ux + uy * s2uy + uz * s2uz;
  const float us2F = ux * s2Fx + uy * s2Fy + uz * s2Fz;
  const float Aeq = phx * M.rm1 - 1.5f * pr * uu;

  // collision: q = (1-omega) f + omega feq + K g + w rho (phi~ - phi)
  float omh = a.omh[c] + (Aeq * s0 + 3.0f * pr * s1u + 4.5f * pr * us2u - qd) -
              0.5f * (3.0f * s1F - 3.0f * s0 * uF + 9.0f * us2F);
  float uhx = K * (9.0f * s2Fx - 3.0f * s0 * Fx), uhy = K * (9.0f * s2Fy - 3.0f * s0 * Fy),
        uhz = K * (9.0f * s2Fz - 3.0f * s0 * Fz);
  float Fhx = K * (3.0f * s1x - 3.0f * s0 * ux + 9.0f * s2ux), Fhy = K * (3.0f * s1y - 3.0f * s0 * uy + 9.0f * s2uy),
        Fhz = K * (3.0f * s1z - 3.0f * s0 * uz + 9.0f * s2uz);
  // equilibrium w phi rho (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u), weighted by omega
  const float brk = om * (s0 * (1.0f - 1.5f * uu) + 3.0f * s1u + 4.5f * us2u);
  const float pro = pr * om;
  uhx += pro * (3.0f * s1x + 9.0f * s2ux - 3.0f * s0 * ux);
  uhy += pro * (3.0f * s1y + 9.0f * s2uy - 3.0f * s0 * uy);
  uhz += pro * (3.0f * s1z + 9.0f * s2uz - 3.0f * s0 * uz);
  float rhoh = phx * brk + sjump;
  float phh = rho * brk - rho * sfl;

  // relaxation rate omega = 2 rho / (6 nu + rho), nu = CY(shear)
  const float den6 = 6.0f * nu + rho;
  const float id2 = fast_rcp(den6 * den6);
  rhoh += omh * 12.0f * nu * id2;
  const float nuh = -omh * 12.0f * rho * id2;
  const float gh = nuh * dnu;
  const float irho = fast_rcp(rho);
  const float omph = gh * 3.0f * Nn * irho;      // adjoint of omega_prev
  const float Nh = gh * 3.0f * omp * irho;
  rhoh -= gh * shear * irho;
  // Pi = sum f c c - phi rho (I/3 + u u) + (F u + u F)/2, |Pi|_F
  const float gsc = Nn > 0.0f ? Nh * fast_rcp(Nn) : 0.0f;
  float G[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) G[k] = gsc * M.P[k];
  float Gux, Guy, Guz, GFx, GFy, GFz;
  sym_mv(G, ux, uy, uz, Gux, Guy, Guz);
  sym_mv(G, Fx, Fy, Fz, GFx, GFy, GFz);
  const float tP = (G[0] + G[1] + G[2]) * (1.0f / 3.0f) + ux * Gux + uy * Guy + uz * Guz;
  rhoh -= phx * tP;
  phh -= rho * tP;
  uhx += GFx - 2.0f * pr * Gux;
  uhy += GFy - 2.0f * pr * Guy;
  uhz += GFz - 2.0f * pr * Guz;
  Fhx += Gux; Fhy += Guy; Fhz += Guz;
  // objective e = rho |u|^2 / 2 on region cells
  const float eh = reg ? ew : 0.0f;
  rhoh += eh * 0.5f * uu;
  uhx += eh * rho * ux; uhy += eh * rho * uy; uhz += eh * rho * uz;
  // force F = rho (g - D u), D = phi^2 nu / k
  rhoh += (Fhx * Fx + Fhy * Fy + Fhz * Fz) * irho;
  uhx -= rho * D * Fhx; uhy -= rho * D * Fhy; uhz -= rho * D * Fhz;
  const float Dh = -rho * (Fhx * ux + Fhy * uy + Fhz * uz);
  phh += Dh * (-kn * (1.0f - phx * phx) * iphi * iphi);
  // u = v / (2 C0), C0 = 1/2 + (phi nu / k)/4
  const float i2c = fast_rcp(2.0f * C0);
  const float vhx = uhx * i2c, vhy = uhy * i2c, vhz = uhz * i2c;
  const float C0h = -(uhx * ux + uhy * uy + uhz * uz) * 2.0f * i2c;
  phh += 0.25f * C0h * (-2.0f * kn * om1 * iphi * iphi * iphi);
  // v = m / S + g / (2 phi)
  const float iS = fast_rcp(S);
  const float mhx = vhx * iS, mhy = vhy * iS, mhz = vhz * iS;
  float Sh = -(vhx * mx + vhy * my + vhz * mz) * iS * iS;
  phh -= (vhx * p.gx + vhy * p.gy + vhz * p.gz) * 0.5f * iphi * iphi;
  // rho = S / phi
  Sh += rhoh * iphi;
  phh -= rhoh * rho * iphi;

  // adjoint of the (filled) pulled populations
  float fh[Q];
  fh[0] = keep * qh[0] + Sh;
#define LBM_FH(I)                                                                                        \
  fh[I] = keep * qh[I] + Sh + mhx * (float)Dir<I>::cx + mhy * (float)Dir<I>::cy + mhz * (float)Dir<I>::cz + \
          (float)(Dir<I>::cx * Dir<I>::cx) * G[0] + (float)(Dir<I>::cy * Dir<I>::cy) * G[1] +             \
          (float)(Dir<I>::cz * Dir<I>::cz) * G[2] + 2.0f * ((float)(Dir<I>::cx * Dir<I>::cy) * G[3] +      \
          (float)(Dir<I>::cx * Dir<I>::cz) * G[4] + (float)(Dir<I>::cy * Dir<I>::cz) * G[5]);
  LBM_FH(1) LBM_FH(2) LBM_FH(3) LBM_FH(4) LBM_FH(5) LBM_FH(6) LBM_FH(7) LBM_FH(8) LBM_FH(9)
  LBM_FH(10) LBM_FH(11) LBM_FH(12) LBM_FH(13) LBM_FH(14) LBM_FH(15) LBM_FH(16) LBM_FH(17) LBM_FH(18)
#undef LBM_FH

  // transpose of the open-face fill: the unknowns' adjoints flow to the knowns
  const bool in = p.inlet && x == 0;
  const bool outl = p.outlet && x == p.nx - 1;
  if (in) {
    const float uin = amp * a.shape[y + p.ny * z];
    fh[2] += fh[1]; fh[8] += fh[7]; fh[10] += fh[9]; fh[12] += fh[11]; fh[14] += fh[13];
    const float rinh = uin * (1.0f / 3.0f) * fh[1] + uin * (1.0f / 6.0f) * (fh[7] + fh[9] + fh[11] + fh[13]);
    const float nyh = 0.5f * (fh[9] - fh[7]), nzh = 0.5f * (fh[13] - fh[11]);
    const float k = rinh / (1.0f - uin);
    fh[0] += k; fh[3] += k; fh[4] += k; fh[5] += k; fh[6] += k; fh[15] += k; fh[16] += k; fh[17] += k; fh[18] += k;
    fh[2] += 2.0f * k; fh[8] += 2.0f * k; fh[10] += 2.0f * k; fh[12] += 2.0f * k; fh[14] += 2.0f * k;
    fh[3] += nyh; fh[4] -= nyh; fh[15] += nyh; fh[16] -= nyh; fh[17] += nyh; fh[18] -= nyh;
    fh[5] += nzh; fh[6] -= nzh; fh[15] += nzh; fh[16] -= nzh; fh[17] -= nzh; fh[18] += nzh;
    fh[1] = 0.f; fh[7] = 0.f; fh[9] = 0.f; fh[11] = 0.f; fh[13] = 0.f;
  } else if (outl) {
    const float ro = p.rho_out;
    fh[1] += fh[2]; fh[7] += fh[8]; fh[9] += fh[10]; fh[11] += fh[12]; fh[13] += fh[14];
    const float uxh = -ro * (1.0f / 3.0f) * fh[2] - ro * (1.0f / 6.0f) * (fh[8] + fh[10] + fh[12] + fh[14]);
    const float nyh = 0.5f * (fh[8] - fh[10]), nzh = 0.5f * (fh[12] - fh[14]);
    const float k = uxh / ro;
    fh[0] += k; fh[3] += k; fh[4] += k; fh[5] += k; fh[6] += k; fh[15] += k; fh[16] += k; fh[17] += k; fh[18] += k;
    fh[1] += 2.0f * k; fh[7] += 2.0f * k; fh[9] += 2.0f * k; fh[11] += 2.0f * k; fh[13] += 2.0f * k;
    fh[3] += nyh; fh[4] -= nyh; fh[15] += nyh; fh[16] -= nyh; fh[17] += nyh; fh[18] -= nyh;
    fh[5] += nzh; fh[6] -= nzh; fh[15] += nzh; fh[16] -= nzh; fh[17] -= nzh; fh[18] += nzh;
    fh[2] = 0.f; fh[8] = 0.f; fh[10] = 0.f; fh[12] = 0.f; fh[14] = 0.f;
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) sto(a.ph_out, (uint32_t)i * p.nbox + idx, fh[i]);
  a.omh[c] = omph;

  // porosity-jump term of step n-1: q_i(x - c_i) depends on phi(x) when
  // x - c_i is a fluid producer; its adjoint is w_i rho_{n-1}(x - c_i) fh_i(x).
  if (a.rho_prev) {
#define LBM_NB(J)                                                                     \
    if (fmask & (1u << J)) {                                                          \
      bool out;                                                                       \
      const int o = nb.template off<Dir<J>::cx, Dir<J>::cy, Dir<J>::cz>(out);         \
      phh += wgt(J) * ldo(a.rho_prev, idx + (uint32_t)o) * fh[Dir<J>::opp];           \
    }
    LBM_NB(1) LBM_NB(2) LBM_NB(3) LBM_NB(4) LBM_NB(5) LBM_NB(6) LBM_NB(7) LBM_NB(8) LBM_NB(9)
    LBM_NB(10) LBM_NB(11) LBM_NB(12) LBM_NB(13) LBM_NB(14) LBM_NB(15) LBM_NB(16) LBM_NB(17) LBM_NB(18)
#undef LBM_NB
  }
  a.phih[c] += phh;
}

// Flush the per-segment FP32 porosity adjoint into the FP64 total.
__global__ __launch_bounds__(BLOCK) void k_adj_flush(int nf, float* phih, double* total) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= (uint32_t)nf) return;
  total[c] += (double)phih[c];
  phih[c] = 0.0f;
}

// Rest state f_i(0, x) = w_i phi(x) on the known links, then scatter the total
// into the box-layout gradient.
__global__ __launch_bounds__(BLOCK) void k_adj_final(Params p, const uint32_t* cells, const float* ph0,
                                                     const double* total, float* grad) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= (uint32_t)p.nf) return;
  int x, y, z;
  bool reg;
  unpack(cells[c], x, y, z, reg);
  const uint32_t idx = (uint32_t)x + p.nx * ((uint32_t)y + p.ny * (uint32_t)z);
  double s = total[c];
#pragma unroll
  for (int i = 0; i < Q; ++i) s += (double)wgt(i) * (double)ldo(ph0, (uint32_t)i * p.nbox + idx);
  grad[idx] = (float)s;
}

}  // namespace lbm
