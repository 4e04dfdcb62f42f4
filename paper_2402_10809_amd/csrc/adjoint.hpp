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
// With the extrapolation outflow, an outflow cell's unknowns (c_x = -1) are
// state: step n computes them as (1 - c_s) times the cell's own value of step
// n-1 plus c_s times the -x neighbour's pulled value of step n-1.  The reverse
// step of n leaves the unknowns' total adjoints per row (aside_out); the reverse
// step of n-1 adds (1 - c_s) of them to the outflow cell's unknowns and c_s of
// them to the -x neighbour's pulled values.
//
// AN: the anisotropic permeability of the method section's Remark, whose
// fixed-point iterates are recomputed from v inside the reverse step.
//
// Supported: FP32 storage, shift mode 0, with or without Forchheimer drag,
// isotropic or anisotropic permeability, D3Q19.  The recompute uses the same
// arithmetic type as the forward step.
#pragma once
#include "step.hpp"

namespace lbm {

struct AdjBufs {
  const uint32_t* code;   // (row << xbits) | x per compact cell
  const uint32_t* links;  // link word per compact cell
  const int* delta;       // neighbour-row deltas
  const float* phi;       // porosity per compact cell
  const float* shape;     // inflow profile per row
  const double* wave;     // sampled inflow waveform
  const float* rec;       // record of step n: [19][nc] pulled values (after the fill), [nc] omega_prev
  const float* rho_prev;  // density of step n-1 per compact cell (null for n = 0)
  const void* ph_next;    // adjoint of the pulled populations of step n+1, [19][nc] (FP32 or FP64)
  void* ph_out;           // adjoint of the pulled populations of step n, [19][nc] (FP32 or FP64)
  double* omh;            // per cell: in adjoint of omega_n, out adjoint of omega_{n-1}
  double* phih;           // per cell: porosity adjoint accumulator
  const double* aside_in; // extrapolation outflow: per row, adjoints of the 5 c_x = -1 unknowns of step n+1
  double* aside_out;      // the same for step n
};

// One FP32 value per lane from a buffer straight into LDS (the wave's 64
// consecutive slots at lds): the load occupies no register while in flight.
__device__ __forceinline__ void gather_to_lds(__amdgpu_buffer_rsrc_t r, float* lds, uint32_t byte_off) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds, 4, byte_off, 0, 0, 0);
}

// One reverse step at every fluid cell.  Arithmetic in FP64 (the adjoint
// recursion has the same slow modes as the forward map, so FP32 rounding of
// per-cell scalars would accumulate the same way); the adjoint populations are
// stored in FP32.
//
// Both instantiations are held to 2 waves per SIMD (at most 256 VGPRs; the
// isotropic one needs 247, the anisotropic one 255, without scratch).
template <bool AN, class PH = float>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2)))
void k_adjoint(Params p, AdjBufs a, uint32_t t, float ew, int kind) {
  using R = double;
  constexpr bool P64 = std::is_same<PH, double>::value;  // FP64 adjoint populations
  // The neighbour gathers (adjoint populations of step n+1, porosities and,
  // for the porosity-jump term, densities of step n-1 at x + c_I) go straight
  // to LDS at the start, so that their latency overlaps the forward recompute
  // at two waves per SIMD without holding registers.  Each wave reads back
  // only the slots its own loads wrote: no barrier, one wait for the loads.
  __shared__ float sq[Q][BLOCK], sp[Q][BLOCK], sr[Q][BLOCK];
  // FP64 adjoint populations: their high words (the low words go to sq)
  __shared__ float sqh[P64 ? Q : 1][BLOCK];
  const uint32_t c = xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  if (c >= (uint32_t)p.nc) return;
  const uint32_t lk = a.links[c];
  if (lk & LK_DEAD) return;
  Pos q = position(p, c, a.code[c]);
  load_deltas(a.delta, q);
  const bool reg = (lk & LK_REG) != 0;
  const float phx_f = ldo(a.phi, c);
  const uint32_t tid = threadIdx.x, wb = tid & ~63u;  // this lane, and its wave's first slot
  // Then the record: the forward recompute waits for these loads only, while
  // the gathers issued after them are still in flight.  The per-cell adjoints
  // read-modified-written at the end are fetched here too, so that neither
  // read stalls the wave later (a wait there would also wait for the stores).
  // Loads complete in issue order for the wait counter, so the row's deltas,
  // which the gather addresses need, are kept ahead of all of these.
  asm volatile("" ::: "memory");
  float d[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) d[i] = __builtin_nontemporal_load(&a.rec[(size_t)i * p.nc + c]);
  const float omp = __builtin_nontemporal_load(&a.rec[(size_t)Q * p.nc + c]);
  const double omh_in = a.omh[c], phih_in = a.phih[c];
  {
    const uint32_t nb = (uint32_t)p.nc * 4u;
    constexpr uint32_t PB = sizeof(PH);  // bytes per adjoint population
    const __amdgpu_buffer_rsrc_t rq = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(a.ph_next), (short)0,
                                                                        (int)((uint32_t)p.nc * PB * (uint32_t)Q),
                                                                        0x00020000);
    const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(a.phi), (short)0,
                                                                        (int)nb, 0x00020000);
    const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(a.rho_prev), (short)0,
                                                                        (int)nb, 0x00020000);
    gather_to_lds(rq, &sq[0][wb], c * PB);
    if constexpr (P64) gather_to_lds(rq, &sqh[0][wb], c * PB + 4u);
    sfor<1, Q>([&](auto ic) {
      constexpr int I = decltype(ic)::value;
      const bool fl = ((lk >> OPP[I]) & 1u) == 0;  // x + c_I is a fluid cell
      const uint32_t tgt = fl ? src_of<OPP[I]>(p, q) : c;  // x + c_I (the cell itself across a wall)
      const uint32_t e = fl ? (uint32_t)I * (uint32_t)p.nc + tgt : (uint32_t)OPP[I] * (uint32_t)p.nc + c;
      gather_to_lds(rq, &sq[I][wb], e * PB);
      if constexpr (P64) gather_to_lds(rq, &sqh[I][wb], e * PB + 4u);
      gather_to_lds(rp, &sp[I][wb], tgt * 4u);
      if (a.rho_prev) gather_to_lds(rr, &sr[I][wb], tgt * 4u);
    });
  }

  // ---- forward recompute from the record --------------------------------
  // the record holds the filled values; the Zou-He fills are recomputed for
  // their transposes below (the extrapolation's unknowns are inputs)
  const bool extrap = p.outlet == 2;
  if (!(extrap && (lk & LK_OUT))) open_fill(p, q.row, lk, t, a.shape, a.wave, nullptr, d);
  Macro<R> M;
  macro<R, AN>(p, phx_f, d, omp, M);
  const R phx = (R)phx_f;
  const R iphi = fast_rcp(phx);
  const Sums<R> sm = moment_sums<R>(d);
  const auto& kc = p.d;
  const R iU = kc.iU;
  const R S = phx + sm.s * iU;  // sum f = phi rho
  const R mx = sm.mx * iU, my = sm.my * iU, mz = sm.mz * iU;
  const R om1 = 1.0 - phx;
  const R kn = kc.kcd * kc.nu_d;
  const R dark = kn * om1 * om1 * iphi * iphi;  // phi nu / k
  const R C0 = 0.5 + 0.25 * dark;
  const R D = phx * dark;                       // phi^2 nu / k
  const R rho = M.rho, ux = M.ux, uy = M.uy, uz = M.uz, uu = M.uu;
  const R Fx = M.Fx, Fy = M.Fy, Fz = M.Fz;
  const R om = M.omega;
  const R Nn = M.pnorm;  // |Pi|_F
  // Carreau-Yasuda viscosity and its derivative in the shear rate, in FP64
  // like the forward passes of the adjoint
  const R shear = M.shear_r;
  const R la = M.cy_la, fac = M.cy_fac;  // (lambda g)^a and (1 + (lambda g)^a)^((n-1)/a)
  // derivative of (lambda g)^a in g
  const R dla = p.cy_a2 ? 2.0 * kc.lam * kc.lam * shear : ((la > 0.0 && shear > 0.0) ? kc.cy_a * la * fast_rcp(shear) : 0.0);
  const R hh = 1.0 + la;
  const R nu = kc.nu_inf + kc.dnu * fac;
  const R dnu = kc.dnu * kc.cy_e * fac * fast_rcp(hh) * dla;

  // ---- the adjoint of the post-collision populations (staged in LDS) ------
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  // as stored (FP32 or FP64); FP32 values are widened exactly where used, which
  // keeps them in half the registers
  auto rdq = [&](int i) -> PH {
    if constexpr (P64) {
      const uint64_t lo = __builtin_bit_cast(uint32_t, sq[i][tid]), hi = __builtin_bit_cast(uint32_t, sqh[i][tid]);
      return __builtin_bit_cast(double, lo | (hi << 32));
    } else {
      return sq[i][tid];
    }
  };
  PH qh[Q];
  qh[0] = rdq(0);
  uint32_t fmask = 0;
  R sfl = 0.0, sjump = 0.0;
  sfor<1, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    const bool fl = ((lk >> OPP[I]) & 1u) == 0;  // x + c_I is a fluid cell
    const R pn = (R)sp[I][tid];
    qh[I] = rdq(I);
    const R ai = (R)kw(I) * (1.0 / 36.0) * (R)qh[I];
    sfl += fl ? ai : 0.0;
    sjump += fl ? ai * (pn - phx) : 0.0;
    fmask |= fl ? (1u << I) : 0u;
  });

  // moments of a_i = w_i qhat_i (exact weights 36 w_i / 36)
  R av[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) av[i] = (R)kw(i) * (R)qh[i] * (1.0 / 36.0);
  R s0 = 0.0, qd = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) { s0 += av[i]; qd += (R)qh[i] * (R)d[i]; }
  qd *= iU;  // sum qhat_i (f_i - w_i phi)
  const R s1x = (av[1] + av[7] + av[9] + av[11] + av[13]) - (av[2] + av[8] + av[10] + av[12] + av[14]);
  const R s1y = (av[3] + av[7] + av[10] + av[15] + av[17]) - (av[4] + av[8] + av[9] + av[16] + av[18]);
  const R s1z = (av[5] + av[11] + av[14] + av[15] + av[18]) - (av[6] + av[12] + av[13] + av[16] + av[17]);
  R s2[6];
  s2[0] = av[1] + av[2] + av[7] + av[8] + av[9] + av[10] + av[11] + av[12] + av[13] + av[14];
  s2[1] = av[3] + av[4] + av[7] + av[8] + av[9] + av[10] + av[15] + av[16] + av[17] + av[18];
  s2[2] = av[5] + av[6] + av[11] + av[12] + av[13] + av[14] + av[15] + av[16] + av[17] + av[18];
  s2[3] = (av[7] + av[8]) - (av[9] + av[10]);
  s2[4] = (av[11] + av[12]) - (av[13] + av[14]);
  s2[5] = (av[15] + av[16]) - (av[17] + av[18]);

  const R pr = phx * rho;
  const R K = 1.0 - 0.5 * om, keep = 1.0 - om;
  const R uF = ux * Fx + uy * Fy + uz * Fz;
  R s2ux, s2uy, s2uz, s2Fx, s2Fy, s2Fz;
  sym_mv(s2, ux, uy, uz, s2ux, s2uy, s2uz);
  sym_mv(s2, Fx, Fy, Fz, s2Fx, s2Fy, s2Fz);
  const R s1u = s1x * ux + s1y * uy + s1z * uz;
  const R s1F = s1x * Fx + s1y * Fy + s1z * Fz;
  const R us2u = ux * s2ux + uy * s2uy + uz * s2uz;
  const R us2F = ux * s2Fx + uy * s2Fy + uz * s2Fz;
  const R Aeq = phx * M.rm1 - 1.5 * pr * uu;

  // WSS objective term of a region wall cell: e = |tau|, tau = sigma n -
  // (n . sigma n) n, sigma = (omega/2 - 1) Pi.  d|tau| = t . d sigma n with
  // the unit t = tau/|tau|, i.e. the symmetric tensor sym(t n) against d sigma;
  // it reaches Pi scaled by (omega/2 - 1) and omega through Pi/2.
  R wG[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  R wom = 0.0;
  if (kind == 1 && reg && ew != 0.0f) {
    float nw[3];
    if (wall_normal(lk, nw)) {
      R tau[3];
      const R tm = wall_tau(M, nw, tau);
      if (tm > 0.0) {
        const R e = (R)ew / tm;
        const R tx = e * tau[0], ty = e * tau[1], tz = e * tau[2];
        const R nx = nw[0], ny = nw[1], nz = nw[2];
        const R sh[6] = {tx * nx, ty * ny, tz * nz, 0.5 * (tx * ny + ty * nx), 0.5 * (tx * nz + tz * nx),
                         0.5 * (ty * nz + tz * ny)};
        const R sg = 0.5 * M.omega - 1.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) wG[k] = sg * sh[k];
        wom = 0.5 * (sh[0] * M.P[0] + sh[1] * M.P[1] + sh[2] * M.P[2] +
                     2.0 * (sh[3] * M.P[3] + sh[4] * M.P[4] + sh[5] * M.P[5]));
      }
    }
  }

  // collision: q = (1-omega) f + omega feq + K g + w rho (phi~ - phi)
  R omh = omh_in + wom + (Aeq * s0 + 3.0 * pr * s1u + 4.5 * pr * us2u - qd) -
          0.5 * (3.0 * s1F - 3.0 * s0 * uF + 9.0 * us2F);
  R uhx = K * (9.0 * s2Fx - 3.0 * s0 * Fx), uhy = K * (9.0 * s2Fy - 3.0 * s0 * Fy),
    uhz = K * (9.0 * s2Fz - 3.0 * s0 * Fz);
  R Fhx = K * (3.0 * s1x - 3.0 * s0 * ux + 9.0 * s2ux), Fhy = K * (3.0 * s1y - 3.0 * s0 * uy + 9.0 * s2uy),
    Fhz = K * (3.0 * s1z - 3.0 * s0 * uz + 9.0 * s2uz);
  // equilibrium w phi rho (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u), weighted by omega
  const R brk = om * (s0 * (1.0 - 1.5 * uu) + 3.0 * s1u + 4.5 * us2u);
  const R pro = pr * om;
  uhx += pro * (3.0 * s1x + 9.0 * s2ux - 3.0 * s0 * ux);
  uhy += pro * (3.0 * s1y + 9.0 * s2uy - 3.0 * s0 * uy);
  uhz += pro * (3.0 * s1z + 9.0 * s2uz - 3.0 * s0 * uz);
  R rhoh = phx * brk + sjump;
  R phh = rho * brk - rho * sfl;

  // relaxation rate omega = 2 rho / (6 nu + rho), nu = CY(shear)
  const R den6 = 6.0 * nu + rho;
  const R id2 = fast_rcp(den6 * den6);
  rhoh += omh * 12.0 * nu * id2;
  const R nuh = -omh * 12.0 * rho * id2;
  const R gh = nuh * dnu;
  const R irho = fast_rcp(rho);
  const R omph = gh * 3.0 * Nn * irho;      // adjoint of omega_prev
  const R Nh = gh * 3.0 * (R)omp * irho;
  rhoh -= gh * shear * irho;
  // Pi = sum f c c - phi rho (I/3 + u u) + (F u + u F)/2, |Pi|_F
  const R gsc = Nn > 0.0 ? Nh * fast_rcp(Nn) : 0.0;
  R G[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) G[k] = gsc * M.P[k] + wG[k];
  R Gux, Guy, Guz, GFx, GFy, GFz;
  sym_mv(G, ux, uy, uz, Gux, Guy, Guz);
  sym_mv(G, Fx, Fy, Fz, GFx, GFy, GFz);
  const R tP = (G[0] + G[1] + G[2]) * (1.0 / 3.0) + ux * Gux + uy * Guy + uz * Guz;
  rhoh -= phx * tP;
  phh -= rho * tP;
  uhx += GFx - 2.0 * pr * Gux;
  uhy += GFy - 2.0 * pr * Guy;
  uhz += GFz - 2.0 * pr * Guz;
  Fhx += Gux; Fhy += Guy; Fhz += Guz;
  // kinetic-energy objective e = rho |u|^2 / 2 on region cells
  const R eh = (reg && kind == 0) ? (R)ew : 0.0;
  rhoh += eh * 0.5 * uu;
  uhx += eh * rho * ux; uhy += eh * rho * uy; uhz += eh * rho * uz;
  // force F = rho (g - D u - E |u| u), D = phi^2 nu / k and, with Forchheimer
  // drag, E = phi^3 C_F sqrt(1/k) = K2 (1 - phi) for 0 < phi <= 1 (C_F = 1.75 /
  // sqrt(150 phi^3)), K2 = 1.75 sqrt(K_c / (150 d^2)); d|u|/du := 0 at u = 0.
  // Anisotropic (AN): F = rho (g - D M^-1 u - E |u| M^-1/2 u).
  const bool forch = p.forch != 0;
  const R K2 = kc.fk2;
  const R E = forch ? K2 * om1 : 0.0;
  const R un = forch ? rsqrt_(uu) : 0.0;
  const R dD = -kn * (1.0 - phx * phx) * iphi * iphi;      // dD/dphi
  const R ddark = -2.0 * kn * om1 * iphi * iphi * iphi;    // d(phi nu / k)/dphi
  rhoh += (Fhx * Fx + Fhy * Fy + Fhz * Fz) * irho;
  R vhx, vhy, vhz;
  const R iS = fast_rcp(S);
  const R vx = mx * iS + 0.5 * kc.gx * iphi, vy = my * iS + 0.5 * kc.gy * iphi, vz = mz * iS + 0.5 * kc.gz * iphi;
  if constexpr (AN) {
    R kdx, kdy, kdz, khx, khy, khz, mfx, mfy, mfz, hfx, hfy, hfz;
    sym_mv(kc.Mi, ux, uy, uz, kdx, kdy, kdz);
    sym_mv(kc.Mh, ux, uy, uz, khx, khy, khz);
    sym_mv(kc.Mi, Fhx, Fhy, Fhz, mfx, mfy, mfz);
    sym_mv(kc.Mh, Fhx, Fhy, Fhz, hfx, hfy, hfz);
    uhx -= rho * (D * mfx + E * un * hfx);
    uhy -= rho * (D * mfy + E * un * hfy);
    uhz -= rho * (D * mfz + E * un * hfz);
    const R Fkd = Fhx * kdx + Fhy * kdy + Fhz * kdz, Fkh = Fhx * khx + Fhy * khy + Fhz * khz;
    if (forch && un > 0.0) {
      const R t = rho * E * Fkh / un;
      uhx -= t * ux; uhy -= t * uy; uhz -= t * uz;
      phh += rho * un * Fkh * K2;
    }
    phh -= rho * Fkd * dD;
    // the fixed-point iterates u_{m+1} = X_m^-1 v, X_m = A + |u_m| B, u_0 = v,
    // A = Id + (phi nu / 2k) M^-1, B = C1 M^-1/2: back through the iterates,
    // recomputing u_m from v each time
    const R ha = 0.5 * dark, hb = forch ? 0.5 * K2 * om1 * iphi : 0.0;
    // y = X^-1 b for X = A + n B (symmetric: the adjugate over the determinant).
    // X is formed from the uniform shape matrices at each solve rather than
    // kept per work-item, which keeps the kernel's registers down.
    auto solve = [&](R n, R bx, R by, R bz, R& yx, R& yy, R& yz) {
      R X[6];
      const R nb = n * hb;
#pragma unroll
      for (int k = 0; k < 6; ++k) X[k] = ha * kc.Mi[k] + nb * kc.Mh[k] + (k < 3 ? 1.0 : 0.0);
      const R a00 = X[1] * X[2] - X[5] * X[5], a11 = X[0] * X[2] - X[4] * X[4], a22 = X[0] * X[1] - X[3] * X[3];
      const R a01 = X[4] * X[5] - X[3] * X[2], a02 = X[3] * X[5] - X[4] * X[1], a12 = X[3] * X[4] - X[0] * X[5];
      const R idet = fast_rcp(X[0] * a00 + X[3] * a01 + X[4] * a02);
      yx = (a00 * bx + a01 * by + a02 * bz) * idet;
      yy = (a01 * bx + a11 * by + a12 * bz) * idet;
      yz = (a02 * bx + a12 * by + a22 * bz) * idet;
    };
    R ubx = uhx, uby = uhy, ubz = uhz;  // adjoint of u_{m+1}
    vhx = 0.0; vhy = 0.0; vhz = 0.0;
    // only two contractions of the adjoints of A and B are needed:
    // aM = sum_m Xh_m : M^-1 and bM = sum_m n_m Xh_m : M^-1/2
    R aM = 0.0, bM = 0.0;
    for (int m = p.an_iters - 1; m >= 0; --m) {
      R ax = vx, ay = vy, az = vz;  // u_m
      for (int j = 0; j < m; ++j) solve(rsqrt_(ax * ax + ay * ay + az * az), vx, vy, vz, ax, ay, az);
      const R n = rsqrt_(ax * ax + ay * ay + az * az);
      R bx, by, bz, wx, wy, wz;
      solve(n, vx, vy, vz, bx, by, bz);     // u_{m+1}
      solve(n, ubx, uby, ubz, wx, wy, wz);  // X^-1 applied to the adjoint (X symmetric)
      vhx += wx; vhy += wy; vhz += wz;
      const R Xh[6] = {-wx * bx, -wy * by, -wz * bz, -(wx * by + wy * bx), -(wx * bz + wz * bx),
                       -(wy * bz + wz * by)};
      R xi = 0.0, xh = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        xi += Xh[k] * kc.Mi[k];
        xh += Xh[k] * kc.Mh[k];
      }
      aM += xi;
      bM += n * xh;
      // d/dn of X = n B, contracted with Xh, then through n = |u_m|
      const R g = n > 0.0 ? hb * xh * fast_rcp(n) : 0.0;
      ubx = g * ax; uby = g * ay; ubz = g * az;
    }
    vhx += ubx; vhy += uby; vhz += ubz;  // u_0 = v
    phh += aM * 0.5 * ddark;
    if (forch) phh += bM * (-0.5 * K2 * iphi * iphi);
  } else {
    uhx -= rho * D * Fhx; uhy -= rho * D * Fhy; uhz -= rho * D * Fhz;
    const R Dh = -rho * (Fhx * ux + Fhy * uy + Fhz * uz);
    phh += Dh * dD;
    if (forch && un > 0.0) {
      const R ku = rho * E * (Fhx * ux + Fhy * uy + Fhz * uz) / un;
      uhx -= rho * E * un * Fhx + ku * ux;
      uhy -= rho * E * un * Fhy + ku * uy;
      uhz -= rho * E * un * Fhz + ku * uz;
      phh -= Dh * un * K2;
    }
    // u = v / den: without Forchheimer den = 2 C0; with it den = C0 + sqrt(C0^2
    // + C1 |v|), C1 = phi^2 C_F sqrt(1/k) / 2 = K2 (1 - phi) / (2 phi)
    R C0h;
    if (!forch) {
      const R i2c = fast_rcp(2.0 * C0);
      vhx = uhx * i2c; vhy = uhy * i2c; vhz = uhz * i2c;
      C0h = -(uhx * ux + uhy * uy + uhz * uz) * 2.0 * i2c;
    } else {
      const R C1 = 0.5 * K2 * om1 * iphi;
      const R vn = rsqrt_(vx * vx + vy * vy + vz * vz);
      const R sq = rsqrt_(C0 * C0 + C1 * vn);
      const R iden = fast_rcp(C0 + sq);
      vhx = uhx * iden; vhy = uhy * iden; vhz = uhz * iden;
      const R denh = -(uhx * ux + uhy * uy + uhz * uz) * iden;
      const R isq = sq > 0.0 ? 0.5 * fast_rcp(sq) : 0.0;
      C0h = denh * (1.0 + 2.0 * C0 * isq);
      const R C1h = denh * vn * isq;
      const R vnh = denh * C1 * isq;
      if (vn > 0.0) {
        const R g = vnh * fast_rcp(vn);
        vhx += g * vx; vhy += g * vy; vhz += g * vz;
      }
      phh += C1h * (-0.5 * K2 * iphi * iphi);
    }
    phh += 0.25 * C0h * ddark;
  }
  // v = m / S + g / (2 phi)
  const R mhx = vhx * iS, mhy = vhy * iS, mhz = vhz * iS;
  R Sh = -(vhx * mx + vhy * my + vhz * mz) * iS * iS;
  phh -= (vhx * kc.gx + vhy * kc.gy + vhz * kc.gz) * 0.5 * iphi * iphi;
  // rho = S / phi
  Sh += rhoh * iphi;
  phh -= rhoh * rho * iphi;

  // adjoint of the (filled) pulled populations
  R fh[Q];
  fh[0] = keep * (R)qh[0] + Sh;
  sfor<1, Q>([&](auto ic) {
    constexpr int I = decltype(ic)::value;
    constexpr int cx = CX[I], cy = CY[I], cz = CZ[I];
    fh[I] = keep * (R)qh[I] + Sh + mhx * (R)cx + mhy * (R)cy + mhz * (R)cz + (R)(cx * cx) * G[0] +
            (R)(cy * cy) * G[1] + (R)(cz * cz) * G[2] +
            2.0 * ((R)(cx * cy) * G[3] + (R)(cx * cz) * G[4] + (R)(cy * cz) * G[5]);
  });

  // the -x neighbour of an extrapolation-outflow cell: its c_x = -1 pulled
  // values enter the next step's unknowns with weight c_s
  if (extrap && (lk & LK_UPS)) {
    const double* e = a.aside_in + (size_t)q.row * 5;
#pragma unroll
    for (int k = 0; k < 5; ++k) fh[XOUT[k]] += (R)CS * e[k];
  }
  // transpose of the open-face fill: the unknowns' adjoints flow to the knowns
  const bool in = (lk & LK_IN) != 0;
  const bool outl = (lk & LK_OUT) != 0;
  if (outl && extrap) {
    // kept unknowns: total adjoint = this step's part + (1 - c_s) (or 1
    // without a fluid -x neighbour) times the next step's; it goes to the row
    // buffer, not to the pulled-value adjoints (no producer streams there)
    const double* e = a.aside_in + (size_t)q.row * 5;
    double* o = a.aside_out + (size_t)q.row * 5;
    const R wo = ((lk >> 1) & 1u) ? (R)1 : (R)1 - (R)CS;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const bool unk = (lk >> (LK_UNK + k)) & 1u;
      o[k] = unk ? (double)(fh[XOUT[k]] + wo * e[k]) : 0.0;
      if (unk) fh[XOUT[k]] = 0.0;
    }
  }
  if (in) {
    const R uin = (R)inflow_amplitude(p, a.wave, t) * (R)a.shape[q.row];
    fh[2] += fh[1]; fh[8] += fh[7]; fh[10] += fh[9]; fh[12] += fh[11]; fh[14] += fh[13];
    const R rinh = uin * (1.0 / 3.0) * fh[1] + uin * (1.0 / 6.0) * (fh[7] + fh[9] + fh[11] + fh[13]);
    const R nyh = 0.5 * (fh[9] - fh[7]), nzh = 0.5 * (fh[13] - fh[11]);
    const R k = rinh / (1.0 - uin);
    fh[0] += k; fh[3] += k; fh[4] += k; fh[5] += k; fh[6] += k; fh[15] += k; fh[16] += k; fh[17] += k; fh[18] += k;
    fh[2] += 2.0 * k; fh[8] += 2.0 * k; fh[10] += 2.0 * k; fh[12] += 2.0 * k; fh[14] += 2.0 * k;
    fh[3] += nyh; fh[4] -= nyh; fh[15] += nyh; fh[16] -= nyh; fh[17] += nyh; fh[18] -= nyh;
    fh[5] += nzh; fh[6] -= nzh; fh[15] += nzh; fh[16] -= nzh; fh[17] -= nzh; fh[18] += nzh;
    fh[1] = 0.0; fh[7] = 0.0; fh[9] = 0.0; fh[11] = 0.0; fh[13] = 0.0;
  } else if (outl && !extrap) {
    const R ro = kc.rho_out;
    fh[1] += fh[2]; fh[7] += fh[8]; fh[9] += fh[10]; fh[11] += fh[12]; fh[13] += fh[14];
    const R uxh = -ro * (1.0 / 3.0) * fh[2] - ro * (1.0 / 6.0) * (fh[8] + fh[10] + fh[12] + fh[14]);
    const R nyh = 0.5 * (fh[8] - fh[10]), nzh = 0.5 * (fh[12] - fh[14]);
    const R k = uxh / ro;
    fh[0] += k; fh[3] += k; fh[4] += k; fh[5] += k; fh[6] += k; fh[15] += k; fh[16] += k; fh[17] += k; fh[18] += k;
    fh[1] += 2.0 * k; fh[7] += 2.0 * k; fh[9] += 2.0 * k; fh[11] += 2.0 * k; fh[13] += 2.0 * k;
    fh[3] += nyh; fh[4] -= nyh; fh[15] += nyh; fh[16] -= nyh; fh[17] += nyh; fh[18] -= nyh;
    fh[5] += nzh; fh[6] -= nzh; fh[15] += nzh; fh[16] -= nzh; fh[17] -= nzh; fh[18] += nzh;
    fh[2] = 0.0; fh[8] = 0.0; fh[10] = 0.0; fh[12] = 0.0; fh[14] = 0.0;
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) sto((PH*)a.ph_out, (uint32_t)i * (uint32_t)p.nc + c, (PH)fh[i]);
  a.omh[c] = omph;

  // porosity-jump term of step n-1: q_i(x - c_i) depends on phi(x) when
  // x - c_i is a fluid producer; its adjoint is w_i rho_{n-1}(x - c_i) fh_i(x).
  if (a.rho_prev) {
    sfor<1, Q>([&](auto ic) {
      constexpr int J = decltype(ic)::value;
      // rho_{n-1}(x + c_J), staged in LDS; every slot is read and the sum
      // selected, so that the LDS reads are not serialised behind branches
      const R t = fma((R)kw(J) * (1.0 / 36.0) * (R)sr[J][tid], fh[OPP[J]], phh);
      phh = (fmask & (1u << J)) ? t : phh;
    });
  }
  a.phih[c] = phih_in + phh;
}

// Rest state f_i(0, x) = w_i phi(x) on the known links (and on the
// extrapolation outflow's unknowns, whose adjoints of step 0 are in aside0),
// then scatter the total into the box-layout gradient.
template <class PH>
__global__ __launch_bounds__(BLOCK) void k_adj_final(Params p, const uint32_t* code, const uint32_t* links,
                                                     const uint32_t* rowbox, const PH* ph0, const double* total,
                                                     const double* aside0, float* grad) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= (uint32_t)p.nc) return;
  const uint32_t lk = links[c];
  if (lk & LK_DEAD) return;
  const Pos q = position(p, c, code[c]);
  double s = total[c];
#pragma unroll
  for (int i = 0; i < Q; ++i) s += (double)kw(i) * (1.0 / 36.0) * (double)ldo(ph0, (uint32_t)i * (uint32_t)p.nc + c);
  if (p.outlet == 2 && (lk & LK_OUT)) {
#pragma unroll
    for (int k = 0; k < 5; ++k) s += (double)kw(XOUT[k]) * (1.0 / 36.0) * aside0[(size_t)q.row * 5 + k];
  }
  grad[(size_t)rowbox[q.row] + (size_t)q.x] = (float)s;
}

}  // namespace lbm
