// lbm_adjoint: the reverse kernel and its checkpointing driver.
#include <algorithm>

#include "adjoint.hpp"
#include "runtime.hpp"

using namespace lbmrt;

// Host side of lbm_adjoint: forward pass with checkpoints, then segment-wise
// recompute (recording pulled values, omega_prev and density) and reverse
// steps.  The checkpoint of segment s (s >= 1) is the state one step before
// the segment start, so the recompute also records the density of the step
// before the segment, which the porosity-jump gather of the segment's first
// reverse step needs.  Checkpoints hold the gathered (layout-independent)
// state; the slot layout of a restored state follows the parity of its time.
// The forward pass records the last segment itself (that segment needs no
// checkpoint and no recompute); with one segment (ckpt_every >= T) nothing is
// recomputed.  The recompute reproduces the forward trajectory bit for bit,
// so the records are the same either way.
extern "C" lbm_status lbm_adjoint(lbm_ctx* c, const lbm_objective* obj, int T, int ckpt, double* J,
                                  float* dJ_dphi) {
  CTX_CHECK(c);
  if (!obj || !J) return fail(LBM_E_INVALID, "obj and J must not be NULL");
  if (T < 1 || ckpt < 1) return fail(LBM_E_INVALID, "T and ckpt_every must be >= 1");
  if (obj->t_begin < 0 || obj->t_end > T || obj->t_begin >= obj->t_end)
    return fail(LBM_E_INVALID, "objective window must satisfy 0 <= t_begin < t_end <= T");
  if (c->grid.storage != LBM_STORE_FP32 || c->grid.shift_mode != 0)
    return fail(LBM_E_INVALID, "the adjoint supports FP32 storage with shift mode 0");
  if (c->q != 19) return fail(LBM_E_INVALID, "the adjoint is built for D3Q19");
  if (obj->fp64_adjoint && (uint64_t)Q * (uint64_t)c->nc * 8u >= (1ull << 31))
    return fail(LBM_E_INVALID, "FP64 adjoint populations need 19 * 8 bytes per cell below 2 GiB");
  if (obj->kind != LBM_OBJ_KINETIC && obj->kind != LBM_OBJ_WSS) return fail(LBM_E_INVALID, "unknown objective kind");
  if (c->nreg == 0) return fail(LBM_E_INVALID, "the objective region has no fluid cell");
  if (obj->kind == LBM_OBJ_WSS && c->nwss == 0) return fail(LBM_E_INVALID, "the objective region has no wall cell");
  const int okind = obj->kind;
  const int64_t ncount = okind == LBM_OBJ_WSS ? c->nwss : c->nreg;
  // without a gradient output only J is computed: forward pass, no checkpoints
  const bool want_grad = dJ_dphi != nullptr;
  const Layout L = make_layout(c->grid, c->nc, c->nrow, want_grad ? T : 0, want_grad ? ckpt : 0);
  if (c->ws_bytes < L.total)
    return fail(LBM_E_WORKSPACE, "workspace too small for this adjoint: need " + std::to_string(L.total) + " bytes");
  // The forward passes compute the collision in FP64: the reverse steps
  // differentiate along the recorded trajectory, and FP32 rounding of the
  // per-cell scalars moves it by a few 1e-6 of J over thousands of steps.
  struct ArithScope {
    lbm_ctx* c;
    int saved;
    ~ArithScope() { c->amode = saved; }
  } arith_scope{c, c->amode};
  c->amode = 2;
  const size_t nc = (size_t)c->nc, nbox = c->nbox;
  const int nseg = (T + ckpt - 1) / ckpt;
  float* ck = (float*)(c->ws + L.ck);
  float* rec = (float*)(c->ws + L.rec);
  float* rho = (float*)(c->ws + L.rho);
  double* omh = (double*)(c->ws + L.omh);
  double* phih = (double*)(c->ws + L.phih);
  double* objp = (double*)(c->ws + L.obj);
  auto slot_rec = [&](int k) { return rec + (size_t)k * (Q + 1) * nc; };
  auto slot_rho = [&](int k) { return rho + (size_t)k * nc; };
  // checkpoint s: the state at time s * ckpt - 1 (c->t at the call)
  auto save_ck = [&](int s) -> lbm_status {
    float* dst = ck + (size_t)s * (Q + 1) * nc;
    lbm_status st = gather_state(c, dst);
    if (st != LBM_OK) return st;
    HIP_TRY(c, hipMemcpyAsync(dst + Q * nc, c->ws + c->L.omega, nc * 4, hipMemcpyDeviceToDevice, c->stream));
    return LBM_OK;
  };
  auto load_ck = [&](int s) -> lbm_status {
    const float* src = ck + (size_t)s * (Q + 1) * nc;
    c->t = (int64_t)s * ckpt - 1;
    launch_set_time(c->stream, (uint32_t*)(c->ws + c->L.tc), (uint32_t)c->t);
    lbm_status st = scatter_state(c, src);
    if (st != LBM_OK) return st;
    HIP_TRY(c, hipMemcpyAsync(c->ws + c->L.omega, src + Q * nc, nc * 4, hipMemcpyDeviceToDevice, c->stream));
    return LBM_OK;
  };

  // forward pass: objective and checkpoints
  lbm_status st = launch_init(c);
  if (st != LBM_OK) return st;
  HIP_TRY(c, hipMemsetAsync(objp, 0, (size_t)c->sblk * 8, c->stream));
  const int s_last = nseg - 1, t0_last = s_last * ckpt;
  for (int t = 0; t < T; ++t) {
    if (want_grad && (t + 1) % ckpt == 0 && (t + 1) / ckpt < s_last) {
      st = save_ck((t + 1) / ckpt);
      if (st != LBM_OK) return st;
    }
    const bool in = t >= obj->t_begin && t < obj->t_end;
    float* r = nullptr;
    float* rr = nullptr;
    if (want_grad && s_last >= 1 && t == t0_last - 1) {
      r = slot_rec(0);
      rr = slot_rho(0);
    } else if (want_grad && t >= t0_last) {
      r = slot_rec(t - t0_last + 1);
      rr = slot_rho(t - t0_last + 1);
    }
    st = launch_step(c, in ? (okind == LBM_OBJ_WSS ? 3 : 2) : 0, r, rr);
    if (st != LBM_OK) return st;
  }
  double jsum = 0.0;
  st = finalize(c, objp, c->sblk, 1, 0u, &jsum);
  if (st != LBM_OK) return st;
  const double ew = 1.0 / ((double)(obj->t_end - obj->t_begin) * (double)ncount);
  *J = jsum * ew;
  if (!want_grad) {
    st = launch_init(c);
    if (st != LBM_OK) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
  }

  // reverse sweep
  // adjoint of the pulled populations of steps n+1 and n, FP32 or FP64 (the
  // workspace holds room for FP64)
  const bool p64 = obj->fp64_adjoint != 0;
  const size_t pb = p64 ? 8 : 4;
  void* phn = (void*)(c->ws + L.ah0);
  void* pho = (void*)(c->ws + L.ah1);
  HIP_TRY(c, hipMemsetAsync(phn, 0, Q * nc * pb, c->stream));
  HIP_TRY(c, hipMemsetAsync(pho, 0, Q * nc * pb, c->stream));
  HIP_TRY(c, hipMemsetAsync(omh, 0, nc * 8, c->stream));
  HIP_TRY(c, hipMemsetAsync(phih, 0, nc * 8, c->stream));
  // extrapolation outflow: adjoints of the kept unknowns, per row, by parity
  // of the step (none after the last step)
  double* aside = (double*)(c->ws + L.aside);
  HIP_TRY(c, hipMemsetAsync(aside, 0, (size_t)2 * c->nrow * 5 * 8, c->stream));
  AdjBufs ab{};
  ab.code = (const uint32_t*)(c->ws + c->L.code);
  ab.links = (const uint32_t*)(c->ws + c->L.links);
  ab.delta = (const int*)(c->ws + c->L.delta);
  ab.phi = (const float*)(c->ws + c->L.phi);
  ab.shape = (const float*)(c->ws + c->L.shape);
  ab.wave = (const double*)(c->ws + c->L.wave);
  ab.omh = omh;
  ab.phih = phih;
  for (int s = nseg - 1; s >= 0; --s) {
    const int t0 = s * ckpt, t1 = std::min(T, t0 + ckpt);
    if (s < s_last) {
      if (s == 0) {
        st = launch_init(c);
        if (st != LBM_OK) return st;
      } else {
        st = load_ck(s);
        if (st != LBM_OK) return st;
        st = launch_step(c, 0, slot_rec(0), slot_rho(0));
        if (st != LBM_OK) return st;
      }
      for (int t = t0; t < t1; ++t) {
        st = launch_step(c, 0, slot_rec(t - t0 + 1), slot_rho(t - t0 + 1));
        if (st != LBM_OK) return st;
      }
    }
    for (int n = t1 - 1; n >= t0; --n) {
      const int k = n - t0 + 1;
      ab.rec = slot_rec(k);
      ab.rho_prev = n > 0 ? slot_rho(k - 1) : nullptr;
      ab.ph_next = phn;
      ab.ph_out = pho;
      ab.aside_in = aside + (size_t)((n + 1) & 1) * c->nrow * 5;
      ab.aside_out = aside + (size_t)(n & 1) * c->nrow * 5;
      const float ewn = (n >= obj->t_begin && n < obj->t_end) ? (float)ew : 0.0f;
      if (c->P.an_iters > 0 && p64)
        hipLaunchKernelGGL((k_adjoint<true, double>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, c->P, ab, (uint32_t)n,
                           ewn, okind);
      else if (c->P.an_iters > 0)
        hipLaunchKernelGGL((k_adjoint<true, float>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, c->P, ab, (uint32_t)n,
                           ewn, okind);
      else if (p64)
        hipLaunchKernelGGL((k_adjoint<false, double>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, c->P, ab,
                           (uint32_t)n, ewn, okind);
      else
        hipLaunchKernelGGL((k_adjoint<false, float>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, c->P, ab,
                           (uint32_t)n, ewn, okind);
      HIP_TRY(c, hipGetLastError());
      std::swap(phn, pho);
    }
  }
  HIP_TRY(c, hipMemsetAsync(dJ_dphi, 0, nbox * 4, c->stream));
  if (p64)
    hipLaunchKernelGGL(k_adj_final<double>, dim3(c->nblk), dim3(BLOCK), 0, c->stream, c->P, ab.code, ab.links,
                       (const uint32_t*)(c->ws + c->L.rowbox), (const double*)phn, (const double*)phih,
                       (const double*)aside, dJ_dphi);
  else
    hipLaunchKernelGGL(k_adj_final<float>, dim3(c->nblk), dim3(BLOCK), 0, c->stream, c->P, ab.code, ab.links,
                       (const uint32_t*)(c->ws + c->L.rowbox), (const float*)phn, (const double*)phih,
                       (const double*)aside, dJ_dphi);
  HIP_TRY(c, hipGetLastError());
  // leave the context at the rest state
  st = launch_init(c);
  if (st != LBM_OK) return st;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}
