// Launches of the D3Q27 kernels for one storage type S (instantiated in
// k27_f32.hip and k27_16.hip).
#pragma once
#include "runtime.hpp"

namespace lbmrt {

template <class S>
void step27(lbm_ctx* c, const lbm::q27::Bufs27& b, int diag) {
  constexpr int NT = std::is_same<S, float>::value ? 256 : STEP_NT16;
  const dim3 grid(c->sblk), block(NT);
  with_shift(c->grid.shift_mode, [&](auto shw) {
    constexpr bool SH = decltype(shw)::value;
    with_arith<S>(c->amode, [&](auto rt) {
      using R = typename decltype(rt)::T;
      constexpr bool PJ = decltype(rt)::proj;
      with_rounding<S>(c->grid.rounding, [&](auto cr) {
        constexpr int RM = decltype(cr)::value;
        with_parity(c->t, [&](auto odd) {
          constexpr bool OD = decltype(odd)::value;
          if (diag == 0)
            hipLaunchKernelGGL((q27::k_step<S, SH, OD, 0, R, PJ, NT, RM>), grid, block, 0, c->stream, c->P, b);
          else
            hipLaunchKernelGGL((q27::k_step<S, SH, OD, 1, R, PJ, NT, RM>), grid, block, 0, c->stream, c->P, b);
        });
      });
    });
  });
}

template <class S>
void moments27(lbm_ctx* c, const lbm::q27::Bufs27& b, bool diag, float* rho, float* u, float* shear, float* omega,
               float* sigma, float* tau) {
  const uint32_t t = (uint32_t)c->t;
  const dim3 grid(c->nblk), block(BLOCK);
  with_shift(c->grid.shift_mode, [&](auto shw) {
    constexpr bool SH = decltype(shw)::value;
    with_arith<S>(c->amode == 2 ? 2 : 0, [&](auto rt) {
      using R = typename decltype(rt)::T;
      with_parity(c->t, [&](auto odd) {
        constexpr bool OD = decltype(odd)::value;
        if (diag)
          hipLaunchKernelGGL((q27::k_moments<S, SH, OD, true, R>), grid, block, 0, c->stream, c->P, b, t, c->nbox,
                             rho, u, shear, omega, sigma, tau);
        else
          hipLaunchKernelGGL((q27::k_moments<S, SH, OD, false, R>), grid, block, 0, c->stream, c->P, b, t, c->nbox,
                             rho, u, shear, omega, sigma, tau);
      });
    });
  });
}

template <class S>
void init27(lbm_ctx* c, const lbm::q27::Bufs27& b) {
  with_shift(c->grid.shift_mode, [&](auto shw) {
    hipLaunchKernelGGL((q27::k_init<S, decltype(shw)::value>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, c->P, b,
                       c->omega0);
  });
}

template <class S>
void gather27(lbm_ctx* c, const lbm::q27::Bufs27& b, float* dst) {
  with_parity(c->t, [&](auto odd) {
    hipLaunchKernelGGL((q27::k_gather_state<S, decltype(odd)::value>), dim3(c->nblk), dim3(BLOCK), 0, c->stream,
                       c->P, b, dst);
  });
}

template <class S>
void scatter27(lbm_ctx* c, const lbm::q27::Bufs27& b, const float* src) {
  with_parity(c->t, [&](auto odd) {
    hipLaunchKernelGGL((q27::k_scatter_state<S, decltype(odd)::value>), dim3(c->nblk), dim3(BLOCK), 0, c->stream,
                       c->P, b, src);
  });
}

}  // namespace lbmrt

#define LBM_INSTANTIATE27(S)                                                                                      \
  namespace lbmrt {                                                                                               \
  template void step27<S>(lbm_ctx*, const lbm::q27::Bufs27&, int);                                                \
  template void moments27<S>(lbm_ctx*, const lbm::q27::Bufs27&, bool, float*, float*, float*, float*, float*,     \
                             float*);                                                                             \
  template void init27<S>(lbm_ctx*, const lbm::q27::Bufs27&);                                                     \
  template void gather27<S>(lbm_ctx*, const lbm::q27::Bufs27&, float*);                                           \
  template void scatter27<S>(lbm_ctx*, const lbm::q27::Bufs27&, const float*);                                    \
  }
