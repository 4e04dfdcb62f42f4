// Launches of the D3Q19 kernels for one storage type S (instantiated in
// k19_f32.hip, k19_f16.hip and k19_bf16.hip).
#pragma once
#include "runtime.hpp"

namespace lbmrt {

template <class S>
void step19(lbm_ctx* c, const lbm::Bufs& b, int diag, bool rec) {
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
          // AN: anisotropic permeability (every form, the adjoint's included)
          auto go = [&](auto an) {
            constexpr bool AN = decltype(an)::value;
            if (diag == 0 && !rec) {
              if constexpr (sizeof(S) == 2) {
                // wave records: when the state exceeds the Infinity Cache, and
                // with rounding to nearest, whose step has the fewest VALU
                // instructions (with stochastic rounding they gain nothing)
                if (c->beyond_cache || RM == 0)
                  hipLaunchKernelGGL((k_step<S, SH, OD, 0, false, R, PJ, NT, AN, RM, true>), grid, block, 0,
                                     c->stream, c->P, b);
                else
                  hipLaunchKernelGGL((k_step<S, SH, OD, 0, false, R, PJ, NT, AN, RM, false>), grid, block, 0,
                                     c->stream, c->P, b);
              } else {
                hipLaunchKernelGGL((k_step<S, SH, OD, 0, false, R, PJ, NT, AN, RM>), grid, block, 0, c->stream,
                                   c->P, b);
              }
            } else if (diag == 1) {
              hipLaunchKernelGGL((k_step<S, SH, OD, 1, false, R, PJ, NT, AN, RM>), grid, block, 0, c->stream, c->P,
                                 b);
            } else if constexpr (std::is_same<S, float>::value) {
              // the adjoint's forms (FP32 storage only)
              if (rec) {
                // the recording step, with the objective term when the
                // forward pass records the last segment
                if constexpr (!SH) {
                  if (diag == 2)
                    hipLaunchKernelGGL((k_step<S, false, OD, 2, true, R, PJ, NT, AN>), grid, block, 0, c->stream,
                                       c->P, b);
                  else if (diag == 3)
                    hipLaunchKernelGGL((k_step<S, false, OD, 3, true, R, PJ, NT, AN>), grid, block, 0, c->stream,
                                       c->P, b);
                  else
                    hipLaunchKernelGGL((k_step<S, false, OD, 0, true, R, PJ, NT, AN>), grid, block, 0, c->stream,
                                       c->P, b);
                }
              } else if (diag == 2) {
                hipLaunchKernelGGL((k_step<S, SH, OD, 2, false, R, PJ, NT, AN>), grid, block, 0, c->stream, c->P,
                                   b);
              } else {
                hipLaunchKernelGGL((k_step<S, SH, OD, 3, false, R, PJ, NT, AN>), grid, block, 0, c->stream, c->P,
                                   b);
              }
            }
          };
          if (c->P.an_iters > 0) go(std::true_type{});
          else go(std::false_type{});
        });
      });
    });
  });
}

template <class S>
void moments19(lbm_ctx* c, const lbm::Bufs& b, bool diag, float* rho, float* u, float* shear, float* omega,
               float* sigma, float* tau) {
  const uint32_t t = (uint32_t)c->t;
  const dim3 grid(c->nblk), block(BLOCK);
  with_shift(c->grid.shift_mode, [&](auto shw) {
    constexpr bool SH = decltype(shw)::value;
    with_arith<S>(c->amode == 2 ? 2 : 0, [&](auto rt) {
      using R = typename decltype(rt)::T;
      with_parity(c->t, [&](auto odd) {
        constexpr bool OD = decltype(odd)::value;
        const bool an = c->P.an_iters > 0;
        if (diag && an)
          hipLaunchKernelGGL((k_moments<S, SH, OD, true, R, true>), grid, block, 0, c->stream, c->P, b, t, c->nbox,
                             rho, u, shear, omega, sigma, tau);
        else if (diag)
          hipLaunchKernelGGL((k_moments<S, SH, OD, true, R>), grid, block, 0, c->stream, c->P, b, t, c->nbox, rho, u,
                             shear, omega, sigma, tau);
        else if (an)
          hipLaunchKernelGGL((k_moments<S, SH, OD, false, R, true>), grid, block, 0, c->stream, c->P, b, t, c->nbox,
                             rho, u, shear, omega, sigma, tau);
        else
          hipLaunchKernelGGL((k_moments<S, SH, OD, false, R>), grid, block, 0, c->stream, c->P, b, t, c->nbox, rho,
                             u, shear, omega, sigma, tau);
      });
    });
  });
}

template <class S>
void init19(lbm_ctx* c, const lbm::Bufs& b) {
  with_shift(c->grid.shift_mode, [&](auto shw) {
    hipLaunchKernelGGL((k_init<S, decltype(shw)::value>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, c->P, b,
                       c->omega0);
  });
}

template <class S>
void gather19(lbm_ctx* c, const lbm::Bufs& b, float* dst) {
  with_parity(c->t, [&](auto odd) {
    hipLaunchKernelGGL((k_gather_state<S, decltype(odd)::value>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, c->P, b,
                       dst);
  });
}

template <class S>
void scatter19(lbm_ctx* c, const lbm::Bufs& b, const float* src) {
  with_parity(c->t, [&](auto odd) {
    hipLaunchKernelGGL((k_scatter_state<S, decltype(odd)::value>), dim3(c->nblk), dim3(BLOCK), 0, c->stream, c->P,
                       b, src);
  });
}

}  // namespace lbmrt

#define LBM_INSTANTIATE19(S)                                                                                    \
  namespace lbmrt {                                                                                             \
  template void step19<S>(lbm_ctx*, const lbm::Bufs&, int, bool);                                               \
  template void moments19<S>(lbm_ctx*, const lbm::Bufs&, bool, float*, float*, float*, float*, float*, float*); \
  template void init19<S>(lbm_ctx*, const lbm::Bufs&);                                                          \
  template void gather19<S>(lbm_ctx*, const lbm::Bufs&, float*);                                                \
  template void scatter19<S>(lbm_ctx*, const lbm::Bufs&, const float*);                                         \
  }
