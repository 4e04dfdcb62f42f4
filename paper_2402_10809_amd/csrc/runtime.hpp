// Host runtime shared by the translation units of liblbm.so: the context, the
// workspace layout, the launch helpers, and the per-storage launch functions
// (each family of kernels is instantiated in a translation unit of its own so
// that the library builds in parallel).
#pragma once
#include "lbm.h"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <type_traits>
#include <vector>

#include "layout.hpp"
#include "step.hpp"
#include "step27.hpp"

namespace lbmrt {

using namespace lbm;

// Error message of the last failure (thread-local) and status.
lbm_status fail(lbm_status s, const std::string& msg);

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }
inline size_t store_bytes(int storage) { return storage == LBM_STORE_FP32 ? 4 : 2; }
inline int qof(const lbm_grid& g) { return g.velocity_set == 27 ? 27 : 19; }
inline int blocks_for(int64_t n) { return (int)((n + BLOCK - 1) / BLOCK); }
inline int blocks_for_nt(int64_t n, int nt) { return (int)((n + nt - 1) / nt); }

// Workgroup size of the step kernel: 256 work-items with FP32 storage, 64 with
// the 16-bit forms (measured fastest for each on the large aneurysm).
constexpr int STEP_NT_MIN = 64;
constexpr int MAX_WAVE_TABLE = 1024;  // samples of a sampled inflow waveform
constexpr int STEP_NT16 = 256;  // work-items per workgroup of the 16-bit step kernels
// Infinity Cache (last-level, memory-side) of MI355X, bytes.
constexpr size_t INFINITY_CACHE_BYTES = (size_t)256 << 20;
inline int step_nt(int storage) { return storage == LBM_STORE_FP32 ? 256 : STEP_NT16; }

struct Layout {
  size_t A, code, links, phi, omega, delta, rel, winfo, shape, rowbox, stage, part, diag, obj, tc, wave, side;
  // adjoint
  size_t ck, rec, rho, ah0, ah1, omh, phih, aside;
  int nck, ckpt, T;
  size_t total;
};

}  // namespace lbmrt

// A context: its host layout (box, rows, per-cell tables, fluid-cell lists)
// plus the run's parameters, workspace and state.
struct lbm_ctx : lbmrt::HostLayout {
  lbm_grid grid{};
  lbm_rheology rh{};
  lbm_porous po{};
  lbm_open op{};
  size_t nbox = 0;
  int nblk = 0;                   // blocks of BLOCK work-items over the compact cells
  int sblk = 0;                   // blocks of the step kernel
  bool beyond_cache = false;      // the step's state (populations + per-cell arrays) exceeds the Infinity Cache
  int64_t nwss = 0;               // region cells on the wall (with a wall normal)
  int q = 19;                     // velocity set
  double U = 36.0;
  int device = 0;                 // HIP device of the workspace (current at lbm_create)
  std::vector<double> phi_f;      // porosity per fluid cell (host, for state transfer)
  bool phi_stale = false;         // phi_f predates a device-side porosity update
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  lbmrt::Layout L{};
  int64_t t = 0;                  // time; its parity selects the slot layout
  bool poisoned = false;
  lbm::Params P{};
  float omega0 = 1.0f;
  int amode = 1;                  // collision arithmetic: 0 FP32, 1 FP32 + projection, 2 FP64
};

#define HIP_TRY(ctx, expr)                                                                      \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) {                                                                     \
      if (ctx) (ctx)->poisoned = true;                                                          \
      return ::lbmrt::fail(LBM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    }                                                                                           \
  } while (0)

#define CTX_CHECK(ctx)                                                                          \
  do {                                                                                          \
    if (!(ctx)) return ::lbmrt::fail(LBM_E_INVALID, "null context");                            \
    if ((ctx)->poisoned) return ::lbmrt::fail(LBM_E_STATE, "context poisoned by an earlier device error"); \
  } while (0)

namespace lbmrt {

struct TF32 { using T = float; };
struct TF16 { using T = _Float16; };
struct TBF16 { using T = __bf16; };
// Arithmetic of the collision: FP32, FP32 with the FP64 momentum projection,
// or FP64.
struct RF32 { using T = float; static constexpr bool proj = false; };
struct RF32P { using T = float; static constexpr bool proj = true; };
struct RF64 { using T = double; static constexpr bool proj = false; };

template <class Fn>
void with_shift(int shw, Fn&& fn) {
  if (shw) fn(std::true_type{}); else fn(std::false_type{});
}

// Rounding of the 16-bit storage forms (lbm_rounding, see round16 in
// step.hpp); FP32 storage has one form.
template <class S, class Fn>
void with_rounding(int rounding, Fn&& fn) {
  using std::integral_constant;
  if constexpr (std::is_same<S, float>::value) fn(integral_constant<int, 0>{});
  else if (rounding == LBM_ROUND_NEAREST) fn(integral_constant<int, 0>{});
  else if (rounding == LBM_ROUND_CONSERVE) fn(integral_constant<int, 1>{});
  else fn(integral_constant<int, 2>{});
}

// Arithmetic for storage S: the FP64 and projected forms only exist for FP32
// storage.  mode: 0 FP32, 1 FP32 + projection, 2 FP64.
template <class S, class Fn>
void with_arith(int mode, Fn&& fn) {
  if constexpr (std::is_same<S, float>::value) {
    if (mode == 2) fn(RF64{});
    else if (mode == 1) fn(RF32P{});
    else fn(RF32{});
  } else {
    fn(RF32{});
  }
}

template <class Fn>
void with_parity(int64_t t, Fn&& fn) {
  if (t & 1) fn(std::true_type{}); else fn(std::false_type{});
}

Layout make_layout(const lbm_grid& g, int64_t nc, int64_t nrow, int T, int ckpt);
lbm::Bufs bufs(lbm_ctx* c);
lbm::q27::Bufs27 bufs27(lbm_ctx* c);

// Per-storage launch functions (kernels instantiated in their own units).
// diag: 0 none, 1 diagnostics partials, 2 region kinetic energy, 3 region
// wall shear stress, accumulated into the objective partials; rec: record
// the step for the adjoint (FP32 storage, shift mode 0 only).
template <class S> void step19(lbm_ctx* c, const lbm::Bufs& b, int diag, bool rec);
template <class S> void moments19(lbm_ctx* c, const lbm::Bufs& b, bool diag, float* rho, float* u, float* shear,
                                  float* omega, float* sigma, float* tau);
template <class S> void init19(lbm_ctx* c, const lbm::Bufs& b);
template <class S> void gather19(lbm_ctx* c, const lbm::Bufs& b, float* dst);
template <class S> void scatter19(lbm_ctx* c, const lbm::Bufs& b, const float* src);
template <class S> void step27(lbm_ctx* c, const lbm::q27::Bufs27& b, int diag);
template <class S> void moments27(lbm_ctx* c, const lbm::q27::Bufs27& b, bool diag, float* rho, float* u,
                                  float* shear, float* omega, float* sigma, float* tau);
template <class S> void init27(lbm_ctx* c, const lbm::q27::Bufs27& b);
template <class S> void gather27(lbm_ctx* c, const lbm::q27::Bufs27& b, float* dst);
template <class S> void scatter27(lbm_ctx* c, const lbm::q27::Bufs27& b, const float* src);

// Storage dispatch for the per-storage launch functions.
template <class Fn>
void with_storage(int storage, Fn&& fn) {
  if (storage == LBM_STORE_FP32) fn(TF32{});
  else if (storage == LBM_STORE_FP16) fn(TF16{});
  else fn(TBF16{});
}

// Kernels without a storage type (kmisc.hip).
void launch_finalize(hipStream_t s, const double* part, int nparts, int n, uint32_t ops, double* out);
void launch_set_time(hipStream_t s, uint32_t* tc, uint32_t t);
void launch_copy(hipStream_t s, const void* src, void* dst, size_t n16, unsigned blocks);
void launch_probe(hipStream_t s, int kind, const void* src, void* dst, size_t n16, unsigned blocks);
lbm_status set_porosity_device(lbm_ctx* c, const float* phib, uint32_t* bad_cell);
lbm_status launch_wave_info(lbm_ctx* c);

// Runtime operations shared by the ABI functions (lbm.hip).
lbm_status launch_init(lbm_ctx* c);
lbm_status launch_step(lbm_ctx* c, int diag, float* rec, float* rho_rec);
// dev_out: device area of the reduced vector (nullptr: the workspace's)
lbm_status finalize(lbm_ctx* c, const double* part, int nparts, int n, uint32_t ops, double* host_out,
                    double* dev_out = nullptr);
lbm_status gather_state(lbm_ctx* c, float* dst);
lbm_status scatter_state(lbm_ctx* c, const float* src);

}  // namespace lbmrt
