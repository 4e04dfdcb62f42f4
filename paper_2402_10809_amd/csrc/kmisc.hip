// Kernels without a storage type: the fixed-order reduction of per-block
// partials, the time-counter set, and the streaming copy of the bandwidth
// reference.
#include "runtime.hpp"

namespace lbm {

// Reduce per-block partials (single workgroup, fixed order: deterministic).
// opmask holds 2 bits per entry: 0 sum, 1 max, 2 min.  Each work-item reads
// whole rows (the n entries of one block, contiguous) and accumulates every
// entry in its own register, rows i = tid, tid + BLOCK, ... in order; then one
// tree reduction per entry in LDS.  n <= FIN_MAX.
constexpr int FIN_MAX = 16;
__global__ __launch_bounds__(BLOCK) void k_finalize(const double* part, int nblk, int n, uint32_t opmask, double* out) {
  __shared__ double sh[BLOCK];
  double r[FIN_MAX];
#pragma unroll
  for (int k = 0; k < FIN_MAX; ++k) {
    const int op = (int)((opmask >> (2 * k)) & 3u);
    r[k] = op == 0 ? 0.0 : (op == 1 ? -1e300 : 1e300);
  }
  for (int i = threadIdx.x; i < nblk; i += BLOCK) {
    const double* row = part + (size_t)i * n;
#pragma unroll
    for (int k = 0; k < FIN_MAX; ++k) {
      if (k < n) {
        const int op = (int)((opmask >> (2 * k)) & 3u);
        const double v = row[k];
        r[k] = op == 0 ? r[k] + v : (op == 1 ? fmax(r[k], v) : fmin(r[k], v));
      }
    }
  }
#pragma unroll
  for (int k = 0; k < FIN_MAX; ++k) {
    if (k >= n) break;
    const int op = (int)((opmask >> (2 * k)) & 3u);
    sh[threadIdx.x] = r[k];
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

// Set the time counter slot of parity t & 1 to t (one work-item).
__global__ void k_set_time(uint32_t* tc, uint32_t t) {
  if (blockIdx.x == 0 && threadIdx.x == 0) tc[t & 1u] = t;
}

// Plain streaming copy (16-byte vectors), the achievable-bandwidth reference.
__global__ __launch_bounds__(BLOCK) void k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
  size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * BLOCK;
  for (; i < n; i += stride) dst[i] = src[i];
}

// Achievable-bandwidth references with more bytes in flight: every work-item
// moves four 16-byte vectors per iteration (issued before any is used), with
// non-temporal accesses (streamed past the caches).  k_read4 folds what it
// reads into one word per work-item so the loads cannot be dropped; k_write4
// stores a constant.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(BLOCK) void k_copy4(const u32x4* __restrict__ src, u32x4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * BLOCK;
  size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    u32x4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = __builtin_nontemporal_load(&src[i + k * stride]);
#pragma unroll
    for (int k = 0; k < 4; ++k) __builtin_nontemporal_store(v[k], &dst[i + k * stride]);
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(BLOCK) void k_read4(const u32x4* __restrict__ src, size_t n, uint32_t* __restrict__ out) {
  const size_t stride = (size_t)gridDim.x * BLOCK;
  size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
  uint32_t acc = 0;
  for (; i + 3 * stride < n; i += 4 * stride) {
    u32x4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = __builtin_nontemporal_load(&src[i + k * stride]);
#pragma unroll
    for (int k = 0; k < 4; ++k) acc ^= v[k].x ^ v[k].y ^ v[k].z ^ v[k].w;
  }
  for (; i < n; i += stride) {
    const u32x4 v = src[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  out[(size_t)blockIdx.x * BLOCK + threadIdx.x] = acc;
}

__global__ __launch_bounds__(BLOCK) void k_write4(u32x4* __restrict__ dst, size_t n, uint32_t value) {
  const size_t stride = (size_t)gridDim.x * BLOCK;
  const u32x4 v = {value, value, value, value};
  size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
#pragma unroll
    for (int k = 0; k < 4; ++k) __builtin_nontemporal_store(v, &dst[i + k * stride]);
  }
  for (; i < n; i += stride) dst[i] = v;
}


// Porosity from a device box-layout field (lbm_set_porosity).  k_phi_check
// records the smallest compact index of a fluid cell whose value breaks the
// rules of lbm_create ((0, 1], and 1 on open-face cells); k_phi_store copies
// the values into the compact array; k_phi_uni19 / k_phi_uni27 recompute each
// cell's uniform-neighbour-porosity flag (every fluid neighbour x + c_i has
// the cell's porosity) from the stored values.
template <class LinkT>
__global__ __launch_bounds__(BLOCK) void k_phi_check(Params p, const uint32_t* code, const LinkT* links,
                                                     const uint32_t* rowbox, const float* phib, LinkT dead,
                                                     LinkT open, unsigned* bad) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= (uint32_t)p.nc) return;
  const LinkT lk = links[c];
  if (lk & dead) return;
  const uint32_t cd = code[c];
  const float v = phib[(size_t)rowbox[cd >> p.xbits] + (cd & ((1u << p.xbits) - 1u))];
  const bool ok = v > 0.0f && v <= 1.0f && (!(lk & open) || v == 1.0f);
  if (!ok) atomicMin(bad, c);
}

template <class LinkT>
__global__ __launch_bounds__(BLOCK) void k_phi_store(Params p, const uint32_t* code, const LinkT* links,
                                                     const uint32_t* rowbox, const float* phib, LinkT dead,
                                                     float* phi) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= (uint32_t)p.nc) return;
  if (links[c] & dead) return;
  const uint32_t cd = code[c];
  phi[c] = phib[(size_t)rowbox[cd >> p.xbits] + (cd & ((1u << p.xbits) - 1u))];
}

__global__ __launch_bounds__(BLOCK) void k_phi_uni19(Params p, const uint32_t* code, uint32_t* links,
                                                     const int* delta, const float* phi) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= (uint32_t)p.nc) return;
  const uint32_t lk = links[c];
  if (lk & LK_DEAD) return;
  Pos q = position(p, c, code[c]);
  load_deltas(delta, q);
  const float ph = phi[c];
  bool uni = true;
  sfor<1, Q>([&](auto ic) {
    constexpr int J = decltype(ic)::value;  // neighbour x + c_OPP(J) = x - c_J, a wall when J's pull bounces back
    if (!((lk >> J) & 1u)) uni = uni && phi[src_of<J>(p, q)] == ph;
  });
  links[c] = uni ? (lk | LK_UNI) : (lk & ~LK_UNI);
}

// Wave records of the D3Q19 step (WaveInfo, step.hpp), one per 64 compact
// cells, from the position codes and the link words; records past the last
// cell get no flags.  Grid: wave_records(nc) / 4 blocks of 256.
__global__ __launch_bounds__(BLOCK) void k_wave_info(Params p, const uint32_t* code, const uint32_t* links,
                                                     WaveInfo* out) {
  static_assert(BLOCK % 64 == 0, "whole waves per block");
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63u;
  const bool in = c < (uint32_t)p.nc;
  const uint32_t row = in ? code[c] >> p.xbits : 0xffffffffu;
  const uint32_t prev = __shfl_up(row, 1u, 64);
  const uint64_t starts = __ballot(in && lane > 0u && row != prev);
  const uint32_t lk = in ? links[c] : LK_DEAD;
  const bool fluid = __all(!(lk & LK_DEAD) && !(lk & (LK_IN | LK_OUT | LK_UPS)));
  const bool uni = __all((lk & LK_UNI) != 0u);
  const bool inr = __all((lk & LK_INR) != 0u);
  const uint32_t row0 = __shfl(row, 0, 64);
  if (lane == 0u)
    out[c >> 6] = WaveInfo{starts, row0, (fluid ? WV_FLUID : 0u) | (uni ? WV_UNI : 0u) | (inr ? WV_INR : 0u)};
}

__global__ __launch_bounds__(BLOCK) void k_phi_uni27(Params p, const uint32_t* code, uint64_t* links,
                                                     const int* delta, const float* phi) {
  const uint32_t c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= (uint32_t)p.nc) return;
  const uint64_t lk = links[c];
  if (lk & q27::L_DEAD) return;
  Pos q = position(p, c, code[c]);
  load_deltas(delta, q);
  const float ph = phi[c];
  bool uni = true;
  sfor<1, q27::Q>([&](auto ic) {
    constexpr int J = decltype(ic)::value;
    if (!((lk >> J) & 1u)) uni = uni && phi[q27::src_of<J>(q)] == ph;
  });
  links[c] = uni ? (lk | q27::L_UNI) : (lk & ~q27::L_UNI);
}

}  // namespace lbm

namespace lbmrt {

void launch_finalize(hipStream_t s, const double* part, int nparts, int n, uint32_t ops, double* out) {
  static_assert(NDIAGP <= lbm::FIN_MAX, "partial rows fit the reduction's registers");
  hipLaunchKernelGGL(lbm::k_finalize, dim3(1), dim3(BLOCK), 0, s, part, nparts, n, ops, out);
}

void launch_set_time(hipStream_t s, uint32_t* tc, uint32_t t) {
  hipLaunchKernelGGL(lbm::k_set_time, dim3(1), dim3(64), 0, s, tc, t);
}

void launch_copy(hipStream_t s, const void* src, void* dst, size_t n16, unsigned blocks) {
  hipLaunchKernelGGL(lbm::k_copy, dim3(blocks), dim3(BLOCK), 0, s, (const uint4*)src, (uint4*)dst, n16);
}

void launch_probe(hipStream_t s, int kind, const void* src, void* dst, size_t n16, unsigned blocks) {
  if (kind == LBM_PROBE_COPY)
    hipLaunchKernelGGL(lbm::k_copy, dim3(blocks), dim3(BLOCK), 0, s, (const uint4*)src, (uint4*)dst, n16);
  else if (kind == LBM_PROBE_COPY_NT)
    hipLaunchKernelGGL(lbm::k_copy4, dim3(blocks), dim3(BLOCK), 0, s, (const lbm::u32x4*)src, (lbm::u32x4*)dst, n16);
  else if (kind == LBM_PROBE_READ)
    hipLaunchKernelGGL(lbm::k_read4, dim3(blocks), dim3(BLOCK), 0, s, (const lbm::u32x4*)src, n16, (uint32_t*)dst);
  else
    hipLaunchKernelGGL(lbm::k_write4, dim3(blocks), dim3(BLOCK), 0, s, (lbm::u32x4*)dst, n16, 0x3f800000u);
}

// lbm_set_porosity's device side: returns the smallest compact index of an
// invalid fluid cell (UINT32_MAX: none); on success the compact porosity and
// the link words' uniform flags are updated.
lbm_status set_porosity_device(lbm_ctx* c, const float* phib, uint32_t* bad_cell) {
  const dim3 grid(c->nblk), block(BLOCK);
  unsigned* bad = (unsigned*)(c->ws + c->L.diag);
  const uint32_t* code = (const uint32_t*)(c->ws + c->L.code);
  const uint32_t* rowbox = (const uint32_t*)(c->ws + c->L.rowbox);
  const int* delta = (const int*)(c->ws + c->L.delta);
  float* phi = (float*)(c->ws + c->L.phi);
  HIP_TRY(c, hipMemsetAsync(bad, 0xff, sizeof(unsigned), c->stream));
  if (c->q == 27) {
    const uint64_t* lk = (const uint64_t*)(c->ws + c->L.links);
    hipLaunchKernelGGL(lbm::k_phi_check<uint64_t>, grid, block, 0, c->stream, c->P, code, lk, rowbox, phib,
                       lbm::q27::L_DEAD, lbm::q27::L_IN | lbm::q27::L_OUT, bad);
  } else {
    const uint32_t* lk = (const uint32_t*)(c->ws + c->L.links);
    hipLaunchKernelGGL(lbm::k_phi_check<uint32_t>, grid, block, 0, c->stream, c->P, code, lk, rowbox, phib,
                       lbm::LK_DEAD, lbm::LK_IN | lbm::LK_OUT, bad);
  }
  HIP_TRY(c, hipGetLastError());
  unsigned hbad = 0;
  HIP_TRY(c, hipMemcpyAsync(&hbad, bad, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  *bad_cell = hbad;
  if (hbad != 0xffffffffu) return LBM_OK;
  if (c->q == 27) {
    uint64_t* lk = (uint64_t*)(c->ws + c->L.links);
    hipLaunchKernelGGL(lbm::k_phi_store<uint64_t>, grid, block, 0, c->stream, c->P, code, (const uint64_t*)lk,
                       rowbox, phib, lbm::q27::L_DEAD, phi);
    hipLaunchKernelGGL(lbm::k_phi_uni27, grid, block, 0, c->stream, c->P, code, lk, delta, (const float*)phi);
  } else {
    uint32_t* lk = (uint32_t*)(c->ws + c->L.links);
    hipLaunchKernelGGL(lbm::k_phi_store<uint32_t>, grid, block, 0, c->stream, c->P, code, (const uint32_t*)lk,
                       rowbox, phib, lbm::LK_DEAD, phi);
    hipLaunchKernelGGL(lbm::k_phi_uni19, grid, block, 0, c->stream, c->P, code, lk, delta, (const float*)phi);
  }
  HIP_TRY(c, hipGetLastError());
  return launch_wave_info(c);
}

lbm_status launch_wave_info(lbm_ctx* c) {
  if (c->q == 27) return LBM_OK;  // the D3Q27 step keeps no wave records
  const int64_t nrec = wave_records(c->nc);
  hipLaunchKernelGGL(lbm::k_wave_info, dim3((unsigned)(nrec / (BLOCK / 64))), dim3(BLOCK), 0, c->stream, c->P,
                     (const uint32_t*)(c->ws + c->L.code), (const uint32_t*)(c->ws + c->L.links),
                     (lbm::WaveInfo*)(c->ws + c->L.winfo));
  HIP_TRY(c, hipGetLastError());
  return LBM_OK;
}

}  // namespace lbmrt
