// D3Q19 velocity set, storage formats and launch helpers shared by the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 19;
constexpr int BLOCK = 256;   // 4 wave64 per workgroup
constexpr int NDIAGP = 10;   // per-block diagnostic partials

// Direction order: rest; +x -x +y -y +z -z; xy edges; xz edges; yz edges,
// each odd-numbered direction followed by its opposite.
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

__host__ __device__ constexpr float wgt(int i) { return i == 0 ? 1.0f / 3.0f : (i < 7 ? 1.0f / 18.0f : 1.0f / 36.0f); }
// Element access through a 32-bit byte offset from a uniform base (the whole
// population buffer is kept below 4 GiB), so loads and stores address as
// scalar base + vector offset.
template <class T>
__device__ __forceinline__ T ldo(const T* base, uint32_t e) {
  return *(const T*)((const char*)base + (uint32_t)(e * (uint32_t)sizeof(T)));
}
template <class T>
__device__ __forceinline__ void sto(T* base, uint32_t e, T v) {
  *(T*)((char*)base + (uint32_t)(e * (uint32_t)sizeof(T))) = v;
}

template <class S> struct Store;
template <> struct Store<float> {
  static __device__ __forceinline__ float ld(const float* b, uint32_t e, int) { return ldo(b, e); }
  static __device__ __forceinline__ void st(float* b, uint32_t e, float v, int) { sto(b, e, v); }
};
template <> struct Store<_Float16> {
  static __device__ __forceinline__ float ld(const _Float16* b, uint32_t e, int) { return (float)ldo(b, e); }
  static __device__ __forceinline__ void st(_Float16* b, uint32_t e, float v, int) { sto(b, e, (_Float16)v); }
};
template <> struct Store<__bf16> {
  static __device__ __forceinline__ float ld(const __bf16* b, uint32_t e, int) { return (float)ldo(b, e); }
  static __device__ __forceinline__ void st(__bf16* b, uint32_t e, float v, int) { sto(b, e, (__bf16)v); }
};

// Consecutive workgroups are dispatched round-robin over the 8 XCDs; remap so
// that each XCD works on one contiguous slice of the fluid list (neighbouring
// cells then share that XCD's L2).
__device__ __forceinline__ uint32_t xcd_block(uint32_t bid, uint32_t nb) {
  const uint32_t q = nb >> 3, r = nb & 7u, k = bid & 7u;
  return k * q + (k < r ? k : r) + (bid >> 3);
}

}  // namespace lbm
