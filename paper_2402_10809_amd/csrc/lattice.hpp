// D3Q19 velocity set, storage formats and launch helpers shared by the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 19;
constexpr int BLOCK = 256;   // 4 wave64 per workgroup
constexpr int NDIAGP = 11;   // per-block diagnostic partials

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

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Remap so that each XCD works on one contiguous eighth of the compact cells:
// the cache lines that two neighbouring waves share (x-shifted slots, rows
// y +- 1 and z +- 1) then meet in one L2 instead of being fetched twice.  The
// map is a permutation of [0, nb).
__device__ __forceinline__ uint32_t xcd_block(uint32_t bid, uint32_t nb) {
  const uint32_t q = nb >> 3, r = nb & 7u, k = bid & 7u;
  return k * q + (k < r ? k : r) + (bid >> 3);
}

// Neighbour-row pairs (cy, cz): the pull source x - c_i lies in the row
// (y - cy, z - cz); PK[i] is the index of that pair, 0 for the cell's own row.
constexpr int NPAIR = 9;
constexpr int PCY[NPAIR] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
constexpr int PCZ[NPAIR] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
__host__ __device__ constexpr int pair_of(int cy, int cz) {
  int k = 0;
  while (k < NPAIR && !(PCY[k] == cy && PCZ[k] == cz)) ++k;
  return k;
}
constexpr int PK[Q] = {pair_of(CY[0], CZ[0]),   pair_of(CY[1], CZ[1]),   pair_of(CY[2], CZ[2]),
                       pair_of(CY[3], CZ[3]),   pair_of(CY[4], CZ[4]),   pair_of(CY[5], CZ[5]),
                       pair_of(CY[6], CZ[6]),   pair_of(CY[7], CZ[7]),   pair_of(CY[8], CZ[8]),
                       pair_of(CY[9], CZ[9]),   pair_of(CY[10], CZ[10]), pair_of(CY[11], CZ[11]),
                       pair_of(CY[12], CZ[12]), pair_of(CY[13], CZ[13]), pair_of(CY[14], CZ[14]),
                       pair_of(CY[15], CZ[15]), pair_of(CY[16], CZ[16]), pair_of(CY[17], CZ[17]),
                       pair_of(CY[18], CZ[18])};

}  // namespace lbm
