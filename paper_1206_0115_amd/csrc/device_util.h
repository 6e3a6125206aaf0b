// Small device helpers shared by the plan and evaluation kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fmm {

// Morton key: bit b of the x, y, z cell coordinates goes to key bits 3b,
// 3b+1, 3b+2 (Sec. 4.2 orders cells along this curve).
__host__ __device__ inline uint64_t morton3(uint32_t x, uint32_t y, uint32_t z,
                                            int bits) {
  uint64_t k = 0;
  for (int b = 0; b < bits; ++b) {
    k |= uint64_t((x >> b) & 1u) << (3 * b);
    k |= uint64_t((y >> b) & 1u) << (3 * b + 1);
    k |= uint64_t((z >> b) & 1u) << (3 * b + 2);
  }
  return k;
}

__host__ __device__ inline void demorton3(uint64_t k, int bits, int* c) {
  uint32_t x = 0, y = 0, z = 0;
  for (int b = 0; b < bits; ++b) {
    x |= uint32_t((k >> (3 * b)) & 1u) << b;
    y |= uint32_t((k >> (3 * b + 1)) & 1u) << b;
    z |= uint32_t((k >> (3 * b + 2)) & 1u) << b;
  }
  c[0] = int(x);
  c[1] = int(y);
  c[2] = int(z);
}

// Level-local cell index of a Morton key: dense table when the level is small
// enough, else binary search in the sorted keys.  -1 if absent.
struct LevelDev {
  const uint64_t* keys;
  const int* table;
  int ncell;
  int bits;  // = level
};

__device__ inline int level_find(const LevelDev& L, uint64_t key) {
  if (L.table) return L.table[key];
  int lo = 0, hi = L.ncell - 1;
  while (lo <= hi) {
    int mid = (lo + hi) >> 1;
    uint64_t v = L.keys[mid];
    if (v == key) return mid;
    if (v < key) lo = mid + 1;
    else hi = mid - 1;
  }
  return -1;
}

__device__ inline int level_find_xyz(const LevelDev& L, int x, int y, int z) {
  const int side = 1 << L.bits;
  if (x < 0 || y < 0 || z < 0 || x >= side || y >= side || z >= side) return -1;
  return level_find(L, morton3(uint32_t(x), uint32_t(y), uint32_t(z), L.bits));
}

inline int ceil_div(int64_t a, int64_t b) { return int((a + b - 1) / b); }

// Global-memory access through pointers the compiler cannot place (loaded
// from a job descriptor): without the address space it emits flat
// instructions, which count against both the vector-memory and the LDS
// wait counters, so every LDS wait also waits for the HBM loads in flight.
#define FMM_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
  return *(const FMM_GLOBAL T*)(p);
}
template <typename T>
__device__ __forceinline__ void gst(T* p, const T& v) {
  *(FMM_GLOBAL T*)(p) = v;
}

// A value known to be the same in every lane of the wavefront, as a scalar:
// branches on it are scalar branches (no lane masking) and loops on it run
// on the scalar unit.
__device__ __forceinline__ int wuni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t wuni(int64_t v) {
  const uint64_t u = uint64_t(v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(u));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(u >> 32));
  return int64_t((uint64_t(hi) << 32) | lo);
}
template <typename T>
__device__ __forceinline__ const T* wuni(const T* p) {
  return reinterpret_cast<const T*>(wuni(int64_t(reinterpret_cast<uintptr_t>(p))));
}
template <typename T>
__device__ __forceinline__ T* wuni(T* p) {
  return reinterpret_cast<T*>(wuni(int64_t(reinterpret_cast<uintptr_t>(p))));
}

}  // namespace fmm
