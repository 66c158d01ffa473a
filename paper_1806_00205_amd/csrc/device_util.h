// Device helpers shared by the traversal and shading kernels (gfx950):
// address-space casts, wave-level primitives, the Philox4x32-10 counter-based
// generator (Salmon et al., SC'11) and the job look-up of a concatenated
// primary index.
#pragma once

#include "rtmc_internal.h"

namespace rtmc {
namespace {

// Explicit address spaces: pointers that arrive through the job table or the
// argument struct are otherwise generic, and generic (flat) accesses wait on
// both the vector-memory and the LDS counters.
#define GAS __attribute__((address_space(1)))
#define LAS __attribute__((address_space(3)))
typedef float f4v __attribute__((ext_vector_type(4)));

template <typename T>
__device__ inline GAS T* gp(T* p) {
  return (GAS T*)p;
}
template <typename T>
__device__ inline const GAS T* gp(const T* p) {
  return (const GAS T*)p;
}

constexpr float kPi = 3.14159265358979323846f;
constexpr float kDeg = 57.295779513082320876f;  // 180 / pi

__device__ inline uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------- Philox

struct U4 {
  uint32_t x, y, z, w;
};

__device__ inline U4 philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

// (0, 1]: ((u >> 8) + 1) * 2^-24, exact in FP32
__device__ inline float u01(uint32_t u) { return (float)((u >> 8) + 1u) * 5.9604644775390625e-8f; }

// Job of concatenated primary index g among jobs [lo, hi] (sorted by gbase).
__device__ inline int find_job(const DevJob* jobs, int lo, int hi, uint64_t g) {
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (gp(jobs)[mid].gbase <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ inline unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline uint32_t wave_incl_scan(uint32_t v, uint32_t lane) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_up(v, off, 64);
    if (lane >= (uint32_t)off) v += o;
  }
  return v;
}

}  // namespace
}  // namespace rtmc
