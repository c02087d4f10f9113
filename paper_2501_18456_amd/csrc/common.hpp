// Device helpers and host plumbing shared by the libbmdca HIP sources.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>

namespace bmdca {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11):
// ten rounds of  (c0,c1,c2,c3) -> (hi(B*c2)^c1^k0, lo(B*c2), hi(A*c0)^c3^k1,
// lo(A*c0)) with A = 0xD2511F53, B = 0xCD9E8D57, and the key advanced by the
// Weyl constants (0x9E3779B9, 0xBB67AE85) between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo_a = 0xD2511F53u * c.x;
    const uint32_t hi_a = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo_b = 0xCD9E8D57u * c.z;
    const uint32_t hi_b = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi_b ^ c.y ^ k0, lo_b, hi_a ^ c.w ^ k1, lo_a);
  }
  return c;
}

__device__ __forceinline__ uint32_t pick_word(uint4 v, int k) {
  return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w;
}

// 24-bit uniform in [0, 1): exactly representable in FP32.
__device__ __forceinline__ float word_to_uniform(uint32_t w) {
  return (float)(w >> 8) * (1.0f / 16777216.0f);
}

// ---------------------------------------------------------------------------
// Wave-level helpers (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
  return v;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Block-wide FP64 sum in a fixed tree order (blockDim.x a multiple of 64,
// at most 1024).  All threads must call it; the result is valid in thread 0.
__device__ __forceinline__ double block_sum_f64(double v, double* sh /* >= 16 */) {
  v = wave_sum_f64(v);
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x / kWave;
    for (int k = 0; k < nw; ++k) r += sh[k];
  }
  __syncthreads();
  return r;
}

// Memory-safe token read: out-of-range tokens raise the device error flag
// and are replaced by 0 so that no index leaves its array.
__device__ __forceinline__ int checked_token(int8_t t, int q, int32_t* dev_err) {
  int v = (int)t;
  if (v < 0 || v >= q) {
    if (dev_err) atomicOr(dev_err, 1);
    v = 0;
  }
  return v;
}

__host__ __device__ constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

__host__ __device__ constexpr int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace bmdca
