// Throughput probes of the device (measurement aids for the benchmark, not
// part of libbmdca).
//
// Integer vector ALU: every lane runs 8 independent chains of three-input bit
// operations (v_bitop3_b32), or of the pair-count kernel's mix (five bit
// operations and one popcount-accumulate per word), long enough that issue
// rate, not latency, bounds it.  Returns 32-bit lane operations per second
// over the timed launch.
//
// Random LDS lookups: the energy kernel's access pattern without its tile
// staging, token loads or step bookkeeping.  512-thread workgroups hold a
// 21 x P float table; per step every thread adds, for 4 (row, 16-column)
// sets, the 16 entries table[r P + 21 jj + c_jj] into FP32 sums, r and the
// c_jj uniform in 0..20 from a hash of the thread (r moves by one each
// step), so a wave's 64 addresses fall on the banks as uniform random
// sequences' tokens do; a step's 64 reads are all issued before its adds.
// Returns 4-byte lookups per second.
//
// Row gathers: the gather sampler's pattern at q = 21 without staging, draws
// or barriers.  One workgroup per CU (its LDS allocation leaves no room for a
// second) of a given number of waves, a chunk of 16 sites x 21 rows of 24
// floats; chains of 6 lanes (narrow: 10 per wave) or 8 lanes (8 per wave, 2
// idle), lane v < 6 of a chain reading quad v of the row (position, token)
// with one 16-byte read per position and adding it to its sums, tokens
// uniform in 0..20 from a hash of (chain, position) and fixed over the
// iterations (no address arithmetic in the loop).  Returns row reads (one row
// per chain and position) per second.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

template <int MIX>
__global__ __launch_bounds__(256) void k_int_valu(uint32_t* out, int iters, uint32_t seed) {
  uint32_t a[8], b[8], c[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    a[k] = seed * (threadIdx.x + 17u * k + 1u);
    b[k] = a[k] ^ (0x9E3779B9u + k);
    c[k] = a[k] + blockIdx.x;
  }
  uint32_t acc = 0;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (MIX == 0) {
        // 6 dependent bit operations per chain
        c[k] = __builtin_amdgcn_bitop3_b32(a[k], b[k], c[k], 0xBE);
        a[k] = __builtin_amdgcn_bitop3_b32(b[k], c[k], a[k], 0x96);
        b[k] = __builtin_amdgcn_bitop3_b32(c[k], a[k], b[k], 0xBE);
        c[k] = __builtin_amdgcn_bitop3_b32(a[k], b[k], c[k], 0x96);
        a[k] = __builtin_amdgcn_bitop3_b32(b[k], c[k], a[k], 0xBE);
        b[k] = __builtin_amdgcn_bitop3_b32(c[k], a[k], b[k], 0x96);
      } else {
        // 5 bit operations and 1 popcount-accumulate, as one word of a pair
        uint32_t d = a[k] ^ b[k];
        d = __builtin_amdgcn_bitop3_b32(c[k], a[k], d, 0xBE);
        d = __builtin_amdgcn_bitop3_b32(b[k], c[k], d, 0xBE);
        d = __builtin_amdgcn_bitop3_b32(a[k], c[k], d, 0xBE);
        d = __builtin_amdgcn_bitop3_b32(b[k], a[k], d, 0xBE);
        acc += __popc(d);
        a[k] = d;
      }
    }
  }
  uint32_t r = acc;
#pragma unroll
  for (int k = 0; k < 8; ++k) r ^= a[k] ^ b[k] ^ c[k];
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

constexpr int kLQ = 21;  // states of the probed lookups

__device__ inline uint32_t probe_hash(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return x;
}

__global__ __launch_bounds__(512) void k_lds_lookups(float* out, int iters, int P) {
  extern __shared__ float table[];  // kLQ x P
  for (int e = threadIdx.x; e < kLQ * P; e += blockDim.x) table[e] = (float)(e & 255) * 0.5f;
  __syncthreads();
  const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
  int r[4];
  int c[4][16];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r[k] = (int)(probe_hash(id * 4u + k) % kLQ);
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) c[k][jj] = (int)(probe_hash(id * 64u + k * 16u + jj + 0x51u) % kLQ);
  }
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int it = 0; it < iters; ++it) {
    // all 64 lookups of the step are read before any is added, so the LDS
    // pipe, not the add chains, sets the pace
    float v[4][16];
#pragma unroll
    for (int jj = 0; jj < 16; ++jj)
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k][jj] = table[r[k] * P + jj * kLQ + c[k][jj]];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float sf = 0.0f;
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) sf += v[k][jj];
      acc[k] += sf;
      r[k] = (r[k] + 1 == kLQ) ? 0 : r[k] + 1;
    }
  }
  out[id] = acc[0] + acc[1] + acc[2] + acc[3];
}

constexpr int kRQ = 21, kRQuads = 6, kRPos = 16;  // states, quads per row, positions

template <int LPC>
__global__ __launch_bounds__(1024) void k_lds_rows(float* out, int iters) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  extern __shared__ f4 chunk[];  // kRPos x kRQ rows of kRQuads quads (more is allocated)
  for (int e = threadIdx.x; e < kRPos * kRQ * kRQuads; e += blockDim.x)
    chunk[e] = f4{(float)(e & 63), 1.0f, 2.0f, 3.0f} * 0.001f;
  __syncthreads();
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int chain = lane / LPC, v = lane - chain * LPC;
  const bool act = chain < 64 / LPC && v < kRQuads;  // narrow: lanes 60..63 idle
  const uint32_t cg = (blockIdx.x * (blockDim.x / 64) + wave) * (64 / LPC) + chain;
  int idx[kRPos];
#pragma unroll
  for (int pos = 0; pos < kRPos; ++pos) {
    const int t = (int)(probe_hash(cg * kRPos + pos + 0x9Du) % kRQ);
    idx[pos] = act ? (pos * kRQ + t) * kRQuads + v : 0;
  }
  f4 acc = f4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int it = 0; it < iters; ++it) {
    asm volatile("" ::: "memory");  // the reads are repeated, not hoisted out of the loop
#pragma unroll
    for (int pos = 0; pos < kRPos; ++pos) acc += chunk[idx[pos]];
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = act ? acc[0] + acc[1] + acc[2] + acc[3] : 0.0f;
}

}  // namespace

// Row reads per second of the row-gather probe with chains of lpc lanes (6
// or 8) and workgroups of `waves` waves (1..16).  Negative on error.
extern "C" double bmdca_probe_lds_rows(int lpc, int waves, int iters, int blocks) {
  if ((lpc != 6 && lpc != 8) || waves < 1 || waves > 16) return -3.0;
  float* out = nullptr;
  if (hipMalloc(&out, sizeof(float) * 64 * waves * (size_t)blocks) != hipSuccess) return -1.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  const size_t lds = 96 * 1024;  // one workgroup per CU, as the sampler runs
  const void* kern = lpc == 6 ? reinterpret_cast<const void*>(k_lds_rows<6>)
                              : reinterpret_cast<const void*>(k_lds_rows<8>);
  ok = ok && hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) ==
                 hipSuccess;
  auto launch = [&](int n) {
    if (lpc == 6)
      hipLaunchKernelGGL(k_lds_rows<6>, dim3(blocks), dim3(64 * waves), lds, 0, out, n);
    else
      hipLaunchKernelGGL(k_lds_rows<8>, dim3(blocks), dim3(64 * waves), lds, 0, out, n);
    return hipGetLastError() == hipSuccess;
  };
  float ms = 0.0f;
  ok = ok && launch(iters / 8);  // warm
  ok = ok && hipEventRecord(e0, 0) == hipSuccess && launch(iters) &&
       hipEventRecord(e1, 0) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
       hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
  if (e0) ok = (hipEventDestroy(e0) == hipSuccess) && ok;
  if (e1) ok = (hipEventDestroy(e1) == hipSuccess) && ok;
  ok = (hipFree(out) == hipSuccess) && ok;
  if (!ok || ms <= 0.0f) return -2.0;
  return (double)kRPos * (64 / lpc) * waves * (double)iters * (double)blocks / (ms * 1e-3);
}

// Lookups per second of the random-lookup probe with a table row pitch of P
// floats (P >= 336).  Negative on error.
extern "C" double bmdca_probe_lds_lookups(int P, int iters, int blocks) {
  if (P < 16 * kLQ || (size_t)kLQ * P * sizeof(float) > 64 * 1024) return -3.0;
  float* out = nullptr;
  if (hipMalloc(&out, sizeof(float) * 512 * (size_t)blocks) != hipSuccess) return -1.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  const size_t lds = sizeof(float) * kLQ * (size_t)P;
  auto launch = [&](int n) {
    hipLaunchKernelGGL(k_lds_lookups, dim3(blocks), dim3(512), lds, 0, out, n, P);
    return hipGetLastError() == hipSuccess;
  };
  float ms = 0.0f;
  ok = ok && launch(iters / 8);  // warm
  ok = ok && hipEventRecord(e0, 0) == hipSuccess && launch(iters) &&
       hipEventRecord(e1, 0) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
       hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
  if (e0) ok = (hipEventDestroy(e0) == hipSuccess) && ok;
  if (e1) ok = (hipEventDestroy(e1) == hipSuccess) && ok;
  ok = (hipFree(out) == hipSuccess) && ok;
  if (!ok || ms <= 0.0f) return -2.0;
  return 64.0 * (double)iters * 512.0 * (double)blocks / (ms * 1e-3);
}

// mix 0: bit operations only; 1: the pair-count mix.  Negative on error.
extern "C" double bmdca_probe_int_valu(int mix, int iters, int blocks) {
  uint32_t* out = nullptr;
  if (hipMalloc(&out, sizeof(uint32_t) * 256 * (size_t)blocks) != hipSuccess) return -1.0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  auto launch = [&](int n) {
    if (mix == 0)
      hipLaunchKernelGGL(k_int_valu<0>, dim3(blocks), dim3(256), 0, 0, out, n, 12345u);
    else
      hipLaunchKernelGGL(k_int_valu<1>, dim3(blocks), dim3(256), 0, 0, out, n, 12345u);
    return hipGetLastError() == hipSuccess;
  };
  float ms = 0.0f;
  ok = ok && launch(iters / 8);  // warm
  ok = ok && hipEventRecord(e0, 0) == hipSuccess && launch(iters) &&
       hipEventRecord(e1, 0) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
       hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
  if (e0) ok = (hipEventDestroy(e0) == hipSuccess) && ok;
  if (e1) ok = (hipEventDestroy(e1) == hipSuccess) && ok;
  ok = (hipFree(out) == hipSuccess) && ok;
  if (!ok || ms <= 0.0f) return -2.0;
  const double ops = 6.0 * 8.0 * (double)iters * 256.0 * (double)blocks;
  return ops / (ms * 1e-3);
}
