// Throughput probe of the 32-bit integer vector ALU on the device (a
// measurement aid for the benchmark, not part of libbmdca): every lane runs
// 8 independent chains of three-input bit operations (v_bitop3_b32), or of
// the pair-count kernel's mix (five bit operations and one popcount-
// accumulate per word), long enough that issue rate, not latency, bounds
// it.  Returns 32-bit lane operations per second over the timed launch.
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

}  // namespace

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
