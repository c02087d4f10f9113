// Equilibrium sampling of a trained model (adabmDCA 2.0, Sec. 4.1, and the
// convergence criterion of its sampling routine): weighted draw of data rows
// to start chains from, gathering those rows, and the SeqID overlaps
//   SeqID(a, b) = (1/L) sum_i [a_i == b_i]
// averaged over pairs of chains (chains vs a permutation of themselves, or
// vs their own earlier state).
#include "common.hpp"
#include "internal.hpp"

namespace bmdca {

// Prefix sums C_m = w_0 + ... + w_m in ascending m (the definition's order):
// the block stages 256 weights at a time in LDS and one thread adds them.
__global__ __launch_bounds__(256) void k_prefix_weights(const double* __restrict__ w, int64_t M,
                                                        double* __restrict__ C) {
  __shared__ double buf[256];
  double run = 0.0;
  for (int64_t m0 = 0; m0 < M; m0 += 256) {
    const int64_t m = m0 + threadIdx.x;
    buf[threadIdx.x] = (m < M) ? w[m] : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
      const int n = (int)min<int64_t>(256, M - m0);
      for (int k = 0; k < n; ++k) {
        run += buf[k];
        buf[k] = run;
      }
    }
    __syncthreads();
    if (m < M) C[m] = buf[threadIdx.x];
    __syncthreads();
  }
}

// Draw k: u from Philox counter (k/4, 0, 0, 2), word k%4, u = (word >> 8)
// 2^-24; the row is the first m with C_m > u W (binary search over the
// non-decreasing prefix sums).  A total that is not positive and finite
// raises BMDCA_DEVERR_NONFINITE and yields row 0.
__global__ void k_draw_rows(const double* __restrict__ C, int64_t M, int64_t n, uint32_t k0,
                            uint32_t k1, int32_t* __restrict__ rows, int32_t* dev_err) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double W = C[M - 1];
  if (!(W > 0.0) || !isfinite(W)) {
    rows[k] = 0;
    if (dev_err && k == 0) atomicOr(dev_err, 2);
    return;
  }
  const uint4 r = philox4x32_10(make_uint4((uint32_t)(k >> 2), 0u, 0u, 2u), k0, k1);
  const double t = (double)word_to_uniform(pick_word(r, (int)(k & 3))) * W;
  int64_t lo = 0, hi = M - 1;  // C[hi] = W > t
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (C[mid] > t)
      hi = mid;
    else
      lo = mid + 1;
  }
  rows[k] = (int32_t)lo;
}

// out[k][.] = X[rows[k]][.]; an index outside 0..M-1 raises
// BMDCA_DEVERR_INDEX and copies row 0.
__global__ void k_gather_rows(const int8_t* __restrict__ X, int64_t M, int L,
                              const int32_t* __restrict__ rows, int64_t n,
                              int8_t* __restrict__ out, int32_t* dev_err) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * L) return;
  const int64_t k = e / L;
  const int i = (int)(e % L);
  int64_t r = rows[k];
  if (r < 0 || r >= M) {
    if (dev_err && i == 0) atomicOr(dev_err, 4);
    r = 0;
  }
  out[e] = X[r * L + i];
}

__global__ void k_seqid_zero(unsigned long long* __restrict__ acc) {
  if (threadIdx.x < 2) acc[threadIdx.x] = 0ull;
}

// Each wave takes pairs (A[k], B[perm[k]]) k = wave, wave + waves, ...:
// identity count n_k over the L positions; the exact integer sums of n_k and
// n_k^2 are reduced per workgroup and added to acc[0], acc[1] once per
// workgroup (a grid of at most kSeqBlocks workgroups, so the two shared
// counters see few atomics).
constexpr int kSeqWaves = 4;
constexpr int kSeqBlocks = 512;

__global__ __launch_bounds__(kSeqWaves * 64) void k_seqid_count(
    const int8_t* __restrict__ A, const int8_t* __restrict__ B, const int32_t* __restrict__ perm,
    int64_t N, int L, unsigned long long* __restrict__ acc, int32_t* dev_err) {
  __shared__ unsigned long long part[2][kSeqWaves];
  const int lane = threadIdx.x % 64;
  const int wid = threadIdx.x / 64;
  const int64_t waves = (int64_t)gridDim.x * kSeqWaves;
  unsigned long long s1 = 0, s2 = 0;
  for (int64_t k = (int64_t)blockIdx.x * kSeqWaves + wid; k < N; k += waves) {
    int64_t kb = k;
    if (perm) {
      kb = perm[k];
      if (kb < 0 || kb >= N) {
        if (dev_err && lane == 0) atomicOr(dev_err, 4);
        continue;
      }
    }
    const int8_t* a = A + k * L;
    const int8_t* b = B + kb * L;
    int same = 0;
    for (int i = lane; i < L; i += 64) same += (a[i] == b[i]) ? 1 : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) same += __shfl_xor(same, o, 64);
    s1 += (unsigned long long)same;
    s2 += (unsigned long long)same * (unsigned long long)same;
  }
  if (lane == 0) {
    part[0][wid] = s1;
    part[1][wid] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t1 = 0, t2 = 0;
#pragma unroll
    for (int w = 0; w < kSeqWaves; ++w) {
      t1 += part[0][w];
      t2 += part[1][w];
    }
    if (t1 | t2) {
      atomicAdd(acc, t1);
      atomicAdd(acc + 1, t2);
    }
  }
}

// mean = S1 / (N L), var = S2 / (N L^2) - mean^2 (0 if negative).
__global__ void k_seqid_finish(const unsigned long long* __restrict__ acc, int64_t N, int L,
                               double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  const double mean = (double)acc[0] / ((double)N * (double)L);
  const double m2 = (double)acc[1] / ((double)N * (double)L * (double)L);
  const double var = m2 - mean * mean;
  out[0] = mean;
  out[1] = sqrt(var > 0.0 ? var : 0.0);
}

size_t draw_ws_bytes(int64_t M) { return align256(sizeof(double) * (size_t)M); }
size_t seqid_ws_bytes() { return 256; }

hipError_t launch_draw_rows(const double* w, int64_t M, int64_t n, uint64_t seed, int32_t* rows,
                            void* ws, int32_t* dev_err, hipStream_t s) {
  double* C = static_cast<double*>(ws);
  hipLaunchKernelGGL(k_prefix_weights, dim3(1), dim3(256), 0, s, w, M, C);
  if (n > 0)
    hipLaunchKernelGGL(k_draw_rows, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, C, M, n,
                       (uint32_t)seed, (uint32_t)(seed >> 32), rows, dev_err);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const int8_t* X, int64_t M, int L, const int32_t* rows, int64_t n,
                              int8_t* out, int32_t* dev_err, hipStream_t s) {
  const int64_t total = n * L;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, X, M, L,
                     rows, n, out, dev_err);
  return hipGetLastError();
}

hipError_t launch_seqid(const int8_t* A, const int8_t* B, const int32_t* perm, int64_t N, int L,
                        double* out, void* ws, int32_t* dev_err, hipStream_t s) {
  unsigned long long* acc = static_cast<unsigned long long*>(ws);
  hipLaunchKernelGGL(k_seqid_zero, dim3(1), dim3(64), 0, s, acc);
  hipLaunchKernelGGL(k_seqid_count, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(N, kSeqWaves), kSeqBlocks))),
                     dim3(kSeqWaves * 64), 0,
                     s, A, B, perm, N, L, acc, dev_err);
  hipLaunchKernelGGL(k_seqid_finish, dim3(1), dim3(64), 0, s, acc, N, L, out);
  return hipGetLastError();
}

}  // namespace bmdca
