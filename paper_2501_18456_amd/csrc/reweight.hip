// Importance weights of Eq. (7) (adabmDCA 2.0, Sec. 2.3, step p.2):
// N^(m) = #{n : identical positions of rows m and n >= T}, w = 1 / N^(m).
//
// Bit-sliced integer kernel: the token at every position is split into
// P = ceil(log2 q) bit planes of ceil(L/32) 32-bit words per row.  Two rows
// differ at a position iff some plane differs there, so
//   mismatches = sum_w popcount(OR_p (plane_p[m][w] XOR plane_p[n][w]))
// and identical positions = L - mismatches (padding bits are 0 in both rows).
// A thread owns one row m and keeps its planes in registers; a workgroup
// stages 256 rows n at a time in LDS and every lane reads the same n
// (broadcast).  Counts are exact integers.
#include "common.hpp"
#include "internal.hpp"

namespace bmdca {

constexpr int kRwThreads = 256;
constexpr int kMaxPlanes = 5;  // q <= 32

static int planes_for(int q) {
  int p = 0;
  while ((1 << p) < q) ++p;
  return std::max(p, 1);
}

ReweightPlan plan_reweight(int64_t M, int L, int q) {
  ReweightPlan r{};
  r.planes = planes_for(q);
  r.words = (int)ceil_div(L, 32);
  r.Mpad = ceil_div(M, kRwThreads) * kRwThreads;
  size_t o = 0;
  r.off_planes = o;
  o = align256(o + sizeof(uint32_t) * (size_t)r.Mpad * kMaxPlanes * r.words);
  r.off_red = o;
  o = align256(o + sizeof(double) * 64);
  r.total = o;
  return r;
}

// planes[m][p][w]: bit t of word w = bit p of the token at position 32w + t.
__global__ void k_encode_planes(const int8_t* __restrict__ msa, int64_t M, int L, int q, int P,
                                int W, uint32_t* __restrict__ planes, int32_t* dev_err) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t m = idx / W;
  const int w = (int)(idx % W);
  if (m >= M) return;
  uint32_t bits[kMaxPlanes] = {0, 0, 0, 0, 0};
  for (int t = 0; t < 32; ++t) {
    const int i = 32 * w + t;
    if (i >= L) break;
    const int tok = checked_token(msa[m * L + i], q, dev_err);
#pragma unroll
    for (int p = 0; p < kMaxPlanes; ++p) bits[p] |= (uint32_t)((tok >> p) & 1) << t;
  }
  for (int p = 0; p < P; ++p) planes[((size_t)m * kMaxPlanes + p) * W + w] = bits[p];
}

template <int W>
__global__ __launch_bounds__(kRwThreads) void k_count_similar(const uint32_t* __restrict__ planes,
                                                              int64_t M, int P, int L, int T,
                                                              int32_t* __restrict__ n_sim) {
  __shared__ uint32_t sh[kRwThreads * kMaxPlanes * W];
  const int64_t m = (int64_t)blockIdx.x * kRwThreads + threadIdx.x;
  uint32_t mine[kMaxPlanes][W];
#pragma unroll
  for (int p = 0; p < kMaxPlanes; ++p)
#pragma unroll
    for (int w = 0; w < W; ++w)
      mine[p][w] = (m < M && p < P) ? planes[((size_t)m * kMaxPlanes + p) * W + w] : 0u;
  int count = 0;
  for (int64_t n0 = 0; n0 < M; n0 += kRwThreads) {
    __syncthreads();
    const int64_t nload = std::min<int64_t>(kRwThreads, M - n0);
    for (int k = threadIdx.x; k < kRwThreads * kMaxPlanes * W; k += kRwThreads) {
      const int nl = k / (kMaxPlanes * W);
      sh[k] = (nl < nload) ? planes[(size_t)(n0 + nl) * kMaxPlanes * W + (k % (kMaxPlanes * W))]
                           : 0u;
    }
    __syncthreads();
    for (int nl = 0; nl < nload; ++nl) {
      const uint32_t* o = sh + nl * kMaxPlanes * W;
      int mism = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        uint32_t d = 0;
#pragma unroll
        for (int p = 0; p < kMaxPlanes; ++p)
          if (p < P) d |= mine[p][w] ^ o[p * W + w];
        mism += __popc(d);
      }
      count += (L - mism >= T) ? 1 : 0;
    }
  }
  if (m < M) n_sim[m] = count;
}

__global__ __launch_bounds__(1024) void k_weights_meff(const int32_t* __restrict__ n_sim,
                                                       int64_t M, double* __restrict__ w,
                                                       double* __restrict__ meff) {
  __shared__ double sh[16];
  double v = 0.0;
  for (int64_t m = threadIdx.x; m < M; m += blockDim.x) {
    const double x = 1.0 / (double)n_sim[m];
    w[m] = x;
    v += x;
  }
  const double t = block_sum_f64(v, sh);
  if (threadIdx.x == 0) *meff = t;
}

template <int W>
static void launch_count_w(const uint32_t* planes, int64_t M, int P, int L, int T, int32_t* n_sim,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_count_similar<W>, dim3((unsigned)ceil_div(M, kRwThreads)),
                     dim3(kRwThreads), 0, s, planes, M, P, L, T, n_sim);
}

hipError_t launch_reweight(const int8_t* msa, int64_t M, int L, int q, int32_t T,
                           const ReweightPlan& plan, void* ws, int32_t* n_sim, double* w,
                           double* meff, int32_t* dev_err, hipStream_t s) {
  uint32_t* planes = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + plan.off_planes);
  const int W = plan.words, P = plan.planes;
  // Unused planes (p >= P) are never read; padding bits are written as 0.
  hipLaunchKernelGGL(k_encode_planes, dim3((unsigned)ceil_div(M * W, 256)), dim3(256), 0, s, msa,
                     M, L, q, P, W, planes, dev_err);
  switch (W) {
#define BMDCA_RW_CASE(n) \
  case n:                \
    launch_count_w<n>(planes, M, P, L, T, n_sim, s); \
    break;
    BMDCA_RW_CASE(1) BMDCA_RW_CASE(2) BMDCA_RW_CASE(3) BMDCA_RW_CASE(4) BMDCA_RW_CASE(5)
    BMDCA_RW_CASE(6) BMDCA_RW_CASE(7) BMDCA_RW_CASE(8) BMDCA_RW_CASE(9) BMDCA_RW_CASE(10)
    BMDCA_RW_CASE(11) BMDCA_RW_CASE(12) BMDCA_RW_CASE(13) BMDCA_RW_CASE(14) BMDCA_RW_CASE(15)
    BMDCA_RW_CASE(16)
#undef BMDCA_RW_CASE
    default:
      return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k_weights_meff, dim3(1), dim3(1024), 0, s, n_sim, M, w, meff);
  return hipGetLastError();
}

}  // namespace bmdca
