// Importance weights of Eq. (7) (adabmDCA 2.0, Sec. 2.3, step p.2):
// N^(m) = #{n : identical positions of rows m and n >= T}, w = 1 / N^(m).
//
// Bit-sliced integer kernel: the token at every position is split into
// P = ceil(log2 q) bit planes of ceil(L/32) 32-bit words per row.  Two rows
// differ at a position iff some plane differs there, so
//   mismatches = sum_w popcount(OR_p (plane_p[m][w] XOR plane_p[n][w]))
// and identical positions = L - mismatches (padding bits are 0 in both rows).
// A thread owns one or two rows m and keeps their planes in registers; a
// workgroup stages 256 rows n at a time in LDS and every lane reads the same
// n (broadcast).  Each unordered pair is compared once (M(M-1)/2 pairs) and
// counted for both rows.  Counts are exact integers.
#include "common.hpp"
#include "internal.hpp"

namespace bmdca {

constexpr int kRwThreads = 256;
constexpr int kMaxPlanes = 5;  // q <= 32
// 256-column stages per work item of the pair count (balance over the CUs)
constexpr int kRwChunk = 16;
// Truth table of (a ^ b) | c for v_bitop3_b32(a, b, c): bit (4a + 2b + c).
#ifndef BMDCA_XOR_OR_TABLE
#define BMDCA_XOR_OR_TABLE 0xBE
#endif
constexpr unsigned kXorOr = BMDCA_XOR_OR_TABLE;

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

// Pair counts over unordered pairs.  A work item is (row block, column
// chunk): 256*R rows (R per thread, planes in registers) against a chunk of
// later columns staged 256 at a time in LDS (every lane reads the same
// column: broadcast).  Each row block starts with its own rows: those R
// stages count every ordered pair inside the block (self included) for the
// rows only.  Every later column n is compared once with the block's rows m
// and the pair counts for both: for m in the thread's counter, for n by a
// wave ballot and popcount per column, summed over the waves in LDS and added
// to N^(n) with one integer atomic per column and stage.  Integer atomics are
// exact in any order, so the counts are bit-exact.
template <int P, int W, int R>
__global__ __launch_bounds__(kRwThreads) void k_count_similar(const uint32_t* __restrict__ planes,
                                                              int64_t M, int L, int T,
                                                              int32_t* __restrict__ n_sim) {
  constexpr int kRows = kRwThreads * R;  // rows per block
  __shared__ uint32_t sh[kRwThreads * P * W];
  __shared__ int colpart[kRwThreads / 64][kRwThreads];
  // work item -> (row block rb, its stages s0 .. s1-1): row blocks in turn,
  // each cut into chunks of kRwChunk stages (the launch counts them alike)
  const int64_t stages = ceil_div(M, kRwThreads);
  int64_t t = blockIdx.x, rb = 0;
  for (;;) {
    const int64_t nch = ceil_div(stages - rb * R, kRwChunk);
    if (t < nch) break;
    t -= nch;
    ++rb;
  }
  const int s0 = (int)(t * kRwChunk);
  const int s1 = (int)std::min<int64_t>(stages - rb * R, (int64_t)s0 + kRwChunk);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t m0 = rb * kRows + threadIdx.x;
  uint32_t mine[R][P][W];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t m = m0 + (int64_t)kRwThreads * r;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int w = 0; w < W; ++w)
        mine[r][p][w] = (m < M) ? planes[((size_t)m * kMaxPlanes + p) * W + w] : 0u;
  }
  const int maxmis = L - T;  // similar iff mismatches <= L - T
  int count[R];
#pragma unroll
  for (int r = 0; r < R; ++r) count[r] = 0;
  for (int st = s0; st < s1; ++st) {
    const int64_t n0 = rb * kRows + (int64_t)st * kRwThreads;
    const bool own = st < R;  // the block's own rows: ordered pairs, rows only
    __syncthreads();
    const int nload = (int)std::min<int64_t>(kRwThreads, M - n0);
    for (int k = threadIdx.x; k < nload * P * W; k += kRwThreads) {
      const int nl = k / (P * W), pw = k % (P * W);
      sh[k] = planes[(size_t)(n0 + nl) * kMaxPlanes * W + pw];
    }
    __syncthreads();
    for (int nl = 0; nl < nload; ++nl) {
      const uint32_t* o = sh + nl * P * W;
      int mism[R];
#pragma unroll
      for (int r = 0; r < R; ++r) mism[r] = 0;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        uint32_t ow[P];
#pragma unroll
        for (int p = 0; p < P; ++p) ow[p] = o[p * W + w];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          // d = OR_p (mine_p ^ other_p), one three-input bit operation per plane
          uint32_t d = mine[r][0][w] ^ ow[0];
#pragma unroll
          for (int p = 1; p < P; ++p) d = __builtin_amdgcn_bitop3_b32(mine[r][p][w], ow[p], d, kXorOr);
          mism[r] += __popc(d);
        }
      }
      int wc = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool sim = (m0 + (int64_t)kRwThreads * r < M) && mism[r] <= maxmis;
        count[r] += sim ? 1 : 0;
        if (!own) wc += __popcll(__ballot(sim));
      }
      if (!own && lane == 0) colpart[wid][nl] = wc;
    }
    if (!own) {
      __syncthreads();
      if (threadIdx.x < nload) {
        int c = 0;
#pragma unroll
        for (int v = 0; v < kRwThreads / 64; ++v) c += colpart[v][threadIdx.x];
        if (c > 0) atomicAdd(n_sim + n0 + threadIdx.x, c);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t m = m0 + (int64_t)kRwThreads * r;
    if (m < M && count[r] > 0) atomicAdd(n_sim + m, count[r]);
  }
}

__global__ void k_zero_counts(int32_t* __restrict__ n, int64_t M) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) n[i] = 0;
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

template <int P, int W>
static void launch_count_pw(const uint32_t* planes, int64_t M, int L, int T, int32_t* n_sim,
                            hipStream_t s) {
  // two rows per thread while the planes fit comfortably in registers
  constexpr int R = (P * W <= 40) ? 2 : 1;
  const int64_t stages = ceil_div(M, kRwThreads);
  const int64_t rowblocks = ceil_div(M, (int64_t)kRwThreads * R);
  int64_t items = 0;
  for (int64_t rb = 0; rb < rowblocks; ++rb) items += ceil_div(stages - rb * R, kRwChunk);
  hipLaunchKernelGGL((k_count_similar<P, W, R>), dim3((unsigned)items), dim3(kRwThreads), 0, s,
                     planes, M, L, T, n_sim);
}

template <int W>
static void launch_count_w(const uint32_t* planes, int64_t M, int P, int L, int T, int32_t* n_sim,
                           hipStream_t s) {
  switch (P) {
    case 1: launch_count_pw<1, W>(planes, M, L, T, n_sim, s); break;
    case 2: launch_count_pw<2, W>(planes, M, L, T, n_sim, s); break;
    case 3: launch_count_pw<3, W>(planes, M, L, T, n_sim, s); break;
    case 4: launch_count_pw<4, W>(planes, M, L, T, n_sim, s); break;
    default: launch_count_pw<5, W>(planes, M, L, T, n_sim, s); break;
  }
}

hipError_t launch_reweight(const int8_t* msa, int64_t M, int L, int q, int32_t T,
                           const ReweightPlan& plan, void* ws, int32_t* n_sim, double* w,
                           double* meff, int32_t* dev_err, hipStream_t s) {
  uint32_t* planes = reinterpret_cast<uint32_t*>(static_cast<char*>(ws) + plan.off_planes);
  const int W = plan.words, P = plan.planes;
  // Unused planes (p >= P) are never read; padding bits are written as 0.
  hipLaunchKernelGGL(k_encode_planes, dim3((unsigned)ceil_div(M * W, 256)), dim3(256), 0, s, msa,
                     M, L, q, P, W, planes, dev_err);
  hipLaunchKernelGGL(k_zero_counts, dim3((unsigned)ceil_div(M, 256)), dim3(256), 0, s, n_sim, M);
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
