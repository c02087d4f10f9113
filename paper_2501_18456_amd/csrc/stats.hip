// One- and two-site frequency statistics, Eq. (3) with the pseudocount of
// Eqs. (8)-(9) (adabmDCA 2.0, Sec. 2.3), and the unit-weight chain counts of
// the model marginals (Sec. 2.1).
//
// The two-site table is the symmetric product C = A^T B over the M rows of an
// alignment, A[m][(i,a)] = w_m [x_mi == a] and B[m][(i,a)] = [x_mi == a] (the
// one-hot matrix).  It runs on the matrix cores:
//   - tokens are first transposed to site-major XT[L][Mpad] so that the
//     tokens of one site for consecutive rows are contiguous;
//   - a workgroup owns a 128x128 output tile (only tiles on or above the
//     diagonal) and walks K in stages of 64 rows; each stage scatters the
//     one-hot entries of its rows into zeroed LDS tiles (one write per
//     (row, site), the rest of the tile is zero), the four waves run
//     32x32 MFMAs on a 64x64 sub-tile each, and the same threads then clear
//     exactly the entries they set;
//   - BF16: one-hot values are exact; a weight is split into hi + lo BF16
//     parts (two products into the same FP32 accumulator); FP32 partial sums
//     are flushed into FP64 registers every 512 rows.  Unit weights give
//     integer counts, exact in FP32 below 2^24 rows.
//   - FP32: 32x32x2 FP32 MFMAs on FP32 operands (the comparator form).
// K may be split across workgroups; every split writes its own FP64 plane
// and the planes are summed in split order (deterministic).
#include "common.hpp"
#include "internal.hpp"

namespace bmdca {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kTile = 128;             // output tile edge
constexpr int kKT = 64;                // rows per K stage
constexpr int kFlushStages = 8;        // 8 * 64 = 512 rows per FP32 partial sum
constexpr int kRowB = kKT * 2 + 16;    // BF16 tile row stride in bytes (padded)
constexpr int kRowF = kKT + 1;         // FP32 tile row stride in floats (padded)
constexpr int kItems = 5;              // packed 4-token items per thread and operand

enum { MODE_UNIT_BF16 = 0, MODE_HILO_BF16 = 1, MODE_F32 = 2 };

static int mode_of(int prec, bool weighted) {
  if (prec == 0) return MODE_F32;
  return weighted ? MODE_HILO_BF16 : MODE_UNIT_BF16;
}

StatsPlan plan_stats(int64_t M, int L, int q, int prec) {
  (void)prec;
  StatsPlan p{};
  const int64_t Lq = (int64_t)L * q;
  p.Mpad = ceil_div(M, kKT) * kKT;
  p.ntile = (int)ceil_div(Lq, kTile);
  p.nupper = p.ntile * (p.ntile + 1) / 2;
  // Split K so that the grid holds at least ~2 workgroups per CU (256 CUs),
  // keeping every split at least 8 stages long.
  const int64_t stages = p.Mpad / kKT;
  int64_t want = ceil_div(512, p.nupper);
  int64_t maxs = std::max<int64_t>(1, stages / 8);
  int64_t sp = std::min<int64_t>(want, maxs);
  sp = std::min<int64_t>(sp, 16);
  p.kchunk = ceil_div(stages, sp) * kKT;
  p.splits = (int)ceil_div(p.Mpad, p.kchunk);
  size_t o = 0;
  p.off_xt = o;    o = align256(o + (size_t)L * p.Mpad);
  p.off_whi = o;   o = align256(o + sizeof(uint16_t) * p.Mpad);
  p.off_wlo = o;   o = align256(o + sizeof(uint16_t) * p.Mpad);
  p.off_wf = o;    o = align256(o + sizeof(float) * p.Mpad);
  p.off_part = o;  o = align256(o + sizeof(double) * (size_t)p.splits * Lq * Lq);
  p.off_red = o;   o = align256(o + sizeof(double) * 64);
  p.total = o;
  return p;
}

// ---------------------------------------------------------------------------
// X [M][L] -> XT [L][Mpad]; padding rows and invalid tokens become -1.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_transpose_tokens(const int8_t* __restrict__ X, int64_t M,
                                                          int L, int q, int8_t* __restrict__ XT,
                                                          int64_t Mpad, int32_t* dev_err) {
  __shared__ int8_t t[64][65];
  const int64_t m0 = (int64_t)blockIdx.x * 64;
  const int i0 = blockIdx.y * 64;
  const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
  for (int r = ty; r < 64; r += 4) {
    const int64_t m = m0 + r;
    const int i = i0 + tx;
    int v = -1;
    if (m < M && i < L) {
      v = X[m * L + i];
      if (v < 0 || v >= q) {
        if (dev_err) atomicOr(dev_err, 1);
        v = -1;
      }
    }
    t[r][tx] = (int8_t)v;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int i = i0 + r;
    const int64_t m = m0 + tx;
    if (i < L && m < Mpad) XT[(size_t)i * Mpad + m] = t[tx][r];
  }
}

__device__ __forceinline__ uint16_t f32_to_bf16_rn(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Weight operands: hi = bf16(w), lo = bf16(w - hi) (FP64 difference), or the
// FP32 weight; padding rows get 0.  w == nullptr means unit weights.
__global__ void k_prep_weights(const double* __restrict__ w, int64_t M, int64_t Mpad,
                               uint16_t* __restrict__ whi, uint16_t* __restrict__ wlo,
                               float* __restrict__ wf) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= Mpad) return;
  const double v = (m < M) ? (w ? w[m] : 1.0) : 0.0;
  const uint16_t hi = f32_to_bf16_rn((float)v);
  const double rest = v - (double)bf16_to_f32(hi);
  whi[m] = hi;
  wlo[m] = f32_to_bf16_rn((float)rest);
  wf[m] = (float)v;
}

// ---------------------------------------------------------------------------
// Main product kernel.
// ---------------------------------------------------------------------------
struct Operand {
  int R0;      // first output row/column of the tile
  int i_lo;    // first site overlapping the tile
  int nitems;  // (site, 4-row group) items: nsites * kKT/4
};

__device__ __forceinline__ Operand make_operand(int R0, int L, int q) {
  Operand o;
  o.R0 = R0;
  o.i_lo = R0 / q;
  const int i_hi = min(L - 1, (R0 + kTile - 1) / q);
  o.nitems = (i_hi - o.i_lo + 1) * (kKT / 4);
  return o;
}

// Packed tokens of the items this thread owns in stage m0.
__device__ __forceinline__ void load_items(const int8_t* __restrict__ XT, int64_t Mpad,
                                           const Operand& o, int64_t m0, uint32_t (&tok)[kItems]) {
#pragma unroll
  for (int t = 0; t < kItems; ++t) {
    const int it = threadIdx.x + t * 256;
    tok[t] = 0xFFFFFFFFu;
    if (it < o.nitems) {
      const int si = o.i_lo + it / (kKT / 4);
      const int g = it % (kKT / 4);
      tok[t] = *reinterpret_cast<const uint32_t*>(XT + (size_t)si * Mpad + m0 + 4 * g);
    }
  }
}

// Scatter (or clear) the one-hot entries of this thread's items.
template <int MODE>
__device__ __forceinline__ void scatter_items(const Operand& o, int q, const uint32_t (&tok)[kItems],
                                              bool weighted_operand, bool clear,
                                              const uint16_t* whi_s, const uint16_t* wlo_s,
                                              const float* wf_s, unsigned char* t0,
                                              unsigned char* t1) {
#pragma unroll
  for (int t = 0; t < kItems; ++t) {
    const int it = threadIdx.x + t * 256;
    if (it >= o.nitems) continue;
    const int si = o.i_lo + it / (kKT / 4);
    const int g = it % (kKT / 4);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int tk = (int)(int8_t)((tok[t] >> (8 * e)) & 0xFF);
      if (tk < 0) continue;
      const int row = si * q + tk - o.R0;
      if (row < 0 || row >= kTile) continue;
      const int ml = 4 * g + e;
      if (MODE == MODE_F32) {
        float v = clear ? 0.0f : (weighted_operand ? wf_s[ml] : 1.0f);
        reinterpret_cast<float*>(t0)[row * kRowF + ml] = v;
      } else {
        uint16_t v0 = clear ? 0 : (weighted_operand ? whi_s[ml] : (uint16_t)0x3F80);
        *reinterpret_cast<uint16_t*>(t0 + row * kRowB + 2 * ml) = v0;
        if (MODE == MODE_HILO_BF16 && weighted_operand) {
          uint16_t v1 = clear ? 0 : wlo_s[ml];
          *reinterpret_cast<uint16_t*>(t1 + row * kRowB + 2 * ml) = v1;
        }
      }
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_onehot_products(const int8_t* __restrict__ XT,
                                                         int64_t Mpad, int L, int q,
                                                         const uint16_t* __restrict__ whi,
                                                         const uint16_t* __restrict__ wlo,
                                                         const float* __restrict__ wf,
                                                         int ntile, int64_t kchunk,
                                                         double* __restrict__ P) {
  constexpr bool kWeighted = (MODE != MODE_UNIT_BF16);
  constexpr int kOpBytes = (MODE == MODE_F32) ? kTile * kRowF * 4 : kTile * kRowB;
  constexpr int kNumA = (MODE == MODE_HILO_BF16) ? 2 : 1;
  __shared__ __attribute__((aligned(16))) unsigned char smem[(kNumA + 1) * kOpBytes];
  __shared__ uint16_t s_whi[2][kKT];
  __shared__ uint16_t s_wlo[2][kKT];
  __shared__ float s_wf[2][kKT];
  unsigned char* tA = smem;
  unsigned char* tA2 = smem + kOpBytes;  // lo part (HILO only)
  unsigned char* tB = smem + kNumA * kOpBytes;

  // Upper-triangle tile of this workgroup.
  int t = blockIdx.x, ti = 0;
  while (t >= ntile - ti) {
    t -= ntile - ti;
    ++ti;
  }
  const int tj = ti + t;
  const int Lq = L * q;
  const Operand oa = make_operand(ti * kTile, L, q);
  const Operand ob = make_operand(tj * kTile, L, q);
  const int64_t kbeg = (int64_t)blockIdx.y * kchunk;
  const int64_t kend = min(kbeg + kchunk, Mpad);

  // Zero the operand tiles once; afterwards every stage clears what it set.
  for (int k = threadIdx.x * 16; k < (kNumA + 1) * kOpBytes; k += 256 * 16)
    *reinterpret_cast<uint4*>(smem + k) = make_uint4(0, 0, 0, 0);

  const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
  const int wr = wid / 2, wc = wid % 2;
  const int lrow = lane % 32, lhalf = lane / 32;

  f32x16 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[b][v] = 0.0f;
  constexpr int kD = kWeighted ? 4 : 1;  // FP64 sums are only kept for weighted forms
  double dacc[kD][16];
#pragma unroll
  for (int b = 0; b < kD; ++b)
#pragma unroll
    for (int v = 0; v < 16; ++v) dacc[b][v] = 0.0;

  uint32_t curA[kItems], curB[kItems], nxtA[kItems], nxtB[kItems];
  // Prologue: stage kbeg.
  if (kbeg < kend) {
    load_items(XT, Mpad, oa, kbeg, curA);
    load_items(XT, Mpad, ob, kbeg, curB);
    if (threadIdx.x < kKT) {
      s_whi[0][threadIdx.x] = whi[kbeg + threadIdx.x];
      s_wlo[0][threadIdx.x] = wlo[kbeg + threadIdx.x];
      s_wf[0][threadIdx.x] = wf[kbeg + threadIdx.x];
    }
  }
  __syncthreads();
  if (kbeg < kend) {
    scatter_items<MODE>(oa, q, curA, kWeighted, false, s_whi[0], s_wlo[0], s_wf[0], tA, tA2);
    scatter_items<MODE>(ob, q, curB, false, false, s_whi[0], s_wlo[0], s_wf[0], tB, tB);
  }
  __syncthreads();

  int stage = 0;
  for (int64_t m0 = kbeg; m0 < kend; m0 += kKT, ++stage) {
    const int64_t mn = m0 + kKT;
    const bool has_next = mn < kend;
    uint16_t pw_hi = 0, pw_lo = 0;
    float pw_f = 0.0f;
    if (has_next) {
      load_items(XT, Mpad, oa, mn, nxtA);
      load_items(XT, Mpad, ob, mn, nxtB);
      if (threadIdx.x < kKT) {
        pw_hi = whi[mn + threadIdx.x];
        pw_lo = wlo[mn + threadIdx.x];
        pw_f = wf[mn + threadIdx.x];
      }
    }
    // ---- matrix-core phase on stage m0
    if (MODE == MODE_F32) {
      const float* fA = reinterpret_cast<const float*>(tA);
      const float* fB = reinterpret_cast<const float*>(tB);
#pragma unroll 4
      for (int kk = 0; kk < kKT / 2; ++kk) {
        const int k = 2 * kk + lhalf;
        const float a0 = fA[(64 * wr + lrow) * kRowF + k];
        const float a1 = fA[(64 * wr + 32 + lrow) * kRowF + k];
        const float b0 = fB[(64 * wc + lrow) * kRowF + k];
        const float b1 = fB[(64 * wc + 32 + lrow) * kRowF + k];
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[3], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < kKT / 16; ++kk) {
        const int kb = 2 * (16 * kk + 8 * lhalf);
        const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(tA + (64 * wr + lrow) * kRowB + kb);
        const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(tA + (64 * wr + 32 + lrow) * kRowB + kb);
        const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(tB + (64 * wc + lrow) * kRowB + kb);
        const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(tB + (64 * wc + 32 + lrow) * kRowB + kb);
        acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[3], 0, 0, 0);
        if (MODE == MODE_HILO_BF16) {
          const bf16x8 c0 = *reinterpret_cast<const bf16x8*>(tA2 + (64 * wr + lrow) * kRowB + kb);
          const bf16x8 c1 =
              *reinterpret_cast<const bf16x8*>(tA2 + (64 * wr + 32 + lrow) * kRowB + kb);
          acc[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(c0, b0, acc[0], 0, 0, 0);
          acc[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(c0, b1, acc[1], 0, 0, 0);
          acc[2] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(c1, b0, acc[2], 0, 0, 0);
          acc[3] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(c1, b1, acc[3], 0, 0, 0);
        }
      }
    }
    const int nb = (stage + 1) & 1;
    if (has_next && threadIdx.x < kKT) {
      s_whi[nb][threadIdx.x] = pw_hi;
      s_wlo[nb][threadIdx.x] = pw_lo;
      s_wf[nb][threadIdx.x] = pw_f;
    }
    __syncthreads();
    // ---- clear stage m0, set stage m0 + kKT (the same thread owns a cell in both)
    scatter_items<MODE>(oa, q, curA, kWeighted, true, nullptr, nullptr, nullptr, tA, tA2);
    scatter_items<MODE>(ob, q, curB, false, true, nullptr, nullptr, nullptr, tB, tB);
    if (has_next) {
      scatter_items<MODE>(oa, q, nxtA, kWeighted, false, s_whi[nb], s_wlo[nb], s_wf[nb], tA, tA2);
      scatter_items<MODE>(ob, q, nxtB, false, false, s_whi[nb], s_wlo[nb], s_wf[nb], tB, tB);
#pragma unroll
      for (int k = 0; k < kItems; ++k) {
        curA[k] = nxtA[k];
        curB[k] = nxtB[k];
      }
    }
    if constexpr (kWeighted) {
      if (((stage + 1) % kFlushStages) == 0 || !has_next) {
#pragma unroll
        for (int b = 0; b < kD; ++b)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            dacc[b][v] += (double)acc[b][v];
            acc[b][v] = 0.0f;
          }
      }
    }
    __syncthreads();
  }

  // ---- write this split's plane.  Accumulator element v of lane l in a
  // 32x32 block holds row 8*(v/4) + 4*(l/32) + v%4, column l%32.
  double* __restrict__ Ps = P + (size_t)blockIdx.y * (size_t)Lq * Lq;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int bi = b / 2, bj = b % 2;
    const int col = tj * kTile + 64 * wc + 32 * bj + lrow;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = ti * kTile + 64 * wr + 32 * bi + 8 * (v / 4) + 4 * lhalf + (v % 4);
      if (row < Lq && col < Lq) {
        double val;
        if constexpr (kWeighted)
          val = dacc[b][v];
        else
          val = (double)acc[b][v];
        Ps[(size_t)row * Lq + col] = val;
      }
    }
  }
}

hipError_t launch_onehot_products(const int8_t* X, const double* w, int64_t M, int L, int q,
                                  int prec, const StatsPlan& plan, void* ws, int32_t* dev_err,
                                  hipStream_t s) {
  char* base = static_cast<char*>(ws);
  int8_t* XT = reinterpret_cast<int8_t*>(base + plan.off_xt);
  uint16_t* whi = reinterpret_cast<uint16_t*>(base + plan.off_whi);
  uint16_t* wlo = reinterpret_cast<uint16_t*>(base + plan.off_wlo);
  float* wf = reinterpret_cast<float*>(base + plan.off_wf);
  double* P = reinterpret_cast<double*>(base + plan.off_part);

  hipLaunchKernelGGL(k_transpose_tokens, dim3((unsigned)(plan.Mpad / 64), (unsigned)ceil_div(L, 64)),
                     dim3(256), 0, s, X, M, L, q, XT, plan.Mpad, dev_err);
  hipLaunchKernelGGL(k_prep_weights, dim3((unsigned)ceil_div(plan.Mpad, 256)), dim3(256), 0, s, w,
                     M, plan.Mpad, whi, wlo, wf);
  dim3 grid((unsigned)plan.nupper, (unsigned)plan.splits);
  switch (mode_of(prec, w != nullptr)) {
    case MODE_UNIT_BF16:
      hipLaunchKernelGGL(k_onehot_products<MODE_UNIT_BF16>, grid, dim3(256), 0, s, XT, plan.Mpad, L,
                         q, whi, wlo, wf, plan.ntile, plan.kchunk, P);
      break;
    case MODE_HILO_BF16:
      hipLaunchKernelGGL(k_onehot_products<MODE_HILO_BF16>, grid, dim3(256), 0, s, XT, plan.Mpad, L,
                         q, whi, wlo, wf, plan.ntile, plan.kchunk, P);
      break;
    default:
      hipLaunchKernelGGL(k_onehot_products<MODE_F32>, grid, dim3(256), 0, s, XT, plan.Mpad, L, q,
                         whi, wlo, wf, plan.ntile, plan.kchunk, P);
      break;
  }
  return hipGetLastError();
}

// Canonical (upper) position of (r1, r2): min/max always lies in a computed tile.
__device__ __forceinline__ double sum_planes(const double* __restrict__ P, int S, size_t plane,
                                             int Lq, int r1, int r2) {
  const int a = min(r1, r2), b = max(r1, r2);
  const size_t k = (size_t)a * Lq + b;
  double v = 0.0;
  for (int s = 0; s < S; ++s) v += P[(size_t)s * plane + k];
  return v;
}

__global__ void k_reduce_partials(const double* __restrict__ P, int S, int Lq,
                                  double* __restrict__ C) {
  const size_t plane = (size_t)Lq * Lq;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < plane;
       k += (size_t)gridDim.x * blockDim.x) {
    const int r1 = (int)(k / Lq), r2 = (int)(k % Lq);
    C[k] = sum_planes(P, S, plane, Lq, r1, r2);
  }
}

hipError_t launch_reduce_partials(const StatsPlan& plan, const void* ws, int Lq, double* C,
                                  hipStream_t s) {
  const double* P = reinterpret_cast<const double*>(static_cast<const char*>(ws) + plan.off_part);
  const size_t plane = (size_t)Lq * Lq;
  const unsigned nb = (unsigned)std::min<size_t>(ceil_div(plane, 256), 16384);
  hipLaunchKernelGGL(k_reduce_partials, dim3(nb), dim3(256), 0, s, P, plan.splits, Lq, C);
  return hipGetLastError();
}

// M_eff = sum_m w_m: fixed thread-to-row map, fixed tree.
__global__ __launch_bounds__(1024) void k_meff(const double* __restrict__ w, int64_t M,
                                               double* __restrict__ meff) {
  __shared__ double sh[16];
  double v = 0.0;
  if (w) {
    for (int64_t m = threadIdx.x; m < M; m += blockDim.x) v += w[m];
  }
  const double t = block_sum_f64(v, sh);
  if (threadIdx.x == 0) *meff = w ? t : (double)M;
}

hipError_t launch_meff(const double* w, int64_t M, double* meff, hipStream_t s) {
  hipLaunchKernelGGL(k_meff, dim3(1), dim3(1024), 0, s, w, M, meff);
  return hipGetLastError();
}

// f1[r] = (1-alpha) * (C[r][r] / meff) + alpha / q
// f2 = (1-alpha) * (C / meff) + alpha / q^2 off the diagonal blocks,
//      delta_ab f1 on them.  Expression order follows the definitions.
__global__ void k_stats_epilogue(const double* __restrict__ P, int S, int L, int q,
                                 const double* __restrict__ meff_p, double pc,
                                 double* __restrict__ f1, double* __restrict__ f2) {
  const int Lq = L * q;
  const size_t plane = (size_t)Lq * Lq;
  const double meff = *meff_p;
  const double alpha = pc < 0.0 ? 1.0 / meff : pc;
  const double qq = (double)q * (double)q;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < plane;
       k += (size_t)gridDim.x * blockDim.x) {
    const int r1 = (int)(k / Lq), r2 = (int)(k % Lq);
    double out;
    if (r1 / q == r2 / q) {
      if (r1 == r2) {
        const double f = sum_planes(P, S, plane, Lq, r1, r1) / meff;
        const double t1 = (1.0 - alpha) * f;
        const double t2 = alpha / (double)q;
        out = t1 + t2;
        f1[r1] = out;
      } else {
        out = 0.0;
      }
    } else {
      const double f = sum_planes(P, S, plane, Lq, r1, r2) / meff;
      const double t1 = (1.0 - alpha) * f;
      const double t2 = alpha / qq;
      out = t1 + t2;
    }
    f2[k] = out;
  }
}

hipError_t launch_stats_epilogue(const StatsPlan& plan, const void* ws, int L, int q,
                                 const double* meff, double pseudocount, double* f1, double* f2,
                                 hipStream_t s) {
  const double* P = reinterpret_cast<const double*>(static_cast<const char*>(ws) + plan.off_part);
  const size_t plane = (size_t)L * q * (size_t)L * q;
  const unsigned nb = (unsigned)std::min<size_t>(ceil_div(plane, 256), 16384);
  hipLaunchKernelGGL(k_stats_epilogue, dim3(nb), dim3(256), 0, s, P, plan.splits, L, q, meff,
                     pseudocount, f1, f2);
  return hipGetLastError();
}

}  // namespace bmdca
