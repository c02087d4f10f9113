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
//     diagonal) and walks K in stages of 64 rows; the operand tiles are
//     double-buffered in LDS: while the four waves run 32x32 MFMAs on a 64x64
//     sub-tile each from one buffer, every thread clears the one-hot entries
//     it set two stages ago in the other buffer and writes those of the next
//     stage there (one write per (row, site); padding and out-of-tile
//     entries go to a trash row that is never read), so a stage needs one
//     barrier;
//   - BF16: one-hot values are exact; a weight is split into hi + lo BF16
//     parts (two products into the same FP32 accumulator); FP32 partial sums
//     are flushed into FP64 registers every 1024 rows.  Unit weights give
//     integer counts, exact in FP32 below 2^24 rows.
//   - the stage loop of the BF16 forms is unrolled four times so that the
//     token registers of the previous, current, next and after-next stage
//     rotate by name: a load issued two stages ahead is first read when its
//     entries are set, one stage later, and no register copy waits for it
//     (the FP32 form and q <= 3 rotate by copies: fewer live registers).
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
constexpr int kRowB = kKT * 2 + 16;    // BF16 tile row stride in bytes (padded)
constexpr int kRowF = kKT + 1;         // FP32 tile row stride in floats (padded)

enum { MODE_UNIT_BF16 = 0, MODE_HILO_BF16 = 1, MODE_F32 = 2 };

// K stages per FP32 partial sum before it is added into FP64: 1024 rows in
// the BF16 hi+lo form (two FP32 roundings per 16-row MFMA step, hi then lo:
// at most 128 roundings of a sum of nonnegative terms, <= 7.7e-6 relative,
// beside the <= 2^-18 of the hi+lo split), 512 rows in the FP32 form (2-row
// MFMA steps).
template <int MODE>
constexpr int flush_stages() { return MODE == MODE_HILO_BF16 ? 16 : 8; }

static int mode_of(int prec, bool weighted) {
  if (prec == 0) return MODE_F32;
  return weighted ? MODE_HILO_BF16 : MODE_UNIT_BF16;
}

// Tiles (ti, tj) of kTR rows x 128 columns that hold some (r, c) with r <= c.
static int64_t product_tiles(int Lq, int tr) {
  const int nA = (int)ceil_div(Lq, tr), nB = (int)ceil_div(Lq, kTile);
  int64_t n = 0;
  for (int ti = 0; ti < nA; ++ti) n += nB - (ti * tr) / kTile;
  return n;
}

StatsPlan plan_stats(int64_t M, int L, int q, int prec) {
  StatsPlan p{};
  const int64_t Lq = (int64_t)L * q;
  p.Mpad = ceil_div(M, kKT) * kKT;
  p.ntile = (int)ceil_div(Lq, kTile);
  p.nupper = p.ntile * (p.ntile + 1) / 2;
  // K splits: trade grid balance against the FP64 plane every split writes
  // and the finish reads back (~5 TB/s).  BF16 (hi+lo tiles of 64 rows, two
  // workgroups per CU): a stage costs 1024 cycles per CU pair of tiles; FP32
  // (128-row tiles, one per CU): 8192 cycles.
  const int64_t stages = p.Mpad / kKT;
  const int64_t tiles = product_tiles((int)Lq, prec == 0 ? kTile : 64);
  const int64_t slots = prec == 0 ? 256 : 512;
  const double stage_us = (prec == 0 ? 8192.0 : 1024.0) / 2400.0;
  const double plane_us = (double)p.nupper * kTile * kTile * 8.0 * 3.0 / 5.0e6;
  const int64_t maxs = std::max<int64_t>(1, std::min<int64_t>(16, stages / 4));
  int64_t sp = 1;
  double best = 0.0;
  for (int64_t c = 1; c <= maxs; ++c) {
    const double t = (double)ceil_div(tiles * c, slots) * (double)ceil_div(stages, c) * stage_us +
                     (double)c * plane_us;
    if (c == 1 || t < best) {
      best = t;
      sp = c;
    }
  }
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
                                                          int64_t Mpad, int32_t* dev_err,
                                                          const int64_t* __restrict__ count) {
  __shared__ int8_t t[64][65];
  if (count && *count < M) M = *count;
  const int64_t m0 = (int64_t)blockIdx.x * 64;
  if (m0 >= M) return;  // whole workgroup (its rows are not read), before the barrier
  const int i0 = blockIdx.y * 64;
  const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
  if ((L & 3) == 0 && (reinterpret_cast<uintptr_t>(X) & 3) == 0) {
    // rows of whole, aligned dwords: thread (row 16 k + tid / 16, dword tid % 16) loads
    // 4 tokens at once; the store side writes dwords of 4 consecutive rows
    __shared__ uint32_t tw[64][17];
    const int c = threadIdx.x % 16;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int r = 16 * k + threadIdx.x / 16;
      const int64_t m = m0 + r;
      const int i = i0 + 4 * c;
      uint32_t w = 0xFFFFFFFFu;  // -1 tokens
      if (m < M && i < L) {
        const uint32_t x = *reinterpret_cast<const uint32_t*>(X + m * L + i);
        w = 0u;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          int v = (int)(int8_t)(x >> (8 * e));
          if (v < 0 || v >= q) {
            if (dev_err) atomicOr(dev_err, 1);
            v = -1;
          }
          w |= ((uint32_t)v & 0xFFu) << (8 * e);
        }
      }
      tw[r][c] = w;
    }
    __syncthreads();
    // output dword (site i0 + j, sequences m0 + 4 d .. + 3): byte j of each row
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int j = 16 * k + threadIdx.x / 16, d = threadIdx.x % 16;
      const int i = i0 + j;
      uint32_t w = 0u;
#pragma unroll
      for (int e = 0; e < 4; ++e) w |= ((tw[4 * d + e][j >> 2] >> (8 * (j & 3))) & 0xFFu) << (8 * e);
      if (i < L) *reinterpret_cast<uint32_t*>(XT + (size_t)i * Mpad + m0 + 4 * d) = w;
    }
    return;
  }
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

hipError_t launch_transpose_tokens(const int8_t* X, int64_t M, int L, int q, int8_t* XT,
                                  int64_t Mpad, int32_t* dev_err, hipStream_t s,
                                  const int64_t* count) {
  hipLaunchKernelGGL(k_transpose_tokens, dim3((unsigned)(Mpad / 64), (unsigned)ceil_div(L, 64)),
                     dim3(256), 0, s, X, M, L, q, XT, Mpad, dev_err, count);
  return hipGetLastError();
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
//
// Entry ownership: wave w owns the sites i_lo + w + 4p (p < NP) of an operand
// tile and lane l owns row m0 + l of a stage, so a thread holds one token per
// (site, stage) and writes one entry, row (site*q + token - R0), column l.
// Distinct sites give distinct rows, so no two threads share a live entry.
// ---------------------------------------------------------------------------
struct Operand {
  int R0;      // first output row/column of the tile
  int i_lo;    // first site overlapping the tile
  int nsites;  // sites overlapping the tile
};

__device__ __forceinline__ Operand make_operand(int R0, int rows, int L, int q) {
  Operand o;
  o.R0 = R0;
  o.i_lo = R0 / q;
  const int i_hi = min(L - 1, (R0 + rows - 1) / q);
  o.nsites = i_hi - o.i_lo + 1;
  return o;
}

// Sites per 128-row tile are at most 127/q + 2; a pass gives one site to
// every wave.
static int passes_needed(int q, int waves) { return (int)ceil_div(127 / q + 2, waves); }

template <int NW, int NP>
__device__ __forceinline__ void load_tokens(const int8_t* __restrict__ XT, int64_t Mpad,
                                            const Operand& o, int64_t m0, int wid, int lane,
                                            int (&tok)[NP]) {
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int s = wid + NW * p;
    // padding (-1) reads as 255: past every tile row for any site base; a
    // site beyond the tile reads a valid site, replaced by 255 when the
    // entry is written (not here: the load stays in flight until then)
    const int site = o.i_lo + min(s, o.nsites - 1);
    tok[p] = (int)(uint8_t)XT[(size_t)site * Mpad + m0 + lane];
  }
}

// Writes value(s) at this thread's entries; a padding token, a site past the
// tile or a row outside the tile goes to the trash row ROWS.
template <int MODE, int NW, int NP, int ROWS>
__device__ __forceinline__ void put_entries(const Operand& o, int q, int wid, int lane,
                                            const int (&tok)[NP], unsigned char* t0,
                                            unsigned char* t1, bool two, uint16_t v0, uint16_t v1,
                                            float vf) {
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int s = wid + NW * p;
    // base is wave-uniform and > -q; tokens are in [0, q) or 255, and 255
    // (padding, or a site past the tile) always lands in the trash row
    const int base = (o.i_lo + s) * q - o.R0;
    const int tk = (s < o.nsites) ? tok[p] : 255;
    const int r = (int)min((unsigned)(tk + base), (unsigned)ROWS);
    if (MODE == MODE_F32) {
      *reinterpret_cast<float*>(t0 + r * (kRowF * 4) + 4 * lane) = vf;
    } else {
      const int off = r * kRowB + 2 * lane;
      *reinterpret_cast<uint16_t*>(t0 + off) = v0;
      if (MODE == MODE_HILO_BF16 && two) *reinterpret_cast<uint16_t*>(t1 + off) = v1;
    }
  }
}

// Output tile kTR x 128 per workgroup of four waves (2 x 2 wave tiles).  The
// hi+lo form takes 64-row tiles: its waves hold 32x64 (FP32 sums of the hi
// and lo products plus FP64 sums) and two workgroups share a CU, so one's barrier is
// covered by the other's matrix work.  The other forms take 128 x 128.
template <int MODE>
struct ProductShape {
  static constexpr int kWaves = 4;
  static constexpr int kTR = (MODE == MODE_HILO_BF16) ? 64 : kTile;
  static constexpr int kRB = kTR / 64;  // 32-row blocks per wave
};


template <int MODE, int NP>
__global__ __launch_bounds__(64 * ProductShape<MODE>::kWaves, (MODE == MODE_HILO_BF16) ? 2 : 1) void k_onehot_products(
    const int8_t* __restrict__ XT, int64_t Mpad, int L, int q, const uint16_t* __restrict__ whi,
    const uint16_t* __restrict__ wlo, const float* __restrict__ wf, int ntile, int64_t kchunk,
    double* __restrict__ P, const int32_t* __restrict__ active) {
  if (active && *active == 0) return;  // whole grid leaves before any barrier
  constexpr int NW = ProductShape<MODE>::kWaves;
  constexpr int RB = ProductShape<MODE>::kRB;
  constexpr int TR = ProductShape<MODE>::kTR;
  constexpr int kThreads = 64 * NW;
  constexpr bool kWeighted = (MODE != MODE_UNIT_BF16);
  constexpr bool kLo = (MODE == MODE_HILO_BF16);
  // one extra (trash) row per operand tile
  constexpr int kRowBytes = (MODE == MODE_F32) ? kRowF * 4 : kRowB;
  constexpr int kOpA = (TR + 1) * kRowBytes;
  constexpr int kOpB = (kTile + 1) * kRowBytes;
  constexpr int kNumA = kLo ? 2 : 1;
  constexpr int kBuf = kNumA * kOpA + kOpB;
  __shared__ __attribute__((aligned(16))) unsigned char smem[2 * kBuf];

  // Tile of this workgroup: row tile ti, column tiles from (ti*TR)/128 on.
  int t = blockIdx.x, ti = 0;
  while (t >= ntile - (ti * TR) / kTile) {
    t -= ntile - (ti * TR) / kTile;
    ++ti;
  }
  const int tj = (ti * TR) / kTile + t;
  const int Lq = L * q;
  const Operand oa = make_operand(ti * TR, TR, L, q);
  const Operand ob = make_operand(tj * kTile, kTile, L, q);
  const int64_t kbeg = (int64_t)blockIdx.y * kchunk;
  const int64_t kend = min(kbeg + kchunk, Mpad);

  for (int k = threadIdx.x * 16; k < 2 * kBuf; k += kThreads * 16)
    *reinterpret_cast<uint4*>(smem + k) = make_uint4(0, 0, 0, 0);

  const int lane = threadIdx.x % 64;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int wr = wid / 2, wc = wid % 2;  // wave tile: rows 32*RB*wr.., columns 64*wc..
  const int lrow = lane % 32, lhalf = lane / 32;
  constexpr uint16_t kOne = 0x3F80;  // BF16 1.0

  // acc[rb][cb]: FP32 partial sums (hi then lo product in the hi+lo form)
  f32x16 acc[RB][2];
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[b][c][v] = 0.0f;
  constexpr int kD = kWeighted ? RB * 2 : 1;  // FP64 sums only for weighted forms
  double dacc[kD][16];
#pragma unroll
  for (int b = 0; b < kD; ++b)
#pragma unroll
    for (int v = 0; v < 16; ++v) dacc[b][v] = 0.0;

  auto load_w = [&](int64_t m, uint16_t& hi, uint16_t& lo, float& f) {
    if (MODE == MODE_HILO_BF16) {
      hi = whi[m + lane];
      lo = wlo[m + lane];
    }
    if (MODE == MODE_F32) f = wf[m + lane];
  };
  auto put_a = [&](const int(&tok)[NP], unsigned char* buf, bool clear, uint16_t hi, uint16_t lo,
                   float f) {
    const uint16_t v0 = clear ? (uint16_t)0 : (MODE == MODE_HILO_BF16 ? hi : kOne);
    const uint16_t v1 = clear ? (uint16_t)0 : lo;
    const float vf = clear ? 0.0f : f;
    put_entries<MODE, NW, NP, TR>(oa, q, wid, lane, tok, buf, buf + kOpA, true, v0, v1, vf);
  };
  auto put_b = [&](const int(&tok)[NP], unsigned char* buf, bool clear) {
    put_entries<MODE, NW, NP, kTile>(ob, q, wid, lane, tok, buf + kNumA * kOpA, nullptr, false,
                              clear ? (uint16_t)0 : kOne, 0, clear ? 0.0f : 1.0f);
  };

  // Token sets T0..T3 (A and B operand) and weight sets W0, W1.  Stage st
  // holds its own tokens in T[st % 4]; the tokens of stage st - 1 (cleared
  // at st) in T[(st + 3) % 4], of st + 1 (set at st) in T[(st + 1) % 4], and
  // loads those of st + 2 into T[(st + 2) % 4]; the weights of st + 1 are in
  // W[(st + 1) % 2], those of st + 2 go to W[st % 2].  Before the first stage
  // the "previous" tokens are 255, so their clears go to the trash row.
  int T0a[NP], T0b[NP], T1a[NP], T1b[NP], T2a[NP], T2b[NP], T3a[NP], T3b[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) T3a[p] = T3b[p] = 255;
  uint16_t W0h = 0, W0l = 0, W1h = 0, W1l = 0;
  float W0f = 0.0f, W1f = 0.0f;
  load_tokens<NW, NP>(XT, Mpad, oa, kbeg, wid, lane, T0a);
  load_tokens<NW, NP>(XT, Mpad, ob, kbeg, wid, lane, T0b);
  {
    uint16_t hi0 = 0, lo0 = 0;
    float f0 = 0.0f;
    load_w(kbeg, hi0, lo0, f0);
    // stage after the first (the last stage again when there is none)
    const int64_t m1 = min(kbeg + kKT, kend - kKT);
    load_tokens<NW, NP>(XT, Mpad, oa, m1, wid, lane, T1a);
    load_tokens<NW, NP>(XT, Mpad, ob, m1, wid, lane, T1b);
    load_w(m1, W1h, W1l, W1f);
    __syncthreads();
    put_a(T0a, smem, false, hi0, lo0, f0);
    put_b(T0b, smem, false);
    __syncthreads();
  }

  const int arow0 = 32 * RB * wr + lrow;  // first A row of this lane
  const int brow0 = 64 * wc + lrow;       // first B row of this lane
  // One stage: matrix work on the buffer of stage st, then the other buffer
  // gets the clears of stage st - 1 and the entries of stage st + 1.
  auto stage = [&](int64_t m0, int st, const int(&aP)[NP], const int(&bP)[NP],
                   const int(&aN)[NP], const int(&bN)[NP], int(&aNN)[NP], int(&bNN)[NP],
                   uint16_t hiN, uint16_t loN, float fN, uint16_t& hiNN, uint16_t& loNN,
                   float& fNN) {
    const bool has1 = m0 + kKT < kend;
    {  // loads two stages ahead (clamped to the last stage: used only if it exists)
      const int64_t m2 = min(m0 + 2 * kKT, kend - kKT);
      load_tokens<NW, NP>(XT, Mpad, oa, m2, wid, lane, aNN);
      load_tokens<NW, NP>(XT, Mpad, ob, m2, wid, lane, bNN);
      load_w(m2, hiNN, loNN, fNN);
    }
    const unsigned char* cur = smem + (st & 1) * kBuf;
    unsigned char* other = smem + ((st & 1) ^ 1) * kBuf;
    const unsigned char* tA = cur;
    const unsigned char* tA2 = cur + kOpA;
    const unsigned char* tB = cur + kNumA * kOpA;
    // ---- matrix-core phase on stage m0
    if (MODE == MODE_F32) {
      const float* fA = reinterpret_cast<const float*>(tA);
      const float* fB = reinterpret_cast<const float*>(tB);
#pragma unroll 4
      for (int kk = 0; kk < kKT / 2; ++kk) {
        const int k = 2 * kk + lhalf;
        float a[RB], b[2];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) a[rb] = fA[(arow0 + 32 * rb) * kRowF + k];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) b[cb] = fB[(brow0 + 32 * cb) * kRowF + k];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb)
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rb], b[cb], acc[rb][cb], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < kKT / 16; ++kk) {
        const int kb = 2 * (16 * kk + 8 * lhalf);
        bf16x8 a[RB], c[RB], b[2];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          a[rb] = *reinterpret_cast<const bf16x8*>(tA + (arow0 + 32 * rb) * kRowB + kb);
          if (kLo) c[rb] = *reinterpret_cast<const bf16x8*>(tA2 + (arow0 + 32 * rb) * kRowB + kb);
        }
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          b[cb] = *reinterpret_cast<const bf16x8*>(tB + (brow0 + 32 * cb) * kRowB + kb);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) {
            acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[rb], b[cb], acc[rb][cb], 0, 0, 0);
            if (kLo)
              acc[rb][cb] =
                  __builtin_amdgcn_mfma_f32_32x32x16_bf16(c[rb], b[cb], acc[rb][cb], 0, 0, 0);
          }
      }
    }
    // ---- other buffer: clear stage m0 - kKT, set stage m0 + kKT.  Nobody
    // reads it during this stage (its last readers passed the previous
    // barrier).  Both run every stage: before the first stage the clears go
    // to the trash row, after the last the buffer is not read again.
    put_a(aP, other, true, 0, 0, 0.0f);
    put_b(bP, other, true);
    put_a(aN, other, false, hiN, loN, fN);
    put_b(bN, other, false);

    if constexpr (kWeighted) {
      if (((st + 1) % flush_stages<MODE>()) == 0 || !has1) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
              dacc[rb * 2 + cb][v] += (double)acc[rb][cb][v];
              acc[rb][cb][v] = 0.0f;
            }
      }
    }
    __syncthreads();
  };

  const int nst = (int)((kend - kbeg) / kKT);
  int st = 0;
  if constexpr (MODE == MODE_F32 || NP > 9) {
    // register-heavy forms: the sets keep their roles and rotate by copies
    // (each copy waits for its load; fewer registers stay live)
    for (; st < nst; ++st) {
      stage(kbeg + (int64_t)st * kKT, st, T3a, T3b, T1a, T1b, T2a, T2b, W1h, W1l, W1f, W0h, W0l,
            W0f);
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        T3a[p] = T0a[p];
        T3b[p] = T0b[p];
        T0a[p] = T1a[p];
        T0b[p] = T1b[p];
        T1a[p] = T2a[p];
        T1b[p] = T2b[p];
      }
      W1h = W0h;
      W1l = W0l;
      W1f = W0f;
    }
  } else {
    // groups of four stages (one loop exit keeps every accumulator in its
    // registers), then the last 0-3 stages
    for (; st + 4 <= nst; st += 4) {
      const int64_t m0 = kbeg + (int64_t)st * kKT;
      stage(m0, st, T3a, T3b, T1a, T1b, T2a, T2b, W1h, W1l, W1f, W0h, W0l, W0f);
      stage(m0 + kKT, st + 1, T0a, T0b, T2a, T2b, T3a, T3b, W0h, W0l, W0f, W1h, W1l, W1f);
      stage(m0 + 2 * kKT, st + 2, T1a, T1b, T3a, T3b, T0a, T0b, W1h, W1l, W1f, W0h, W0l, W0f);
      stage(m0 + 3 * kKT, st + 3, T2a, T2b, T0a, T0b, T1a, T1b, W0h, W0l, W0f, W1h, W1l, W1f);
    }
    if (st < nst) {
      const int64_t m0 = kbeg + (int64_t)st * kKT;
      stage(m0, st, T3a, T3b, T1a, T1b, T2a, T2b, W1h, W1l, W1f, W0h, W0l, W0f);
      if (st + 1 < nst) {
        stage(m0 + kKT, st + 1, T0a, T0b, T2a, T2b, T3a, T3b, W0h, W0l, W0f, W1h, W1l, W1f);
        if (st + 2 < nst)
          stage(m0 + 2 * kKT, st + 2, T1a, T1b, T3a, T3b, T0a, T0b, W1h, W1l, W1f, W0h, W0l,
                W0f);
      }
    }
  }

  // ---- write this split's plane.  Accumulator element v of lane l in a
  // 32x32 block holds row 8*(v/4) + 4*(l/32) + v%4, column l%32.
  double* __restrict__ Ps = P + (size_t)blockIdx.y * (size_t)Lq * Lq;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      const int col = tj * kTile + 64 * wc + 32 * cb + lrow;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = ti * TR + 32 * RB * wr + 32 * rb + 8 * (v / 4) + 4 * lhalf + (v % 4);
        if (row < Lq && col < Lq) {
          double val;
          if constexpr (kWeighted)
            val = dacc[rb * 2 + cb][v];
          else
            val = (double)acc[rb][cb][v];
          Ps[(size_t)row * Lq + col] = val;
        }
      }
    }
}

template <int MODE>
static void launch_products_mode(int q, int splits, hipStream_t s, const int8_t* XT, int64_t Mpad,
                                 int L, const uint16_t* whi, const uint16_t* wlo, const float* wf,
                                 int64_t kchunk, double* P, const int32_t* active) {
  constexpr int NW = ProductShape<MODE>::kWaves;
  const int np = passes_needed(q, NW);
  const dim3 block(64 * NW);
  const int ntile = (int)ceil_div(L * q, kTile);
  const dim3 grid((unsigned)product_tiles(L * q, ProductShape<MODE>::kTR), (unsigned)splits);
#define BMDCA_LAUNCH_NP(N)                                                                    \
  hipLaunchKernelGGL((k_onehot_products<MODE, N>), grid, block, 0, s, XT, Mpad, L, q, whi, wlo, \
                     wf, ntile, kchunk, P, active)
  if (np <= 1)
    BMDCA_LAUNCH_NP(1);
  else if (np <= 2)
    BMDCA_LAUNCH_NP(2);
  else if (np <= 4)
    BMDCA_LAUNCH_NP(4);
  else if (np <= 9)
    BMDCA_LAUNCH_NP(9);
  else
    BMDCA_LAUNCH_NP(17);  // q >= 2 needs at most 17 passes of 4 waves
#undef BMDCA_LAUNCH_NP
}

hipError_t launch_onehot_products(const int8_t* X, const double* w, int64_t M, int L, int q,
                                  int prec, const StatsPlan& plan, void* ws, int32_t* dev_err,
                                  hipStream_t s, const int32_t* active) {
  char* base = static_cast<char*>(ws);
  int8_t* XT = reinterpret_cast<int8_t*>(base + plan.off_xt);
  uint16_t* whi = reinterpret_cast<uint16_t*>(base + plan.off_whi);
  uint16_t* wlo = reinterpret_cast<uint16_t*>(base + plan.off_wlo);
  float* wf = reinterpret_cast<float*>(base + plan.off_wf);
  double* P = reinterpret_cast<double*>(base + plan.off_part);

  hipLaunchKernelGGL(k_transpose_tokens, dim3((unsigned)(plan.Mpad / 64), (unsigned)ceil_div(L, 64)),
                     dim3(256), 0, s, X, M, L, q, XT, plan.Mpad, dev_err, nullptr);
  hipLaunchKernelGGL(k_prep_weights, dim3((unsigned)ceil_div(plan.Mpad, 256)), dim3(256), 0, s, w,
                     M, plan.Mpad, whi, wlo, wf);
  switch (mode_of(prec, w != nullptr)) {
    case MODE_UNIT_BF16:
      launch_products_mode<MODE_UNIT_BF16>(q, plan.splits, s, XT, plan.Mpad, L, whi, wlo, wf,
                                           plan.kchunk, P, active);
      break;
    case MODE_HILO_BF16:
      launch_products_mode<MODE_HILO_BF16>(q, plan.splits, s, XT, plan.Mpad, L, whi, wlo, wf,
                                           plan.kchunk, P, active);
      break;
    default:
      launch_products_mode<MODE_F32>(q, plan.splits, s, XT, plan.Mpad, L, whi, wlo, wf,
                                     plan.kchunk, P, active);
      break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Finish: the partial planes hold only tiles on or above the diagonal.  A
// 64x64 output block (bi, bj) reads the stored block (min, max) coalesced,
// summed over the splits in split order, and mirrors it through LDS.
// ---------------------------------------------------------------------------
constexpr int kFin = 64;

__device__ __forceinline__ void load_sym_block(const double* __restrict__ P, int S, int Lq, int bi,
                                               int bj, double (*sh)[kFin + 1]) {
  const int r0 = min(bi, bj) * kFin, c0 = max(bi, bj) * kFin;
  const size_t plane = (size_t)Lq * Lq;
  for (int e = threadIdx.x; e < kFin * kFin; e += blockDim.x) {
    const int r = e / kFin, c = e % kFin;
    double v = 0.0;
    if (r0 + r < Lq && c0 + c < Lq) {
      const size_t k = (size_t)(r0 + r) * Lq + c0 + c;
      for (int sp = 0; sp < S; ++sp) v += P[(size_t)sp * plane + k];
    }
    sh[r][c] = v;
  }
  __syncthreads();
}

// Value of output (R1, R2) = stored (min, max), both inside block (bi, bj).
__device__ __forceinline__ double sym_value(const double (*sh)[kFin + 1], int bi, int bj, int R1,
                                            int R2) {
  const int a = min(R1, R2), b = max(R1, R2);
  return sh[a - min(bi, bj) * kFin][b - max(bi, bj) * kFin];
}

// One workgroup per stored block (bi <= bj): the block is read once and
// written to (bi, bj) and, transposed through LDS, to (bj, bi).
__global__ __launch_bounds__(256) void k_reduce_partials(const double* __restrict__ P, int S,
                                                         int Lq, double* __restrict__ C) {
  __shared__ double sh[kFin][kFin + 1];
  // triangular index t -> (bi, bj), bj (bj + 1) / 2 <= t < (bj + 1) (bj + 2) / 2
  const int t = blockIdx.x;
  int bj = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((bj + 1) * (bj + 2) / 2 <= t) ++bj;
  while (bj * (bj + 1) / 2 > t) --bj;
  const int bi = t - bj * (bj + 1) / 2;
  load_sym_block(P, S, Lq, bi, bj, sh);
  for (int e = threadIdx.x; e < kFin * kFin; e += blockDim.x) {
    const int R1 = bi * kFin + e / kFin, R2 = bj * kFin + e % kFin;
    if (R1 < Lq && R2 < Lq) C[(size_t)R1 * Lq + R2] = sym_value(sh, bi, bj, R1, R2);
  }
  if (bi == bj) return;
  for (int e = threadIdx.x; e < kFin * kFin; e += blockDim.x) {
    const int R1 = bj * kFin + e / kFin, R2 = bi * kFin + e % kFin;
    if (R1 < Lq && R2 < Lq) C[(size_t)R1 * Lq + R2] = sym_value(sh, bj, bi, R1, R2);
  }
}

hipError_t launch_reduce_partials(const StatsPlan& plan, const void* ws, int Lq, double* C,
                                  hipStream_t s) {
  const double* P = reinterpret_cast<const double*>(static_cast<const char*>(ws) + plan.off_part);
  const unsigned nb = (unsigned)ceil_div(Lq, kFin);
  hipLaunchKernelGGL(k_reduce_partials, dim3(nb * (nb + 1) / 2), dim3(256), 0, s, P, plan.splits,
                     Lq, C);
  return hipGetLastError();
}

// M_eff = sum_m w_m: fixed thread-to-row map, fixed tree.
// ---------------------------------------------------------------------------
// Chain counts by direct counting (Eq. 3 with unit weights): C[(i,a)][(j,b)] =
// #{n : s_i(n) = a, s_j(n) = b}, exact in u32 and written as FP64 to the full
// symmetric matrix (the diagonal block of site i holds n_i(a) on its
// diagonal).  Workgroup (jg, i) counts site i against the sites
// j = kPCG jg .. kPCG jg + kPCG - 1 with i <= j < L, one LDS histogram per j,
// reading the site-major tokens XT [L][Mpad] four chains per dword.  The bin
// of (a, b) is a * ROW + b with both tokens clamped to ROW - 1 (33 for q > 8,
// 9 for q <= 8): padding and invalid tokens (0xFF) land in that row or
// column, which is never written out, and the odd row length spreads a
// wave's increments over the LDS banks.  Histograms of 33 x 33 bins (4.4 KB)
// leave room for several workgroups per CU (64 x 65 bins over the tokens'
// low 6 bits, without the clamps, ran 1.2-2.1x longer).
// ---------------------------------------------------------------------------
constexpr int kPCG = 4;

// ROW: bins per histogram row (tokens clamped to ROW - 1, the trash row and
// column); NC: copies of each histogram, lane group l / (64 / NC) of a wave
// adding to copy l * NC / 64, summed when written out.  For q <= 8 a wave's
// 64 increments fall on at most 64 bins and the same-bin adds serialize, so
// 8 copies of 9 x 9 bins spread them.
template <int ROW, int NC>
__global__ __launch_bounds__(256) void k_pair_counts(const int8_t* __restrict__ XT, int64_t Mpad,
                                                     int L, int q, double* __restrict__ C,
                                                     const int32_t* __restrict__ active) {
  constexpr int kBins = ROW * ROW;
  constexpr uint32_t kTrash = ROW - 1;
  __shared__ uint32_t hist[kPCG][NC * kBins];
  if (active && *active == 0) return;
  const int i = blockIdx.y, j0 = blockIdx.x * kPCG;
  if (j0 + kPCG - 1 < i) return;  // the whole group lies below the diagonal
  for (int e = threadIdx.x; e < kPCG * NC * kBins; e += 256) (&hist[0][0])[e] = 0u;
  __syncthreads();
  const uint32_t cbase = (uint32_t)((threadIdx.x % 64) / (64 / NC)) * kBins;
  const int64_t nd = Mpad / 4;
  const uint32_t* xi = reinterpret_cast<const uint32_t*>(XT + (size_t)i * Mpad);
  const uint32_t* xj[kPCG];
  bool on[kPCG];
#pragma unroll
  for (int g = 0; g < kPCG; ++g) {
    on[g] = j0 + g >= i && j0 + g < L;
    xj[g] = reinterpret_cast<const uint32_t*>(XT + (size_t)min(j0 + g, L - 1) * Mpad);
  }
  // two dwords per thread and iteration, all loads issued before the first
  // increment (the sites past L or below i load a valid row and skip)
  for (int64_t d0 = threadIdx.x; d0 < nd; d0 += 512) {
    const bool two = d0 + 256 < nd;
    const int64_t d1 = two ? d0 + 256 : d0;
    uint32_t wi[2], wj[2][kPCG];
    wi[0] = xi[d0];
    wi[1] = xi[d1];
#pragma unroll
    for (int g = 0; g < kPCG; ++g) {
      wj[0][g] = xj[g][d0];
      wj[1][g] = xj[g][d1];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (u == 1 && !two) break;
      uint32_t ra[4];
#pragma unroll
      for (int e = 0; e < 4; ++e)
        ra[e] = cbase + min(__builtin_amdgcn_ubfe(wi[u], 8 * e, 8), kTrash) * ROW;
#pragma unroll
      for (int g = 0; g < kPCG; ++g) {
        if (!on[g]) continue;  // uniform
#pragma unroll
        for (int e = 0; e < 4; ++e)
          atomicAdd(&hist[g][ra[e] + min(__builtin_amdgcn_ubfe(wj[u][g], 8 * e, 8), kTrash)], 1u);
      }
    }
  }
  __syncthreads();
  const int Lq = L * q, qq = q * q;
  auto count = [&](int g, int a, int b) {
    uint32_t c = 0u;
#pragma unroll
    for (int k = 0; k < NC; ++k) c += hist[g][k * kBins + a * ROW + b];
    return (double)c;
  };
#pragma unroll
  for (int g = 0; g < kPCG; ++g) {
    if (!on[g]) continue;
    const int j = j0 + g;
    for (int e = threadIdx.x; e < qq; e += 256) {
      const int a = e / q, b = e - a * q;  // rows (i, a), b fastest
      C[(size_t)(i * q + a) * Lq + j * q + b] = count(g, a, b);
    }
    if (j == i) continue;
    for (int e = threadIdx.x; e < qq; e += 256) {
      const int b = e / q, a = e - b * q;  // rows (j, b), a fastest
      C[(size_t)(j * q + b) * Lq + i * q + a] = count(g, a, b);
    }
  }
}

hipError_t launch_pair_counts(const int8_t* X, int64_t N, int L, int q, const StatsPlan& plan,
                              void* ws, double* C, int32_t* dev_err, hipStream_t s,
                              const int32_t* active) {
  if (q > 32 || L < 1) return hipErrorInvalidValue;
  int8_t* XT = reinterpret_cast<int8_t*>(static_cast<char*>(ws) + plan.off_xt);
  const hipError_t e = launch_transpose_tokens(X, N, L, q, XT, plan.Mpad, dev_err, s);
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)ceil_div(L, kPCG), (unsigned)L);
  if (q <= 8)
    hipLaunchKernelGGL((k_pair_counts<9, 8>), grid, dim3(256), 0, s, XT, plan.Mpad, L, q, C, active);
  else
    hipLaunchKernelGGL((k_pair_counts<33, 1>), grid, dim3(256), 0, s, XT, plan.Mpad, L, q, C,
                       active);
  return hipGetLastError();
}

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
__global__ __launch_bounds__(256) void k_stats_epilogue(const double* __restrict__ P, int S, int L,
                                                        int q, const double* __restrict__ meff_p,
                                                        double pc, double* __restrict__ f1,
                                                        double* __restrict__ f2) {
  __shared__ double sh[kFin][kFin + 1];
  const int Lq = L * q;
  // one workgroup per stored block (bi <= bj, triangular index as in
  // k_reduce_partials): output blocks (bi, bj) and, if distinct, (bj, bi)
  const int t = blockIdx.x;
  int bj = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while ((bj + 1) * (bj + 2) / 2 <= t) ++bj;
  while (bj * (bj + 1) / 2 > t) --bj;
  const int bi = t - bj * (bj + 1) / 2;
  load_sym_block(P, S, Lq, bi, bj, sh);
  const double meff = *meff_p;
  const double alpha = pc < 0.0 ? 1.0 / meff : pc;
  const double qq = (double)q * (double)q;
  auto emit = [&](int b1, int b2) {
    for (int e = threadIdx.x; e < kFin * kFin; e += blockDim.x) {
      const int r1 = b1 * kFin + e / kFin, r2 = b2 * kFin + e % kFin;
      if (r1 >= Lq || r2 >= Lq) continue;
      double out;
      if (r1 / q == r2 / q) {
        if (r1 == r2) {
          const double f = sym_value(sh, b1, b2, r1, r1) / meff;
          const double t1 = (1.0 - alpha) * f;
          const double t2 = alpha / (double)q;
          out = t1 + t2;
          f1[r1] = out;
        } else {
          out = 0.0;
        }
      } else {
        const double f = sym_value(sh, b1, b2, r1, r2) / meff;
        const double t1 = (1.0 - alpha) * f;
        const double t2 = alpha / qq;
        out = t1 + t2;
      }
      f2[(size_t)r1 * Lq + r2] = out;
    }
  };
  emit(bi, bj);
  if (bi != bj) emit(bj, bi);
}

hipError_t launch_stats_epilogue(const StatsPlan& plan, const void* ws, int L, int q,
                                 const double* meff, double pseudocount, double* f1, double* f2,
                                 hipStream_t s) {
  const double* P = reinterpret_cast<const double*>(static_cast<const char*>(ws) + plan.off_part);
  const unsigned nb = (unsigned)ceil_div(L * q, kFin);
  hipLaunchKernelGGL(k_stats_epilogue, dim3(nb * (nb + 1) / 2), dim3(256), 0, s, P, plan.splits, L,
                     q, meff, pseudocount, f1, f2);
  return hipGetLastError();
}

}  // namespace bmdca
