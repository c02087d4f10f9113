// Downstream scores of a trained model (adabmDCA 2.0, Sec. 4):
//   - energies of a batch of sequences, Eq. (1) (Sec. 4.3);
//   - single-mutant energy differences from the wild type's local fields
//     (Sec. 4.4);
//   - zero-sum-gauge Frobenius norms with the average-product correction,
//     Eq. (13) (Sec. 4.2).
#include "common.hpp"
#include "internal.hpp"

namespace bmdca {

// ---------------------------------------------------------------------------
// Energy of a batch, Eq. (1), tiled over sequences and coupling tiles.
//
// The pairs i < j are walked as steps (column chunk jc of kEJC sites, row
// site i), jc outer: a step needs the q x (kEJC*q) tile of J with rows
// (i, a) and columns (j, b), j in the chunk.  A workgroup owns 2048 (q > 8)
// or 1024 sequences (four per thread) and one contiguous range of steps; it stages
// each tile in LDS once (double-buffered through registers) and every
// sequence picks J[(i, s_i), (j, s_j)] for its own tokens.  A step's 16
// terms are summed in FP32 in column order and the step sums in FP64 in step
// order, one FP64 partial sum per (range, sequence); the finish adds the
// fields and the partials in range order.
// The ranges depend on L only, so a sequence's energy does not depend on the
// rest of the batch (nor on the workgroup size).
// ---------------------------------------------------------------------------
constexpr int kEJC = 16;
constexpr int kESeq = 4;  // sequences per thread
// Threads per workgroup: 512 (2048 sequences) for q > 8, so that each staged
// tile serves twice the lookups (a workgroup loads its own copy of every
// tile; at q = 21 the tile stores were about 30% of the LDS traffic): L = 512,
// q = 21, 1e5 sequences 4.37 -> 3.30 ms, q = 32 -1/3.  For q <= 8 (tiles of
// at most 8 KB) 256, where 512 measured 3-4% slower.
constexpr int energy_threads(int Q) { return Q > 8 ? 512 : 256; }

// Row pitch of the LDS tile in floats: 16 Q plus a pad of 0, 4, 8 or 12
// (rows stay 16-byte aligned).  A lookup's bank is (P s_i + s_j + const) mod
// 64 over the 64 four-byte banks; the pad is the one whose largest share of
// the Q^2 pairs (s_i, s_j) in one bank is smallest, then the smallest sum of
// squared shares, among the pads that keep as many workgroups per CU (two
// tiles in 160 KB of LDS).  With P = 16 Q the row offsets take
// 64 / gcd(16 Q, 64) values only: at q = 21 four, so twenty banks carry twice
// the pairs of the rest; at q = 8 one, so all rows share the banks of their
// first 8 floats.
constexpr int energy_pitch(int Q) {
  constexpr long long kLdsCU = 160 * 1024;
  const long long wg_cap = 32 / (energy_threads(Q) / 64);  // 32 waves of a CU
  auto wgs = [wg_cap](long long bytes) { return kLdsCU / bytes < wg_cap ? kLdsCU / bytes : wg_cap; };
  const long long wg0 = wgs(2LL * Q * 16 * Q * 4);
  int best = 16 * Q;
  long long best_mx = -1, best_sq = 0;
  for (int pad = 0; pad <= 12; pad += 4) {
    const int P = 16 * Q + pad;
    if (wgs(2LL * Q * P * 4) < wg0) continue;
    int cnt[64] = {};
    for (int a = 0; a < Q; ++a)
      for (int b = 0; b < Q; ++b) ++cnt[(P * a + b) % 64];
    long long mx = 0, sq = 0;
    for (int k = 0; k < 64; ++k) {
      mx = cnt[k] > mx ? cnt[k] : mx;
      sq += (long long)cnt[k] * cnt[k];
    }
    if (best_mx < 0 || mx < best_mx || (mx == best_mx && sq < best_sq)) {
      best = P;
      best_mx = mx;
      best_sq = sq;
    }
  }
  return best;
}

// Row sites of chunk jc that pair with some j > i in the chunk.
__host__ __device__ inline int energy_rows(int jc, int L) {
  return min(jc * kEJC + kEJC - 1, L - 1);
}

EnergyPlan plan_energy(int64_t B, int L, int q) {
  (void)q;
  EnergyPlan p{};
  p.Bpad = ceil_div(std::max<int64_t>(B, 1), 64) * 64;
  p.steps = 0;
  for (int jc = 0; jc * kEJC < L; ++jc) p.steps += energy_rows(jc, L);
  p.parts = p.steps == 0 ? 0 : (int)std::min<int64_t>(128, std::max<int64_t>(1, p.steps / 32));
  size_t o = 0;
  p.off_xt = o;   o = align256(o + (size_t)L * p.Bpad);
  p.off_part = o; o = align256(o + sizeof(double) * (size_t)p.parts * p.Bpad);
  p.total = o;
  return p;
}

template <int Q>
__global__ __launch_bounds__(energy_threads(Q)) void k_energy_pairs(const float* __restrict__ J,
                                                            const int8_t* __restrict__ XT,
                                                            int64_t Bpad, int64_t B, int L,
                                                            int64_t steps, int parts,
                                                            double* __restrict__ part,
                                                            const int64_t* __restrict__ count) {
  constexpr int kEThreads = energy_threads(Q);
  constexpr int kESeqBlock = kEThreads * kESeq;  // sequences per workgroup
  if (count && *count < B) B = *count;  // live sequences of a launch sized for B
  if ((int64_t)blockIdx.x * kESeqBlock >= B) return;  // whole workgroup, before any barrier
  constexpr int kW = kEJC * Q;                                 // tile row length (16 Q floats)
  constexpr int kP = energy_pitch(Q);                          // its pitch in LDS
  constexpr int kRowQ = kW / 4;                                // 16-byte quads per tile row
  constexpr int kQuads = Q * kRowQ;                            // quads per tile
  constexpr int kNQ = (kQuads + kEThreads - 1) / kEThreads;    // tile quads per thread
  typedef float f4 __attribute__((ext_vector_type(4)));
  __shared__ __attribute__((aligned(16))) float tile[2][Q * kP];
  const int tid = threadIdx.x;
  const int p = blockIdx.y;
  const int64_t t0 = steps * p / parts, t1 = steps * (p + 1) / parts;
  const int Lq = L * Q;
  const int64_t b0 = (int64_t)blockIdx.x * kESeqBlock;  // first sequence of the workgroup
  int64_t bs[kESeq];
#pragma unroll
  for (int k = 0; k < kESeq; ++k) bs[k] = b0 + tid + kEThreads * k;

  // (jc, i) of step t0
  int jc = 0;
  int64_t r = t0;
  while (r >= energy_rows(jc, L)) {
    r -= energy_rows(jc, L);
    ++jc;
  }
  int i = (int)r;

  // Tokens of a site through a buffer resource over the workgroup's part of
  // that site's row of XT [L][Bpad] (64-bit base, at most Bpad - b0 bytes,
  // under 2^31): reads past the row (sequences beyond Bpad) return 0,
  // padding rows hold -1 (read as 0).
  auto site_rsrc = [&](int site) {
    const int64_t left = Bpad - b0;  // > 0: b0 < B <= Bpad
    return __builtin_amdgcn_make_buffer_rsrc(
        (void*)(XT + (size_t)site * Bpad + b0), (short)0,
        (int)std::min<int64_t>(left, 0x7FFFFFFF), 0x00020000);
  };
  auto tok_in = [&](__amdgpu_buffer_rsrc_t rs, int k) -> int {
    const int t = (int)(int8_t)__builtin_amdgcn_raw_buffer_load_b8(rs, tid + kEThreads * k, 0, 0);
    return t < 0 ? 0 : t;  // invalid tokens were flagged by the transpose
  };
  // Tile (ti, tjc): rows (ti Q + a), columns tjc kW + c of J, as 16-byte
  // quads; quad e = a kRowQ + c4 of the tile comes from float
  // a Lq + 4 c4 past the tile's corner (32-bit offsets fixed per thread).
  // Columns past the last site (partial last chunk) bring values of the next
  // row, or zeros past the end of J: lookups never read them.
  uint32_t qoff[kNQ];
#pragma unroll
  for (int n = 0; n < kNQ; ++n) {
    const int e = tid + kEThreads * n;
    qoff[n] = (uint32_t)((e / kRowQ) * Lq + 4 * (e % kRowQ)) * 4u;
  }
  const size_t jbytes = (size_t)Lq * Lq * sizeof(float);  // up to 2^32 (L 1024, q 32)
  auto load_tile = [&](f4(&v)[kNQ], int ti, int tjc) {
    // a resource from the tile's corner to the end of J, at most 2^31 - 1
    // bytes (a tile spans under q Lq 4 + 16 q 4 bytes, far less)
    const size_t corner = ((size_t)ti * Q * Lq + (size_t)tjc * kW) * sizeof(float);
    const __amdgpu_buffer_rsrc_t rj = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(reinterpret_cast<const char*>(J) + corner), (short)0,
        (int)std::min<size_t>(jbytes - corner, 0x7FFFFFFF), 0x00020000);
#pragma unroll
    for (int n = 0; n < kNQ; ++n) {
      if (tid + kEThreads * n < kQuads) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b128(rj, (int)qoff[n], 0, 0);
        v[n] = f4{__uint_as_float(w[0]), __uint_as_float(w[1]), __uint_as_float(w[2]),
                  __uint_as_float(w[3])};
      }
    }
  };
  auto store_tile = [&](const f4(&v)[kNQ], int buf) {
#pragma unroll
    for (int n = 0; n < kNQ; ++n) {
      const int e = tid + kEThreads * n;
      if (e < kQuads)
        *reinterpret_cast<f4*>(&tile[buf][(e / kRowQ) * kP + 4 * (e % kRowQ)]) = v[n];
    }
  };
  auto advance = [&](int& ii, int& jj) {
    if (++ii >= energy_rows(jj, L)) {
      ii = 0;
      ++jj;
    }
  };

  double acc[kESeq];
#pragma unroll
  for (int k = 0; k < kESeq; ++k) acc[k] = 0.0;
  int sj[kESeq][kEJC];
  auto load_chunk = [&](int cjc) {
#pragma unroll
    for (int jj = 0; jj < kEJC; ++jj) {
      const int j = cjc * kEJC + jj;
      const __amdgpu_buffer_rsrc_t rs = site_rsrc(min(j, L - 1));
#pragma unroll
      for (int k = 0; k < kESeq; ++k) sj[k][jj] = (j < L) ? tok_in(rs, k) : 0;
    }
  };
  auto row_tokens = [&](int(&s)[kESeq], int site) {
    const __amdgpu_buffer_rsrc_t rs = site_rsrc(site);
#pragma unroll
    for (int k = 0; k < kESeq; ++k) s[k] = tok_in(rs, k) * kP;
  };
  // The lookups of one step (row site si_, chunk cjc, LDS buffer buf): the
  // step's terms summed in FP32 in column order, then added to the FP64 sum.
  auto lookups = [&](int si_, int cjc, const int(&srow)[kESeq], int buf) {
    const float* tb = tile[buf];
    float sf[kESeq];
#pragma unroll
    for (int k = 0; k < kESeq; ++k) sf[k] = 0.0f;
    // for q <= 8 a step whose columns all pair with the row site skips the
    // per-column tests (q = 5: 11% shorter; for larger q the tests cost
    // nothing and the second copy of the loop 1-4%)
    if (Q <= 8 && cjc * kEJC > si_ && cjc * kEJC + kEJC <= L) {
#pragma unroll
      for (int jj = 0; jj < kEJC; ++jj)
#pragma unroll
        for (int k = 0; k < kESeq; ++k) sf[k] += tb[srow[k] + jj * Q + sj[k][jj]];
    } else {
#pragma unroll
      for (int jj = 0; jj < kEJC; ++jj) {
        const int j = cjc * kEJC + jj;
        if (j > si_ && j < L) {  // uniform over the workgroup
#pragma unroll
          for (int k = 0; k < kESeq; ++k) sf[k] += tb[srow[k] + jj * Q + sj[k][jj]];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kESeq; ++k) acc[k] += (double)sf[k];
  };

  // The tile of step t + 1 is fetched into registers during step t and
  // stored to LDS buffer (t + 1 - t0) % 2 at its end; the row tokens of step
  // t + 2 are fetched during step t into the registers of t's parity (A: even
  // offsets from t0, B: odd), so the lookups never wait on a load issued in
  // their own step and no register copy waits for one.
  f4 v[kNQ];
  int sA[kESeq], sB[kESeq];
  int iA = i, jA = jc, iB = i, jB = jc;
  advance(iB, jB);
  if (t0 < t1) {
    load_tile(v, iA, jA);
    store_tile(v, 0);
    load_chunk(jA);
    row_tokens(sA, iA);
  }
  if (t0 + 1 < t1) {
    row_tokens(sB, iB);
  }
  __syncthreads();
  for (int64_t t = t0; t < t1; t += 2) {
    // ---- step t (A)
    int iC = iB, jC = jB;  // step t + 2
    advance(iC, jC);
    if (t + 1 < t1) load_tile(v, iB, jB);
    lookups(iA, jA, sA, 0);
    if (t + 2 < t1) {
      row_tokens(sA, iC);
    }
    if (t + 1 < t1) {
      store_tile(v, 1);
      if (jB != jA) load_chunk(jB);
    }
    __syncthreads();
    if (t + 1 >= t1) break;
    // ---- step t + 1 (B)
    int iD = iC, jD = jC;  // step t + 3
    advance(iD, jD);
    if (t + 2 < t1) load_tile(v, iC, jC);
    lookups(iB, jB, sB, 1);
    if (t + 3 < t1) {
      row_tokens(sB, iD);
    }
    if (t + 2 < t1) {
      store_tile(v, 0);
      if (jC != jB) load_chunk(jC);
    }
    __syncthreads();
    iA = iC;
    jA = jC;
    iB = iD;
    jB = jD;
  }
#pragma unroll
  for (int k = 0; k < kESeq; ++k)
    if (bs[k] < B) part[(size_t)p * Bpad + bs[k]] = acc[k];
}

__global__ void k_energy_finish(const float* __restrict__ h, const int8_t* __restrict__ XT,
                                int64_t Bpad, int64_t B, int L, int q, int parts,
                                const double* __restrict__ part, float* __restrict__ E,
                                const int64_t* __restrict__ count) {
  if (count && *count < B) B = *count;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  // loads in batches of 16 (tokens, then their fields; then partial sums),
  // subtractions in site order, then in range order
  double acc = 0.0;
  int i = 0;
  for (; i + 16 <= L; i += 16) {
    int t[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) t[u] = XT[(size_t)(i + u) * Bpad + b];
    float hv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) hv[u] = h[(i + u) * q + (t[u] < 0 ? 0 : t[u])];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc -= (double)hv[u];
  }
  for (; i < L; ++i) {
    int t = XT[(size_t)i * Bpad + b];
    if (t < 0) t = 0;
    acc -= (double)h[i * q + t];
  }
  int p = 0;
  for (; p + 16 <= parts; p += 16) {
    double pv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) pv[u] = part[(size_t)(p + u) * Bpad + b];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc -= pv[u];
  }
  for (; p < parts; ++p) acc -= part[(size_t)p * Bpad + b];
  E[b] = (float)acc;
}

template <int Q>
static void launch_energy_q(const float* J, const int8_t* XT, int64_t B, int L,
                            const EnergyPlan& plan, double* part, hipStream_t s,
                            const int64_t* count) {
  const dim3 grid((unsigned)ceil_div(B, energy_threads(Q) * kESeq), (unsigned)plan.parts);
  hipLaunchKernelGGL(k_energy_pairs<Q>, grid, dim3(energy_threads(Q)), 0, s, J, XT, plan.Bpad, B, L,
                     plan.steps, plan.parts, part, count);
}

hipError_t launch_energy(const float* h, const float* J, const int8_t* seqs, int64_t B, int L,
                         int q, float* E, const EnergyPlan& plan, void* ws, int32_t* dev_err,
                         hipStream_t s, const int64_t* count) {
  char* base = static_cast<char*>(ws);
  int8_t* XT = reinterpret_cast<int8_t*>(base + plan.off_xt);
  double* part = reinterpret_cast<double*>(base + plan.off_part);
  hipError_t e = launch_transpose_tokens(seqs, B, L, q, XT, plan.Bpad, dev_err, s, count);
  if (e != hipSuccess) return e;
  if (plan.parts > 0) {
    switch (q) {
#define BMDCA_EQ(n)                                        \
  case n:                                                  \
    launch_energy_q<n>(J, XT, B, L, plan, part, s, count); \
    break;
      BMDCA_EQ(2) BMDCA_EQ(3) BMDCA_EQ(4) BMDCA_EQ(5) BMDCA_EQ(6) BMDCA_EQ(7) BMDCA_EQ(8)
      BMDCA_EQ(9) BMDCA_EQ(10) BMDCA_EQ(11) BMDCA_EQ(12) BMDCA_EQ(13) BMDCA_EQ(14) BMDCA_EQ(15)
      BMDCA_EQ(16) BMDCA_EQ(17) BMDCA_EQ(18) BMDCA_EQ(19) BMDCA_EQ(20) BMDCA_EQ(21) BMDCA_EQ(22)
      BMDCA_EQ(23) BMDCA_EQ(24) BMDCA_EQ(25) BMDCA_EQ(26) BMDCA_EQ(27) BMDCA_EQ(28) BMDCA_EQ(29)
      BMDCA_EQ(30) BMDCA_EQ(31) BMDCA_EQ(32)
#undef BMDCA_EQ
      default:
        return hipErrorInvalidValue;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_energy_finish, dim3((unsigned)ceil_div(B, 256)), dim3(256), 0, s, h, XT,
                     plan.Bpad, B, L, q, plan.parts, part, E, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Single mutants: dE[b][i*q+a] = -(H[b][i*q+a] - H[b][i*q+wt_i]), with H the
// wild type's local fields (h + sum_{j != i} J_ij(., wt_j)).
// ---------------------------------------------------------------------------
__global__ void k_mutant_delta(const float* __restrict__ H, const int8_t* __restrict__ wt,
                               int64_t B, int L, int q, float* __restrict__ dE,
                               const int64_t* __restrict__ count) {
  if (count && *count < B) B = *count;
  const int64_t Lq = (int64_t)L * q;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * Lq) return;
  const int64_t b = idx / Lq;
  const int r = (int)(idx % Lq);
  const int i = r / q;
  int w = wt[b * L + i];
  if (w < 0 || w >= q) w = 0;  // flagged by the field build
  const float* Hb = H + b * Lq;
  dE[idx] = (r == i * q + w) ? 0.0f : -(Hb[r] - Hb[i * q + w]);
}

hipError_t launch_mutant_delta(const float* H, const int8_t* wt, int64_t B, int L, int q,
                               float* dE, hipStream_t s, const int64_t* count) {
  const int64_t total = B * (int64_t)L * q;
  hipLaunchKernelGGL(k_mutant_delta, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, H, wt,
                     B, L, q, dE, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// APC Frobenius.  k_frob_blocks: each wave takes 64 / q blocks (i, j), j > i,
// of one block-row i; lane (block, t) owns row t and column t of its block,
// both held in registers: the row by 16-byte loads, the column by 4-byte
// loads that are coalesced over the block's lanes (and hit the cache lines
// the row loads brought in).  In FP64 the lane forms the row mean r_t and the
// column mean c_t over all q states; the column means go through LDS, every
// lane of the block reads all q of them and their mean m, and sums the
// squares of the gauged entries J_tb - r_t - c_b + m of its row with
// t, b != gap; one lane per block adds the q row sums in order, and
// F_ij = F_ji = the square root.  Block-rows i and L - 1 - i share a run of
// wave tasks (L - 1 blocks between them), so every run is as long.  J is read
// once, without LDS staging.  k_apc_rows: S_i = sum_k F_ik (one wave per
// row); k_apc_total: S = sum_i S_i; k_apc_out: F_apc = F - S_i S_j / S,
// diagonals 0 (the diagonal of F is never read).
// ---------------------------------------------------------------------------
size_t apc_ws_bytes(int L) { return align256(sizeof(double) * ((size_t)L * L + L + 8)); }

// Wave tasks per pair of block-rows (p, L - 1 - p): ceil((L - 1 - p) / bpw)
// tasks of row p and ceil(p / bpw) of row L - 1 - p, at most this many.
inline int frob_tasks_per_pair(int L, int q) { return (int)ceil_div(L - 1, 64 / q) + 1; }

// QP4: quads per block row, ceil(q / 4).
template <int QP4>
__global__ __launch_bounds__(256) void k_frob_blocks(const float* __restrict__ J, int L, int q,
                                                     int gap, int tpp, double* __restrict__ F) {
  constexpr int QB = 4 * QP4;  // columns a lane walks (q rounded up to quads)
  __shared__ double cmean[4][64];  // per wave: c_t of lane (block, t) at block * q + t
  __shared__ double rowss[4][64];  // per wave: the lanes' sums of squares
  const int lane = threadIdx.x % 64;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);  // wave-uniform, as is the wave task below
  const int task = (int)blockIdx.x * 4 + wv;  // below 2^19 (L <= 1024, tpp <= 1024)
  const int npair = (L + 1) / 2;
  if (task >= npair * tpp) return;  // whole wave; only wave barriers below
  const int p = task / tpp, k = task - (task / tpp) * tpp;
  const int bpw = 64 / q;
  const int i0 = p, i1 = L - 1 - p;
  const int n0 = (int)ceil_div(L - 1 - i0, bpw);  // tasks of row i0
  int i, jfirst;
  if (k < n0) {
    i = i0;
    jfirst = i0 + 1 + k * bpw;
  } else {
    if (i1 == i0) return;  // the middle row of an odd L has no partner
    i = i1;
    jfirst = i1 + 1 + (k - n0) * bpw;
    if (jfirst >= L) return;
  }
  const int jb = lane / q, t = lane - jb * q;
  const bool live = jb < bpw && jfirst + jb < L;
  const int j = live ? jfirst + jb : i;  // dead lanes read block (i, i): in bounds, unused
  const int Lq = L * q;
  // Block-row i as one buffer (q Lq floats, at most 4 MiB).  Row t of block
  // (i, j) starts at float t Lq + j q; the quads past its q-th float read the
  // next block (or, past the buffer, zeros) and are cleared.
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(J + (size_t)i * q * Lq), (short)0, (int)((size_t)q * Lq * sizeof(float)), 0x00020000);
  const int rowoff = (t * Lq + j * q) * (int)sizeof(float);
  double x[QB];
#pragma unroll
  for (int u = 0; u < QP4; ++u) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, rowoff + 16 * u, 0, 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) x[4 * u + e] = (double)__uint_as_float(v[e]);
  }
  float y[QB];
#pragma unroll
  for (int a = 0; a < QB; ++a)
    y[a] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(
        rs, (min(a, q - 1) * Lq + j * q + t) * (int)sizeof(float), 0, 0));
  // entries past q (compile-time positions in the last quad) become +0, which
  // leaves every sum below unchanged (a sum that starts at +0 never is -0)
#pragma unroll
  for (int b = 4 * (QP4 - 1); b < QB; ++b) {
    x[b] = (b < q) ? x[b] : 0.0;
    y[b] = (b < q) ? y[b] : 0.0f;
  }
  double rsum = 0.0, csum = 0.0;
#pragma unroll
  for (int b = 0; b < QB; ++b) {
    rsum += x[b];
    csum += (double)y[b];
  }
  const double r = rsum / (double)q;
  double* cm = cmean[wv];
  cm[lane] = csum / (double)q;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  const int base = min(jb, bpw - 1) * q;  // this lane's block in the wave's arrays
  double cb[QB];
  double all = 0.0;
#pragma unroll
  for (int b = 0; b < QB; ++b) {
    // the read is unconditional (a select around it becomes a branch); past q
    // it is scaled to +-0
    cb[b] = cm[base + min(b, q - 1)];
    if (b >= 4 * (QP4 - 1)) cb[b] *= (b < q) ? 1.0 : 0.0;
    all += cb[b];
  }
  const double m = all / (double)q;
  double ss = 0.0;
#pragma unroll
  for (int b = 0; b < QB; ++b) {
    const double w = (b < q && b != gap) ? 1.0 : 0.0;  // uniform per b
    const double z = ((x[b] - r) - cb[b]) + m;
    ss = __builtin_fma(z * w, z, ss);  // +-0 for the skipped columns: ss unchanged
  }
  double* rss = rowss[wv];
  rss[lane] = (t == gap) ? 0.0 : ss;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  if (live && t == 0) {
    double tot = 0.0;
    for (int u = 0; u < q; ++u) tot += rss[base + u];
    const double f = sqrt(tot);
    F[(size_t)i * L + j] = f;
    F[(size_t)j * L + i] = f;
  }
}

__global__ __launch_bounds__(256) void k_apc_rows(const double* __restrict__ F, int L,
                                                  double* __restrict__ S) {
  const int lane = threadIdx.x % 64;
  const int i = blockIdx.x * 4 + threadIdx.x / 64;
  if (i >= L) return;
  double s = 0.0;
  for (int k = lane; k < L; k += 64) s += (k == i) ? 0.0 : F[(size_t)i * L + k];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) S[i] = s;
}

// S = sum_i S_i: thread t adds S_t, S_{t+256}, ... in ascending order, then a
// fixed tree over the 256 partial sums (one workgroup, deterministic).
__global__ __launch_bounds__(256) void k_apc_total(double* __restrict__ S, int L) {
  __shared__ double part[256];
  double tot = 0.0;
  for (int i = threadIdx.x; i < L; i += 256) tot += S[i];
  part[threadIdx.x] = tot;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) S[L] = part[0];
}

__global__ void k_apc_out(const double* __restrict__ F, const double* __restrict__ S, int L,
                          float* __restrict__ Fout, float* __restrict__ Fapc) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (size_t)L * L) return;
  const int i = (int)(k / L), j = (int)(k % L);
  const double f = (i == j) ? 0.0 : F[k];
  if (Fout) Fout[k] = (float)f;
  Fapc[k] = (i == j) ? 0.0f : (float)(f - S[i] * S[j] / S[L]);
}

hipError_t launch_apc(const float* J, int L, int q, int gap, float* F, float* Fapc, void* ws,
                      hipStream_t s) {
  double* Fd = static_cast<double*>(ws);
  double* S = Fd + (size_t)L * L;
  const int tpp = frob_tasks_per_pair(L, q);
  const unsigned nwg = (unsigned)ceil_div((int64_t)((L + 1) / 2) * tpp, 4);
  switch ((q + 3) / 4) {
#define BMDCA_FROB(QP4)                                                                     \
  case QP4:                                                                                 \
    hipLaunchKernelGGL(k_frob_blocks<QP4>, dim3(nwg), dim3(256), 0, s, J, L, q, gap, tpp, Fd); \
    break;
    BMDCA_FROB(1) BMDCA_FROB(2) BMDCA_FROB(3) BMDCA_FROB(4)
    BMDCA_FROB(5) BMDCA_FROB(6) BMDCA_FROB(7) BMDCA_FROB(8)
#undef BMDCA_FROB
    default:
      return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(k_apc_rows, dim3((unsigned)ceil_div(L, 4)), dim3(256), 0, s, Fd, L, S);
  hipLaunchKernelGGL(k_apc_total, dim3(1), dim3(256), 0, s, S, L);
  hipLaunchKernelGGL(k_apc_out, dim3((unsigned)ceil_div((size_t)L * L, (size_t)256)), dim3(256), 0,
                     s, Fd, S, L, F, Fapc);
  return hipGetLastError();
}

}  // namespace bmdca
