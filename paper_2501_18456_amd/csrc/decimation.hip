// Element decimation (edDCA; adabmDCA 2.0, Sec. 2.2, options in Sec. 3.2): one graph update
// removes the active coupling elements whose removal changes the model least.
// For the element J_ij(a,b) with pairwise model marginal p (chain frequency),
// the symmetric Kullback-Leibler distance between the model and the model
// without that element follows from Eq. (1):
//   p' = p e^-J / (1 - p + p e^-J),   D = J (p - p') >= 0.
// The k smallest (D, r1 Lq + r2) over active elements r1 < r2 are removed
// (mask and J zeroed on both triangles), k = min(max(1, floor(drate n_act)),
// n_act - ceil(density n_total)).
//
// Selection is an exact radix select on 64-bit keys (the IEEE bits of D >= 0
// order like the values): eight passes of 8-bit digit histograms narrow the
// key of the k-th smallest element; ties at that key are taken in index
// order with a block-level scan.  Everything after the counts stays on the
// device.
//
// Element activation (eaDCA; Sec. 2.2, options in Sec. 3.1) shares the selection: every element
// (r1 < r2, different sites), active or not, is scored by how far the model
// marginal p is from the data's f, taken as the Kullback-Leibler divergence
// of the two Bernoulli laws of [s_i == a][s_j == b],
//   D = f log(f/p) + (1-f) log((1-f)/(1-p))   (0 log 0 = 0, +inf where the
//   data has mass the model lacks),
// and the k = max(1, floor(factivate n_inactive)) largest (D, then smallest
// r1 Lq + r2) are set active; the ones already active add nothing.  Keys
// 0x7FF0000000000000 - bits(D) order the largest D first.
#include "common.hpp"
#include "internal.hpp"

namespace bmdca {

constexpr uint64_t kNoKey = ~0ull;
constexpr int kDecThreads = 256;

// Select state (device): [0] prefix of the k-th key found so far, [1] its
// mask of decided bits, [2] rank still to find inside the prefix, [3] k,
// [4] n_act, [5] count of keys below the final key, [6] ties to take, [7]
// elements newly set active (activation).
struct DecState {
  unsigned long long prefix, pmask, rank, k, n_act, below, ties, added;
};
constexpr unsigned long long kActTop = 0x7FF0000000000000ull;  // bits of +inf

__global__ __launch_bounds__(kDecThreads) void k_dec_keys(const float* __restrict__ J,
                                                          const uint8_t* __restrict__ mask,
                                                          const double* __restrict__ C, int64_t N,
                                                          int L, int q,
                                                          unsigned long long* __restrict__ keys,
                                                          unsigned long long* __restrict__ n_act) {
  __shared__ unsigned long long sh[kDecThreads / 64];
  const int Lq = L * q;
  const size_t total = (size_t)Lq * Lq;
  unsigned long long cnt = 0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int r1 = (int)(e / Lq), r2 = (int)(e % Lq);
    uint64_t key = kNoKey;
    if (r1 < r2 && r1 / q != r2 / q && mask[e]) {
      const double p = C[e] / (double)N;
      const double Jv = (double)J[e];
      const double ex = exp(-Jv);
      const double d = 1.0 - p + p * ex;
      const double pp = p * ex / d;
      const double D = Jv * (p - pp);
      key = (uint64_t)__double_as_longlong(D > 0.0 ? D : 0.0);
      ++cnt;
    }
    keys[e] = key;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int w = 0; w < kDecThreads / 64; ++w) s += sh[w];
    if (s) atomicAdd(n_act, s);
  }
}

// k from the active count and the targets; rank = k (1-based k-th smallest).
__global__ void k_dec_init(DecState* st, double drate, int64_t n_target) {
  if (threadIdx.x != 0) return;
  const int64_t n_act = (int64_t)st->n_act;
  int64_t k = 0;
  if (n_act > n_target) {
    k = (int64_t)floor(drate * (double)n_act);
    if (k < 1) k = 1;
    if (k > n_act - n_target) k = n_act - n_target;
  }
  st->k = (unsigned long long)k;
  st->rank = (unsigned long long)k;
  st->prefix = 0;
  st->pmask = 0;
  st->below = 0;
  st->ties = 0;
}

__global__ __launch_bounds__(kDecThreads) void k_act_keys(const uint8_t* __restrict__ mask,
                                                          const double* __restrict__ C,
                                                          const double* __restrict__ f2, int64_t N,
                                                          int L, int q,
                                                          unsigned long long* __restrict__ keys,
                                                          unsigned long long* __restrict__ n_act,
                                                          int32_t* dev_err) {
  __shared__ unsigned long long sh[kDecThreads / 64];
  const int Lq = L * q;
  const size_t total = (size_t)Lq * Lq;
  unsigned long long cnt = 0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int r1 = (int)(e / Lq), r2 = (int)(e % Lq);
    uint64_t key = kNoKey;
    if (r1 < r2 && r1 / q != r2 / q) {
      const double p = C[e] / (double)N;
      const double f = f2[e];
      double D = 0.0;
      if (f >= 0.0 && f <= 1.0) {
        if (f > 0.0) D += (p > 0.0) ? f * log(f / p) : INFINITY;
        if (f < 1.0) D += (p < 1.0) ? (1.0 - f) * log((1.0 - f) / (1.0 - p)) : INFINITY;
        if (!(D > 0.0)) D = 0.0;
      } else if (dev_err) {
        atomicOr(dev_err, 2);  // a data frequency outside [0, 1]: scored 0
      }
      key = kActTop - (uint64_t)__double_as_longlong(D);
      if (mask[e]) ++cnt;
    }
    keys[e] = key;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int w = 0; w < kDecThreads / 64; ++w) s += sh[w];
    if (s) atomicAdd(n_act, s);
  }
}

// Activation count: k = max(1, floor(factivate n_inactive)), 0 when every
// element is active.
__global__ void k_act_init(DecState* st, double factivate, int64_t n_total) {
  if (threadIdx.x != 0) return;
  const int64_t n_inact = n_total - (int64_t)st->n_act;
  int64_t k = 0;
  if (n_inact > 0) {
    k = (int64_t)floor(factivate * (double)n_inact);
    if (k < 1) k = 1;
  }
  st->k = (unsigned long long)k;
  st->rank = (unsigned long long)k;
  st->prefix = 0;
  st->pmask = 0;
  st->below = 0;
  st->ties = 0;
  st->added = 0;
}

__global__ void k_dec_zero(unsigned long long* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

// Histogram of digit `shift` over the keys that match the decided prefix.
__global__ __launch_bounds__(kDecThreads) void k_dec_hist(const unsigned long long* __restrict__ keys,
                                                          size_t total, const DecState* st,
                                                          int shift,
                                                          unsigned long long* __restrict__ hist) {
  __shared__ unsigned int h[256];
  if (st->k == 0) return;
  for (int b = threadIdx.x; b < 256; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const unsigned long long pm = st->pmask, pf = st->prefix;
  const int lane = threadIdx.x & 63;
  // The keys of one pass mostly share a digit (positive doubles in a narrow
  // range), so the lanes of a wave are grouped by digit with ballots and one
  // lane per group adds the group's count: one LDS atomic per distinct digit
  // in the wave instead of one per key.
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e0 = (size_t)blockIdx.x * blockDim.x; e0 < total; e0 += stride) {
    const size_t e = e0 + threadIdx.x;
    const unsigned long long key = e < total ? keys[e] : kNoKey;
    const bool valid = key != kNoKey && (key & pm) == pf;
    const int bin = valid ? (int)((key >> shift) & 255) : -1;
    unsigned long long todo = __ballot(valid);  // wave-uniform
    while (todo) {
      const int leader = __ffsll((long long)todo) - 1;
      const int lb = __shfl(bin, leader, 64);
      const unsigned long long same = __ballot(bin == lb) & todo;
      if (lane == leader) atomicAdd(&h[lb], (unsigned int)__popcll(same));
      todo &= ~same;
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < 256; b += blockDim.x)
    if (h[b]) atomicAdd(hist + b, (unsigned long long)h[b]);
}

// Fix digit `shift`: the bin where the running count reaches the rank.
__global__ void k_dec_pick(DecState* st, int shift, const unsigned long long* __restrict__ hist) {
  if (threadIdx.x != 0 || st->k == 0) return;
  unsigned long long run = 0;
  int b = 0;
  for (; b < 256; ++b) {
    if (run + hist[b] >= st->rank) break;
    run += hist[b];
  }
  st->rank -= run;
  st->below += run;
  st->prefix |= (unsigned long long)b << shift;
  st->pmask |= 255ull << shift;
}

// After the last digit: `below` counts keys < x inside the matching prefix
// only at each level, which adds up to all keys < x; ties = k - below.
__global__ void k_dec_finish(DecState* st) {
  if (threadIdx.x != 0 || st->k == 0) return;
  st->ties = st->k - st->below;
}

// Per-block count of keys equal to x.
__global__ __launch_bounds__(kDecThreads) void k_dec_tie_count(const unsigned long long* __restrict__ keys,
                                                               size_t total, const DecState* st,
                                                               unsigned long long* __restrict__ blk) {
  __shared__ unsigned long long sh[kDecThreads / 64];
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long c = 0;
  if (st->k != 0 && e < total && keys[e] == st->prefix) c = 1;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int w = 0; w < kDecThreads / 64; ++w) s += sh[w];
    blk[blockIdx.x] = s;
  }
}

// Exclusive scan of the block tie counts in block order (one workgroup:
// each thread sums a contiguous segment, the segment sums are scanned in LDS,
// then each thread writes its segment's running counts; exact integers).
constexpr int kDecScanThreads = 1024;
__global__ __launch_bounds__(kDecScanThreads) void k_dec_tie_scan(unsigned long long* __restrict__ blk,
                                                                  int64_t nblk) {
  __shared__ unsigned long long part[kDecScanThreads];
  const int t = threadIdx.x;
  const int64_t per = (nblk + kDecScanThreads - 1) / kDecScanThreads;
  const int64_t b0 = std::min<int64_t>(nblk, (int64_t)t * per);
  const int64_t b1 = std::min<int64_t>(nblk, b0 + per);
  unsigned long long sum = 0;
  for (int64_t b = b0; b < b1; ++b) sum += blk[b];
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < kDecScanThreads; o <<= 1) {  // inclusive scan of the segment sums
    const unsigned long long v = t >= o ? part[t - o] : 0ull;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  unsigned long long run = t > 0 ? part[t - 1] : 0ull;
  for (int64_t b = b0; b < b1; ++b) {
    const unsigned long long c = blk[b];
    blk[b] = run;
    run += c;
  }
}

// Take keys < x, and keys == x whose index-order rank is below `ties`:
// ACT = false removes them (mask and J zeroed on both triangles), ACT = true
// sets them active (mask on both triangles) and counts the ones that were not.
template <bool ACT>
__global__ __launch_bounds__(kDecThreads) void k_sel_apply(const unsigned long long* __restrict__ keys,
                                                           size_t total, int Lq, DecState* st,
                                                           const unsigned long long* __restrict__ blk,
                                                           float* __restrict__ J,
                                                           uint8_t* __restrict__ mask) {
  __shared__ unsigned int tie_prefix[kDecThreads];
  __shared__ unsigned int added[kDecThreads / 64];
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (st->k == 0) return;  // the same for the whole grid
  const unsigned long long x = st->prefix;
  const unsigned long long key = (e < total) ? keys[e] : kNoKey;
  const unsigned int tie = (key == x) ? 1u : 0u;
  // inclusive scan of ties inside the block (index order)
  tie_prefix[threadIdx.x] = tie;
  __syncthreads();
  for (int o = 1; o < kDecThreads; o <<= 1) {
    const unsigned int v = threadIdx.x >= o ? tie_prefix[threadIdx.x - o] : 0u;
    __syncthreads();
    tie_prefix[threadIdx.x] += v;
    __syncthreads();
  }
  bool take = key < x;
  if (tie) take = (blk[blockIdx.x] + tie_prefix[threadIdx.x] - 1) < st->ties;
  bool fresh = false;
  if (take && key != kNoKey) {
    const int r1 = (int)(e / Lq), r2 = (int)(e % Lq);
    if constexpr (ACT) {
      fresh = mask[e] == 0;
      mask[e] = 1;
      mask[(size_t)r2 * Lq + r1] = 1;
    } else {
      mask[e] = 0;
      mask[(size_t)r2 * Lq + r1] = 0;
      J[e] = 0.0f;
      J[(size_t)r2 * Lq + r1] = 0.0f;
    }
  }
  if constexpr (ACT) {
    const unsigned long long b = __ballot(fresh);
    if ((threadIdx.x & 63) == 0) added[threadIdx.x >> 6] = (unsigned int)__popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long n = 0;
      for (int w = 0; w < kDecThreads / 64; ++w) n += added[w];
      if (n) atomicAdd(&st->added, n);
    }
  }
}

__global__ void k_dec_out(const DecState* st, long long* n_active_out) {
  if (threadIdx.x == 0) *n_active_out = (long long)(st->n_act - st->k);
}

__global__ void k_act_out(const DecState* st, long long* n_active_out) {
  if (threadIdx.x == 0) *n_active_out = (long long)(st->n_act + st->added);
}

size_t dec_ws_bytes(int L, int q) {
  const size_t Lq = (size_t)L * q;
  return align256(sizeof(unsigned long long) * Lq * Lq) + align256(sizeof(DecState)) +
         align256(sizeof(unsigned long long) * 256) +
         align256(sizeof(unsigned long long) * ceil_div(Lq * Lq, (size_t)kDecThreads));
}

// Workspace carve-up shared by both graph updates.
struct SelBufs {
  unsigned long long* keys;
  DecState* st;
  unsigned long long* hist;
  unsigned long long* blk;
  size_t total;
  int64_t nblk;
  unsigned grid;
};

static SelBufs sel_bufs(int L, int q, void* ws) {
  SelBufs b{};
  const size_t Lq = (size_t)L * q;
  b.total = Lq * Lq;
  char* base = static_cast<char*>(ws);
  b.keys = reinterpret_cast<unsigned long long*>(base);
  base += align256(sizeof(unsigned long long) * b.total);
  b.st = reinterpret_cast<DecState*>(base);
  base += align256(sizeof(DecState));
  b.hist = reinterpret_cast<unsigned long long*>(base);
  base += align256(sizeof(unsigned long long) * 256);
  b.blk = reinterpret_cast<unsigned long long*>(base);
  b.nblk = (int64_t)ceil_div(b.total, (size_t)kDecThreads);
  // grid-stride kernels that end in global atomics on a few shared addresses
  // (the active count, the hot digits) get at most 512 workgroups: 8192 of
  // them made each pass wait ~0.1 ms on serialized atomics
  b.grid = (unsigned)std::min<size_t>(ceil_div(b.total, (size_t)kDecThreads), 512);
  return b;
}

// Radix select of the k-th smallest key (k in the state) and the tie ranks.
static void enqueue_select(const SelBufs& b, hipStream_t s) {
  for (int shift = 56; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(k_dec_zero, dim3(4), dim3(64), 0, s, b.hist, 256);
    hipLaunchKernelGGL(k_dec_hist, dim3(b.grid), dim3(kDecThreads), 0, s, b.keys, b.total, b.st,
                       shift, b.hist);
    hipLaunchKernelGGL(k_dec_pick, dim3(1), dim3(64), 0, s, b.st, shift, b.hist);
  }
  hipLaunchKernelGGL(k_dec_finish, dim3(1), dim3(64), 0, s, b.st);
  hipLaunchKernelGGL(k_dec_tie_count, dim3((unsigned)b.nblk), dim3(kDecThreads), 0, s, b.keys,
                     b.total, b.st, b.blk);
  hipLaunchKernelGGL(k_dec_tie_scan, dim3(1), dim3(kDecScanThreads), 0, s, b.blk, b.nblk);
}

hipError_t launch_decimate(float* J, uint8_t* mask, const double* C, int64_t N, int L, int q,
                           double drate, double density, long long* n_active_out, void* ws,
                           hipStream_t s) {
  const SelBufs b = sel_bufs(L, q, ws);
  const int64_t n_total = (int64_t)L * (L - 1) / 2 * q * q;
  const int64_t n_target = (int64_t)ceil(density * (double)n_total);
  hipLaunchKernelGGL(k_dec_zero, dim3(1), dim3(64), 0, s,
                     reinterpret_cast<unsigned long long*>(b.st), (int)(sizeof(DecState) / 8));
  hipLaunchKernelGGL(k_dec_keys, dim3(b.grid), dim3(kDecThreads), 0, s, J, mask, C, N, L, q,
                     b.keys, &b.st->n_act);
  hipLaunchKernelGGL(k_dec_init, dim3(1), dim3(64), 0, s, b.st, drate, n_target);
  enqueue_select(b, s);
  hipLaunchKernelGGL(k_sel_apply<false>, dim3((unsigned)b.nblk), dim3(kDecThreads), 0, s, b.keys,
                     b.total, L * q, b.st, b.blk, J, mask);
  if (n_active_out)
    hipLaunchKernelGGL(k_dec_out, dim3(1), dim3(64), 0, s, b.st, n_active_out);
  return hipGetLastError();
}

hipError_t launch_activate(uint8_t* mask, const double* C, const double* f2, int64_t N, int L,
                           int q, double factivate, long long* n_active_out, void* ws,
                           int32_t* dev_err, hipStream_t s) {
  const SelBufs b = sel_bufs(L, q, ws);
  const int64_t n_total = (int64_t)L * (L - 1) / 2 * q * q;
  hipLaunchKernelGGL(k_dec_zero, dim3(1), dim3(64), 0, s,
                     reinterpret_cast<unsigned long long*>(b.st), (int)(sizeof(DecState) / 8));
  hipLaunchKernelGGL(k_act_keys, dim3(b.grid), dim3(kDecThreads), 0, s, mask, C, f2, N, L, q,
                     b.keys, &b.st->n_act, dev_err);
  hipLaunchKernelGGL(k_act_init, dim3(1), dim3(64), 0, s, b.st, factivate, n_total);
  enqueue_select(b, s);
  hipLaunchKernelGGL(k_sel_apply<true>, dim3((unsigned)b.nblk), dim3(kDecThreads), 0, s, b.keys,
                     b.total, L * q, b.st, b.blk, nullptr, mask);
  if (n_active_out)
    hipLaunchKernelGGL(k_act_out, dim3(1), dim3(64), 0, s, b.st, n_active_out);
  return hipGetLastError();
}

}  // namespace bmdca

namespace bmdca {

// ----- coupling graphs as masks (Sec. 2.2): the fully connected graph of
// bmDCA, the empty graph eaDCA starts from, and the couplings of a graph.

// mask[r1][r2] = full && site(r1) != site(r2).
__global__ __launch_bounds__(kDecThreads) void k_mask_init(uint8_t* __restrict__ mask, int L,
                                                           int q, int full) {
  const int Lq = L * q;
  const size_t total = (size_t)Lq * Lq;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int r1 = (int)(e / Lq), r2 = (int)(e % Lq);
    mask[e] = (uint8_t)(full && r1 / q != r2 / q);
  }
}

__global__ void k_count_zero(unsigned long long* n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *n = 0;
}

// J = 0 where the element is inactive (mask 0 or a diagonal block); the
// active elements r1 < r2 are counted (integer atomics: exact in any order).
__global__ __launch_bounds__(kDecThreads) void k_mask_apply(float* __restrict__ J,
                                                            const uint8_t* __restrict__ mask,
                                                            int L, int q,
                                                            unsigned long long* __restrict__ n) {
  __shared__ unsigned long long sh[kDecThreads / 64];
  const int Lq = L * q;
  const size_t total = (size_t)Lq * Lq;
  unsigned long long cnt = 0;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int r1 = (int)(e / Lq), r2 = (int)(e % Lq);
    const bool on = mask[e] != 0 && r1 / q != r2 / q;
    if (!on && J) J[e] = 0.0f;
    cnt += (on && r1 < r2) ? 1ull : 0ull;
  }
  if (!n) return;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int w = 0; w < kDecThreads / 64; ++w) s += sh[w];
    if (s) atomicAdd(n, s);
  }
}

static unsigned mask_blocks(int L, int q) {
  const size_t total = (size_t)L * q * (size_t)L * q;
  return (unsigned)std::min<size_t>(ceil_div(total, kDecThreads), 2048);
}

hipError_t launch_mask_init(uint8_t* mask, int L, int q, int full, hipStream_t s) {
  hipLaunchKernelGGL(k_mask_init, dim3(mask_blocks(L, q)), dim3(kDecThreads), 0, s, mask, L, q,
                     full);
  return hipGetLastError();
}

hipError_t launch_mask_apply(float* J, const uint8_t* mask, int L, int q, long long* n_active,
                             hipStream_t s) {
  auto* n = reinterpret_cast<unsigned long long*>(n_active);
  if (n) {
    hipLaunchKernelGGL(k_count_zero, dim3(1), dim3(64), 0, s, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_mask_apply, dim3(mask_blocks(L, q)), dim3(kDecThreads), 0, s, J, mask, L,
                     q, n);
  return hipGetLastError();
}

}  // namespace bmdca
