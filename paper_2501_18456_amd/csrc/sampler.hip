// Persistent-chain Gibbs sampler of the Potts model of Eq. (1)
// (adabmDCA 2.0, Sec. 2.1, "Monte Carlo estimation of the gradient").
//
// Layout: chains int8 [N][L]; local fields H float32 [N][Lq] in HBM, one row
// per chain; couplings J float32 [Lq][Lq] full-symmetric, so the row of
// vertex (i, a) is one contiguous Lq vector and H can be kept current with two
// coalesced row reads per accepted change.
#include "common.hpp"
#include "gather_kernel.hpp"
#include "internal.hpp"

namespace bmdca {

// ---------------------------------------------------------------------------
// Uniform random initial chains: counter (i/4, 0, c, 1), word i%4,
// token = (word * q) >> 32.
// ---------------------------------------------------------------------------
__global__ void k_init_chains(int8_t* __restrict__ chains, int64_t N, int L, int q, uint32_t k0,
                              uint32_t k1) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= N * (int64_t)L) return;
  const int64_t c = idx / L;
  const int i = (int)(idx % L);
  const uint4 r = philox4x32_10(make_uint4((uint32_t)i >> 2, 0u, (uint32_t)c, 1u), k0, k1);
  const uint32_t w = pick_word(r, i & 3);
  chains[idx] = (int8_t)(((uint64_t)w * (uint64_t)q) >> 32);
}

hipError_t launch_init_chains(int8_t* chains, int64_t N, int L, int q, uint64_t seed,
                              hipStream_t s) {
  const int64_t total = N * (int64_t)L;
  const int bs = 256;
  hipLaunchKernelGGL(k_init_chains, dim3((unsigned)ceil_div(total, bs)), dim3(bs), 0, s, chains,
                     N, L, q, (uint32_t)seed, (uint32_t)(seed >> 32));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Local fields from scratch: H[c][r] = h[r] + sum_{k != site(r)} J[(k, s_k)][r],
// summed in FP32 in the order k = 0..L-1.  By the symmetry of J this equals
// h_j(b) + sum_{k != j} J_jk(b, s_k) for r = (j, b).
// Workgroups over (chain, column block): blocks of equal width, at most 1024
// columns; a thread owns four consecutive columns and reads them with one 16-byte load per coupling
// row, through a resource that ends with the row (4-byte aligned loads; past
// the row end they return 0).  The term of a column's own site is dropped by
// a select on the sum, so each column's sum is that of the plain loop.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_local_fields(const float* __restrict__ h,
                                                      const float* __restrict__ J,
                                                      const int8_t* __restrict__ chains, int64_t N,
                                                      int L, int q, float* __restrict__ H,
                                                      int32_t* dev_err,
                                                      const int32_t* __restrict__ active,
                                                      const int64_t* __restrict__ count,
                                                      int64_t g0, int wq) {
  if (active && *active == 0) return;
  // Workgroups are numbered so that each XCD runs a contiguous range of the
  // (column block, chain) order, chain fastest: the chains of one column
  // block walk the sites together on one XCD, and a coupling row segment that
  // several of them read (the same residue at a site) comes from that XCD's
  // L2 after the first.  The hardware deals consecutive workgroup ids to the
  // 8 XCDs in turn; the mapping is a bijection whatever the real placement.
  const uint32_t nwg = gridDim.x, f = blockIdx.x, xcd = f % 8u, per = nwg / 8u;
  const int64_t g = g0 + (int64_t)(xcd * per + min(xcd, nwg % 8u) + f / 8u);
  const int64_t c = g % N;
  const int yb = (int)(g / N);
  if (count && c >= *count) return;  // whole workgroup, before any barrier
  extern __shared__ int rowbase[];  // L entries: (k*q + s_k)
  const int Lq = L * q;
  for (int k = threadIdx.x; k < L; k += blockDim.x) {
    const int t = checked_token(chains[c * L + k], q, dev_err);
    rowbase[k] = k * q + t;
  }
  __syncthreads();
  const int r0 = 4 * (yb * wq + (int)threadIdx.x);
  if ((int)threadIdx.x >= wq || r0 >= Lq) return;
  int site[4];
  float acc[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    site[e] = (r0 + e) / q;
    acc[e] = (r0 + e < Lq) ? h[r0 + e] : 0.0f;
  }
  auto row = [&](int k) {
    const int rb = __builtin_amdgcn_readfirstlane(rowbase[k]);  // uniform
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(J + (size_t)rb * Lq), (short)0, (int)(Lq * sizeof(float)), 0x00020000);
    return __builtin_amdgcn_raw_buffer_load_b128(rs, r0 * (int)sizeof(float), 0, 0);
  };
  auto add = [&](int k, decltype(row(0)) w) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float sum = acc[e] + __uint_as_float(w[e]);
      acc[e] = (k == site[e]) ? acc[e] : sum;
    }
  };
  // four rows in flight, added in k order
  int k = 0;
  for (; k + 4 <= L; k += 4) {
    const auto w0 = row(k), w1 = row(k + 1), w2 = row(k + 2), w3 = row(k + 3);
    add(k, w0);
    add(k + 1, w1);
    add(k + 2, w2);
    add(k + 3, w3);
  }
  for (; k < L; ++k) add(k, row(k));
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (r0 + e < Lq) H[(size_t)c * Lq + r0 + e] = acc[e];
}

hipError_t launch_local_fields(const float* h, const float* J, const int8_t* chains, int64_t N,
                               int L, int q, float* H, int32_t* dev_err, hipStream_t s,
                               const int32_t* active, const int64_t* count) {
  const int Lq = L * q;
  // column blocks of equal width, wq quads (at most 256), so that every XCD's
  // range of workgroups holds the same work (a ragged last block left whole
  // XCDs with the light blocks: 14% longer at L = 256, q = 21)
  const int quads = (int)ceil_div(Lq, 4), nyb = (int)ceil_div(quads, 256);
  const int wq = (int)ceil_div(quads, nyb), bs = (int)ceil_div(wq, 64) * 64;
  // one launch per 2^22 workgroups (a grid dimension holds fewer than 2^32
  // work-items)
  const int64_t nwg = N * nyb, chunk = (int64_t)1 << 22;
  for (int64_t g0 = 0; g0 < nwg; g0 += chunk) {
    hipLaunchKernelGGL(k_local_fields, dim3((unsigned)std::min(chunk, nwg - g0)), dim3(bs),
                       sizeof(int) * L, s, h, J, chains, N, L, q, H, dev_err, active, count, g0, wq);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Gibbs sweeps, one wave64 per chain.
//
// Per site visit: lanes 0..q-1 read H[c][i*q + a], form l_a = beta*H, the
// wave maximum, e_a = exp(l_a - max), the inclusive prefix sum S_a in lane
// order, CDF_a = S_a / S_{q-1}, and the new state as the number of lanes
// a <= q-2 with CDF_a <= u (ballot + popcount).  The uniform u comes from
// Philox4x32-10 with counter (i/4, sweep, chain, 0), word i%4; one call per
// four sites.
// On a change a_old -> a_new all 64 lanes stream the chain's H row and the
// two coupling rows: H[r] += J[(i,a_new)][r] - J[(i,a_old)][r], r outside
// site i's own block.
// ---------------------------------------------------------------------------
// MH = true: single-site Metropolis instead of the heat-bath draw.  The
// proposal a' is uniform among the q-1 states != a (Philox counter (i/2,
// sweep, chain, 3), word 2(i%2): a' = (a + 1 + ((w (q-1)) >> 32)) mod q) and
// is accepted iff u < exp(beta (H_i(a') - H_i(a))), u from word 2(i%2)+1.
template <int WPB, bool MH>
__global__ __launch_bounds__(WPB * 64) void k_gibbs_hbm(const float* __restrict__ J,
                                                        int8_t* __restrict__ chains,
                                                        float* __restrict__ H, int64_t N, int L,
                                                        int q, int sweeps, uint32_t k0,
                                                        uint32_t k1, uint64_t sweep_offset,
                                                        float beta,
                                                        unsigned long long* flips_out,
                                                        const uint64_t* __restrict__ epoch,
                                                        const int32_t* __restrict__ active,
                                                        const ChainStream* __restrict__ streams) {
  if (active && *active == 0) return;
  if (epoch) sweep_offset += *epoch * (uint64_t)sweeps;
  extern __shared__ int8_t tok_all[];
  const int lane = threadIdx.x % kWave;
  const int wid = threadIdx.x / kWave;
  const int64_t c = (int64_t)blockIdx.x * WPB + wid;
  if (c >= N) return;  // whole wave leaves; no block barriers below
  uint32_t cid = (uint32_t)c;
  if (streams) {
    const ChainStream st = streams[c];
    k0 = (uint32_t)st.seed;
    k1 = (uint32_t)(st.seed >> 32);
    cid = st.chain;
    sweep_offset += st.sweep_offset;
  }
  const int Lpad = (L + 3) & ~3;
  int8_t* tok = tok_all + wid * Lpad;
  for (int i = lane; i < L; i += kWave) {
    const int t = chains[c * L + i];
    tok[i] = (int8_t)((t >= 0 && t < q) ? t : 0);  // invalid tokens were flagged by the field build
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();

  const int Lq = L * q;
  float* __restrict__ Hc = H + (size_t)c * Lq;
  unsigned long long nflip = 0;
  uint4 rnd = make_uint4(0, 0, 0, 0);
  for (int sw = 0; sw < sweeps; ++sw) {
    const uint32_t sg = (uint32_t)(sweep_offset + (uint64_t)sw);
    for (int i = 0; i < L; ++i) {
      const int a_old = tok[i];
      int a_new;
      if constexpr (MH) {
        if ((i & 1) == 0) rnd = philox4x32_10(make_uint4((uint32_t)i >> 1, sg, cid, 3u), k0, k1);
        const uint32_t wp = pick_word(rnd, 2 * (i & 1));
        const float u = word_to_uniform(pick_word(rnd, 2 * (i & 1) + 1));
        const int a_prop =
            (a_old + 1 + (int)(((uint64_t)wp * (uint64_t)(q - 1)) >> 32)) % q;
        const float d = Hc[i * q + a_prop] - Hc[i * q + a_old];  // same address in all lanes
        a_new = (u < expf(beta * d)) ? a_prop : a_old;
      } else {
        if ((i & 3) == 0) rnd = philox4x32_10(make_uint4((uint32_t)i >> 2, sg, cid, 0u), k0, k1);
        const float u = word_to_uniform(pick_word(rnd, i & 3));
        const float l = lane < q ? beta * Hc[i * q + lane] : -INFINITY;
        const float mx = wave_max(l);
        float e = lane < q ? expf(l - mx) : 0.0f;
        // inclusive prefix sum over lanes (q <= 32)
#pragma unroll
        for (int o = 1; o < 32; o <<= 1) {
          const float t = __shfl_up(e, o, kWave);
          if (lane >= o) e += t;
        }
        const float Z = __shfl(e, q - 1, kWave);
        const float cdf = e / Z;
        const bool below = (lane < q - 1) && (cdf <= u);
        a_new = __popcll(__ballot(below));
      }
      if (a_new != a_old) {
        const float* __restrict__ Jn = J + (size_t)(i * q + a_new) * Lq;
        const float* __restrict__ Jo = J + (size_t)(i * q + a_old) * Lq;
        const int blo = i * q, bhi = i * q + q;
        for (int r = lane; r < Lq; r += kWave) {
          if (r >= blo && r < bhi) continue;
          Hc[r] += Jn[r] - Jo[r];
        }
        if (lane == 0) tok[i] = (int8_t)a_new;
        ++nflip;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
      }
    }
  }
  for (int i = lane; i < L; i += kWave) chains[c * L + i] = tok[i];
  if (flips_out && lane == 0) atomicAdd(flips_out, nflip);
}

hipError_t launch_gibbs_sweeps(const float* J, int8_t* chains, float* H, int64_t N, int L, int q,
                               int sweeps, uint64_t seed, uint64_t sweep_offset, float beta,
                               unsigned long long* flips_out, hipStream_t s, const DevCtl& ctl,
                               bool metropolis) {
  constexpr int WPB = 4;
  const int Lpad = (L + 3) & ~3;
  auto kern = metropolis ? k_gibbs_hbm<WPB, true> : k_gibbs_hbm<WPB, false>;
  hipLaunchKernelGGL(kern, dim3((unsigned)ceil_div(N, WPB)), dim3(WPB * kWave), WPB * Lpad, s, J,
                     chains, H, N, L, q, sweeps, (uint32_t)seed, (uint32_t)(seed >> 32),
                     sweep_offset, beta, flips_out, ctl.epoch, ctl.active, ctl.streams);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gather form: the workspace layout here; the kernel in gather_kernel.hpp.
// ---------------------------------------------------------------------------
bool gather_supported(int L, int q) {
  return L >= 1 && L <= 512 && q >= 2 && q <= 32 && gather_shape(L, q, 1, 8).waves > 0;
}

size_t gather_ws_bytes(int L, int q) {
  return align256(sizeof(float) * (size_t)L * L * q * gather_qp(q));
}

// Jt[i][j][b][a'] = J[(j*q + b)][(i*q + a')] for a' < q and j != i, else 0
// (the block j = i is zero, so the sum over j may include it).
__global__ void k_gather_layout(const float* __restrict__ J, int L, int q, float* __restrict__ Jt,
                                const int32_t* __restrict__ active) {
  if (active && *active == 0) return;
  const int QP = gather_qp(q);
  const size_t total = (size_t)L * L * q * QP;
  const size_t Lq = (size_t)L * q;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int a = (int)(e % QP);
    const size_t r = e / QP;  // ((i*L + j)*q + b)
    const int b = (int)(r % q);
    const size_t ij = r / q;
    const int j = (int)(ij % L), i = (int)(ij / L);
    Jt[e] = (a < q && j != i) ? J[((size_t)j * q + b) * Lq + (size_t)i * q + a] : 0.0f;
  }
}

hipError_t launch_gibbs_gather(const float* h, const float* J, int8_t* chains, int64_t N, int L,
                               int q, int sweeps, uint64_t seed, uint64_t sweep_offset, float beta,
                               unsigned long long* flips_out, int32_t* dev_err, void* ws,
                               hipStream_t s, const DevCtl& ctl, bool metropolis) {
  float* Jt = static_cast<float*>(ws);
  if (!ctl.keep_layout) {
    const size_t total = (size_t)L * L * q * gather_qp(q);
    const unsigned nb = (unsigned)std::min<size_t>(ceil_div(total, 256), 65536);
    hipLaunchKernelGGL(k_gather_layout, dim3(nb), dim3(256), 0, s, J, L, q, Jt, ctl.active);
  }
  if (metropolis)
    return launch_gather_metropolis(h, Jt, chains, N, L, q, sweeps, seed, sweep_offset, beta,
                                    flips_out, dev_err, s, ctl);
  return launch_gather_form<false>(h, Jt, chains, N, L, q, sweeps, seed, sweep_offset, beta,
                                   flips_out, dev_err, s, ctl);
}

}  // namespace bmdca
