// Persistent-chain Gibbs sampler of the Potts model of Eq. (1)
// (adabmDCA 2.0, Sec. 2.1, "Monte Carlo estimation of the gradient").
//
// Layout: chains int8 [N][L]; local fields H float32 [N][Lq] in HBM, one row
// per chain; couplings J float32 [Lq][Lq] full-symmetric, so the row of
// vertex (i, a) is one contiguous Lq vector and H can be kept current with two
// coalesced row reads per accepted change.
#include "common.hpp"
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
// Grid: x over chains, y over 256-column slices of the row.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_local_fields(const float* __restrict__ h,
                                                      const float* __restrict__ J,
                                                      const int8_t* __restrict__ chains, int64_t N,
                                                      int L, int q, float* __restrict__ H,
                                                      int32_t* dev_err,
                                                      const int32_t* __restrict__ active) {
  if (active && *active == 0) return;
  extern __shared__ int rowbase[];  // L entries: (k*q + s_k)
  const int64_t c = blockIdx.x;
  const int Lq = L * q;
  for (int k = threadIdx.x; k < L; k += blockDim.x) {
    const int t = checked_token(chains[c * L + k], q, dev_err);
    rowbase[k] = k * q + t;
  }
  __syncthreads();
  const int r = blockIdx.y * blockDim.x + threadIdx.x;
  if (r >= Lq) return;
  const int site = r / q;
  float acc = h[r];
  for (int k = 0; k < L; ++k) {
    if (k == site) continue;
    acc += J[(size_t)rowbase[k] * Lq + r];
  }
  H[(size_t)c * Lq + r] = acc;
}

hipError_t launch_local_fields(const float* h, const float* J, const int8_t* chains, int64_t N,
                               int L, int q, float* H, int32_t* dev_err, hipStream_t s,
                               const int32_t* active) {
  const int Lq = L * q;
  const int bs = 256;
  dim3 grid((unsigned)N, (unsigned)ceil_div(Lq, bs));
  hipLaunchKernelGGL(k_local_fields, grid, dim3(bs), sizeof(int) * L, s, h, J, chains, N, L, q, H,
                     dev_err, active);
  return hipGetLastError();
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
// Gibbs sweeps with the local fields recomputed at every visit (gather form).
//
// A workgroup runs a group of chains in lockstep over the sites.  At site i
// every chain needs H_i(a) = h_i(a) + sum_{j != i} J_ij(a, s_j), i.e. row s_j
// of the q x q block J_ji for every j, the same blocks for all chains.
//
//   - Each call first copies J into the workspace as Jt[i][j][b][a'] (a'
//     padded to QP = q rounded up to 4, pad entries 0): Jt[i][j][b][a] =
//     J_ij(a, b) = J[(j,b)][(i,a)].  Site i's blocks are then one contiguous
//     L*q*QP run and the row a' = 0..QP-1 a chain needs is 16-byte aligned.
//   - Site i's run is streamed into LDS in chunks of JC sites by direct
//     global->LDS loads issued ahead of use into a ring of slots.
//   - G lanes serve one chain; lane g owns the R = JC/G consecutive sites
//     g*R .. g*R+R-1 of every chunk, reads their tokens with one LDS load, and
//     adds the row of each with QP/4 16-byte LDS loads.
//   - At the end of the site the G partial sums meet by xor-shuffles (the same
//     value in every lane of the chain), all G lanes run the same draw and lane
//     g = 0 stores the new token.
// Draw rule and Philox counters are those of the field form (the CDF test
// S_a / S_{q-1} <= u is evaluated as S_a <= u * S_{q-1}).
//
// Synchronisation: one workgroup barrier per chunk-step.  The slot written at
// step t + A (A = loads ahead, ring of A + 2 slots) was last read at step
// t + A - (A + 2) = t - 2, which every wave finished before the barrier of
// step t - 1; the loads of step t are complete once at most the A younger
// steps' loads are outstanding (s_waitcnt vmcnt).
// ---------------------------------------------------------------------------
#ifndef BMDCA_GATHER_G
#define BMDCA_GATHER_G 4
#endif
#ifndef BMDCA_GATHER_W
#define BMDCA_GATHER_W 4
#endif
#ifndef BMDCA_GATHER_ODD_QUADS
#define BMDCA_GATHER_ODD_QUADS 0
#endif
constexpr int kGG = BMDCA_GATHER_G;   // lanes per chain
constexpr int kGWv = BMDCA_GATHER_W;  // waves per workgroup
constexpr int kGR = kGG >= 4 ? 16 / kGG : 4;  // sites per lane per chunk (divides 4)
constexpr int kGJC = kGG * kGR;       // sites per chunk

typedef __attribute__((address_space(3))) void lds_void_t;

// Row pitch of Jt: q rounded up to a multiple of 4 floats (16-byte rows); with
// an odd number of 16-byte quads per row, consecutive rows start in 8
// different LDS bank groups, which keeps the 16-byte gathers of lanes that
// read different rows mostly conflict-free.
__host__ __device__ constexpr int gather_qp(int q) {
  return BMDCA_GATHER_ODD_QUADS ? ((((q + 3) / 4) % 2) ? ((q + 3) & ~3) : ((q + 3) & ~3) + 4)
                                : ((q + 3) & ~3);
}

// 16-byte loads per thread per chunk-step.
__host__ __device__ constexpr int gather_items(int q) {
  return (kGJC * q * gather_qp(q) + 4 * kGWv * 64 - 1) / (4 * kGWv * 64);
}

struct GatherShape {
  int ahead;   // chunk-steps loaded ahead (ring = ahead + 2 slots)
  int slot;    // floats per slot
  size_t lds;  // dynamic LDS bytes
};

static GatherShape gather_shape(int L, int q) {
  const int slot = 4 * kGWv * 64 * gather_items(q);
  const size_t tok = (size_t)((L + 3) / 4) * ((64 / kGG) * kGWv) * sizeof(uint32_t);
  for (int ahead = 2; ahead >= 1; --ahead) {
    const size_t lds = (size_t)(ahead + 2) * slot * sizeof(float) + tok;
    if (lds <= 160 * 1024 - 256) return {ahead, slot, lds};
  }
  return {0, 0, 0};
}

bool gather_supported(int L, int q) { return L <= 512 && q <= 32 && gather_shape(L, q).ahead > 0; }

size_t gather_ws_bytes(int L, int q) {
  return align256(sizeof(float) * (size_t)L * L * q * gather_qp(q));
}

// Jt[i][j][b][a'] = J[(j*q + b)][(i*q + a')] for a' < q, else 0.
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
    Jt[e] = (a < q) ? J[((size_t)j * q + b) * Lq + (size_t)i * q + a] : 0.0f;
  }
}

__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

template <int Q>
__global__ __launch_bounds__(kGWv * 64) void k_gibbs_gather(
    const float* __restrict__ h, const float* __restrict__ Jt, int8_t* __restrict__ chains,
    int64_t N, int L, int ahead, int slot, int cpb, int sweeps, uint32_t k0, uint32_t k1,
    uint64_t sweep_offset, float beta, unsigned long long* flips_out, int32_t* dev_err,
    const uint64_t* __restrict__ epoch, const int32_t* __restrict__ run,
    const ChainStream* __restrict__ streams) {
  if (run && *run == 0) return;  // whole grid leaves before any barrier
  if (epoch) sweep_offset += *epoch * (uint64_t)sweeps;
  constexpr int G = kGG, W = kGWv, R = kGR, JC = kGJC;
  constexpr int kT = W * 64, kCPW = 64 / G, kCPB = kCPW * W;
  constexpr int QP = gather_qp(Q), kQ4 = QP / 4;
  constexpr int kP = gather_items(Q);
  typedef float f4 __attribute__((ext_vector_type(4)));
  extern __shared__ __attribute__((aligned(16))) unsigned char g_smem[];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int cl = lane % kCPW, g = lane / kCPW;
  const int cb = wid * kCPW + cl;  // chain slot in the workgroup
  const int nslot = ahead + 2;
  float* ring = reinterpret_cast<float*>(g_smem);                             // [nslot][slot]
  uint32_t* tokw = reinterpret_cast<uint32_t*>(ring + (size_t)nslot * slot);  // [L/4][kCPB]
  unsigned char* tokb = reinterpret_cast<unsigned char*>(tokw);
  const int L4 = (L + 3) >> 2;
  const int64_t c = (int64_t)blockIdx.x * cpb + cb;
  const bool has_chain = cb < cpb;
  const bool active = has_chain && (c < N);
  uint32_t cid = (uint32_t)c;
  if (streams && active) {
    const ChainStream st = streams[c];
    k0 = (uint32_t)st.seed;
    k1 = (uint32_t)(st.seed >> 32);
    cid = st.chain;
    sweep_offset += st.sweep_offset;
  }
  const int nchunk = (L + JC - 1) / JC;
  const uint32_t site_bytes = (uint32_t)((size_t)L * Q * QP * sizeof(float));
  const uint32_t chunk_bytes = (uint32_t)(JC * Q * QP * sizeof(float));

  for (int k = g; k < L4; k += G) {
    uint32_t v = 0;
    for (int e = 0; e < 4; ++e) {
      const int j = 4 * k + e;
      int t = 0;
      if (active && j < L) t = checked_token(chains[c * L + j], Q, dev_err);
      v |= (uint32_t)t << (8 * e);
    }
    tokw[k * kCPB + cb] = v;
  }

  // Chunk-step (i, k) -> ring slot sl: bytes [k*chunk_bytes, +chunk_bytes) of
  // site i's run, read through a buffer resource that ends with the run (the
  // hardware returns 0 past it).  Item p of this thread is the 16 bytes at
  // 16*(tid + kT*p) of the slot.
  auto issue_chunk = [&](int i, int k, int sl) {
    const uint32_t off = (uint32_t)i * site_bytes + (uint32_t)k * chunk_bytes;
    const uint32_t left = site_bytes - (uint32_t)k * chunk_bytes;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(reinterpret_cast<const char*>(Jt) + off), (short)0, (int)left, 0x00020000);
    float* dst0 = ring + (size_t)sl * slot;
#pragma unroll
    for (int p = 0; p < kP; ++p) {
      float* dst = dst0 + 4 * (wid * 64 + kT * p);  // wave-uniform base; lane adds 16*lane
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t*)dst, 16, 16 * (tid + kT * p), 0, 0, 0);
    }
  };

  const int64_t T = (int64_t)sweeps * L * nchunk;
  // prefetch cursor: step tn = t + ahead, as (site, chunk, slot)
  int pi = 0, pk = 0, psl = 0;
  auto advance = [&](int& ii, int& kk, int& sl) {
    if (++kk == nchunk) {
      kk = 0;
      if (++ii == L) ii = 0;
    }
    if (++sl == nslot) sl = 0;
  };
  for (int64_t t = 0; t < ahead && t < T; ++t) {
    issue_chunk(pi, pk, psl);
    advance(pi, pk, psl);
  }

  float acc[QP];
  float hreg[Q];
#pragma unroll
  for (int a = 0; a < QP; ++a) acc[a] = 0.0f;
  unsigned long long nflip = 0;
  int i = 0, k = 0, sw = 0, csl = 0;
  for (int64_t t = 0; t < T; ++t) {
    if (k == 0) {
#pragma unroll
      for (int a = 0; a < Q; ++a) hreg[a] = h[i * Q + a];  // used at the draw of site i
    }
    const int64_t rest = T - 1 - t;  // steps after this one
    if (rest >= ahead) {
      issue_chunk(pi, pk, psl);
      advance(pi, pk, psl);
    }
    compiler_fence();
    // this step's loads are done once at most the younger steps' are pending
    const int64_t younger = rest < ahead ? rest : ahead;
    if (younger >= 2) {
      __builtin_amdgcn_s_waitcnt(((2 * kP) & 15) | (((2 * kP) >> 4) << 14) | 0x0F70);
    } else if (younger == 1) {
      __builtin_amdgcn_s_waitcnt((kP & 15) | ((kP >> 4) << 14) | 0x0F70);
    } else {
      __builtin_amdgcn_s_waitcnt(0x0F70);
    }
    __builtin_amdgcn_s_barrier();
    compiler_fence();

    // ---- this lane's R sites of the chunk
    const float* jb = ring + (size_t)csl * slot;
    const int j0 = k * JC + g * R;
    if (has_chain && j0 < L) {
      // the R tokens of j0 .. j0+R-1 share one dword (R divides 4 and j0 % R == 0)
      const uint32_t tk = tokw[(j0 >> 2) * kCPB + cb] >> (8 * (j0 & 3));
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int j = j0 + r;
        if (j < L && j != i) {
          const int s = (int)((tk >> (8 * r)) & 0xFF);
          const f4* row = reinterpret_cast<const f4*>(jb + ((g * R + r) * Q + s) * QP);
#pragma unroll
          for (int v = 0; v < kQ4; ++v) {
            const f4 x = row[v];
            acc[4 * v + 0] += x[0];
            acc[4 * v + 1] += x[1];
            acc[4 * v + 2] += x[2];
            acc[4 * v + 3] += x[3];
          }
        }
      }
    }

    if (k == nchunk - 1) {
      // ---- combine the G partial sums, draw, store the token
#pragma unroll
      for (int o = kCPW; o < 64; o <<= 1)
#pragma unroll
        for (int a = 0; a < Q; ++a) acc[a] += __shfl_xor(acc[a], o, kWave);
      float mx = -INFINITY;
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        acc[a] = beta * (hreg[a] + acc[a]);
        mx = fmaxf(mx, acc[a]);
      }
      float run = 0.0f;
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        run += __expf(acc[a] - mx);
        acc[a] = run;  // S_a
      }
      const uint32_t sg = (uint32_t)(sweep_offset + (uint64_t)sw);
      const uint4 rnd = philox4x32_10(make_uint4((uint32_t)i >> 2, sg, cid, 0u), k0, k1);
      const float uz = word_to_uniform(pick_word(rnd, i & 3)) * run;
      int anew = 0;
#pragma unroll
      for (int a = 0; a < Q - 1; ++a) anew += (acc[a] <= uz) ? 1 : 0;
      if (g == 0 && has_chain) {
        unsigned char* tp = tokb + ((i >> 2) * kCPB + cb) * 4 + (i & 3);
        if (active && anew != (int)*tp) ++nflip;
        *tp = (unsigned char)anew;
      }
#pragma unroll
      for (int a = 0; a < QP; ++a) acc[a] = 0.0f;
    }
    if (++csl == nslot) csl = 0;
    if (++k == nchunk) {
      k = 0;
      if (++i == L) {
        i = 0;
        ++sw;
      }
    }
  }
  __syncthreads();
  if (active)
    for (int j = g; j < L; j += G) chains[c * L + j] = (int8_t)tokb[((j >> 2) * kCPB + cb) * 4 + (j & 3)];
  if (flips_out) {
    unsigned long long tot = nflip;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, kWave);
    if (lane == 0 && tot) atomicAdd(flips_out, tot);
  }
}

static int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      cus = n;
    else
      cus = 256;
  }
  return cus;
}

template <int Q>
static hipError_t launch_gather_q(const float* h, const float* Jt, int8_t* chains, int64_t N,
                                  int L, int sweeps, uint64_t seed, uint64_t sweep_offset,
                                  float beta, unsigned long long* flips_out, int32_t* dev_err,
                                  hipStream_t s, const DevCtl& ctl) {
  const GatherShape gs = gather_shape(L, Q);
  if (gs.ahead == 0) return hipErrorInvalidValue;
  constexpr int kCPB = (64 / kGG) * kGWv;
  // chains per workgroup: spread the chains over all CUs in as few rounds as
  // the workgroup size allows (one workgroup per CU at a time)
  const int64_t cus = ctl.cu_share > 0 ? std::min<int64_t>(ctl.cu_share, device_cus()) : device_cus();
  const int64_t rounds = ceil_div(N, cus * kCPB);
  const int cpb = (int)std::min<int64_t>(kCPB, ceil_div(N, rounds * cus));
  const unsigned nb = (unsigned)ceil_div(N, cpb);
  auto kern = k_gibbs_gather<Q>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)gs.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(nb), dim3(kGWv * 64), gs.lds, s, h, Jt, chains, N, L, gs.ahead,
                     gs.slot, cpb, sweeps, (uint32_t)seed, (uint32_t)(seed >> 32), sweep_offset,
                     beta, flips_out, dev_err, ctl.epoch, ctl.active, ctl.streams);
  return hipGetLastError();
}

hipError_t launch_gibbs_gather(const float* h, const float* J, int8_t* chains, int64_t N, int L,
                               int q, int sweeps, uint64_t seed, uint64_t sweep_offset, float beta,
                               unsigned long long* flips_out, int32_t* dev_err, void* ws,
                               hipStream_t s, const DevCtl& ctl) {
  float* Jt = static_cast<float*>(ws);
  {
    const size_t total = (size_t)L * L * q * gather_qp(q);
    const unsigned nb = (unsigned)std::min<size_t>(ceil_div(total, 256), 65536);
    hipLaunchKernelGGL(k_gather_layout, dim3(nb), dim3(256), 0, s, J, L, q, Jt, ctl.active);
  }
  switch (q) {
#define BMDCA_GQ(n) \
  case n:           \
    return launch_gather_q<n>(h, Jt, chains, N, L, sweeps, seed, sweep_offset, beta, flips_out, \
                              dev_err, s, ctl);
    BMDCA_GQ(2) BMDCA_GQ(3) BMDCA_GQ(4) BMDCA_GQ(5) BMDCA_GQ(6) BMDCA_GQ(7) BMDCA_GQ(8)
    BMDCA_GQ(9) BMDCA_GQ(10) BMDCA_GQ(11) BMDCA_GQ(12) BMDCA_GQ(13) BMDCA_GQ(14) BMDCA_GQ(15)
    BMDCA_GQ(16) BMDCA_GQ(17) BMDCA_GQ(18) BMDCA_GQ(19) BMDCA_GQ(20) BMDCA_GQ(21) BMDCA_GQ(22)
    BMDCA_GQ(23) BMDCA_GQ(24) BMDCA_GQ(25) BMDCA_GQ(26) BMDCA_GQ(27) BMDCA_GQ(28) BMDCA_GQ(29)
    BMDCA_GQ(30) BMDCA_GQ(31) BMDCA_GQ(32)
#undef BMDCA_GQ
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace bmdca
