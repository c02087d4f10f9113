// Gather-form sampler kernel (adabmDCA 2.0, Sec. 2.1): the heat-bath draw
// and single-site Metropolis share the whole kernel but its draw step; the
// two are instantiated in separate sources (sampler.hip, sampler_mh.hip) so
// that they compile in parallel.
#pragma once
#include <type_traits>

#include "common.hpp"
#include "gather_plan.hpp"
#include "internal.hpp"

namespace bmdca {

// ---------------------------------------------------------------------------
// Gibbs sweeps with the local fields recomputed at every visit (gather form).
//
// A workgroup runs a group of chains in lockstep over the sites.  At site i
// every chain needs H_i(a) = h_i(a) + sum_{j != i} J_ij(a, s_j), i.e. row s_j
// of the q x q block J_ji for every j, the same blocks for all chains.
//
//   - Each call first copies J into the workspace as Jt[i][j][b][a'] (a'
//     padded to QP = q rounded up to 4, pad entries 0): Jt[i][j][b][a] =
//     J_ij(a, b) = J[(j,b)][(i,a)].  Site i's blocks are one contiguous
//     L*q*QP run, and the row a' = 0..QP-1 a chain needs is QP/4 16-byte
//     quads.
//   - Site i's run is streamed into LDS in chunks of JC sites by direct
//     buffer->LDS loads, A = 3 chunks ahead of use, into a ring of A + 1
//     slots.  JC is chosen per (L, q) to fill the LDS left over by the
//     tokens.
//   - Each chain owns LPC = 8 or 16 consecutive lanes (16 for Metropolis at
//     q <= 8; heat-bath chains with 5..7 quads per row may be narrow, one
//     lane per quad, the lanes of the row group only), lane p = u * V + v
//     (V = QP/4 rounded up to a power of two, S = LPC / V site groups): lane
//     (u, v) adds quad v of the rows of the sites j = u, u + S, u + 2S, ...
//     of every chunk.  For q > 16 each 8 lanes of a chain read one row as
//     contiguous quads; lanes v >= QP/4 stay idle.
//   - Tokens live in LDS as bytes, position (j mod S, j div S), so that a
//     lane reads the tokens of its next four sites with one 32-bit load.
//   - At the end of the site the S partial quads meet by xor-shuffles, and
//     the draw runs across the V lanes of a quad group: group max, FP32
//     exponentials, an inclusive scan of the quad sums over v, the total
//     S_{q-1} broadcast from the lane that holds state q-1, and a count of
//     the states a <= q-2 with S_a <= u S_{q-1} summed over v.  Lane p = 0
//     stores the new token.
// Draw rule and Philox counters are those of the field form (the CDF test
// S_a / S_{q-1} <= u is evaluated as S_a <= u * S_{q-1}).
//   - MH = true makes single-site Metropolis visits with the field form's
//     proposal, counters and acceptance test.  The proposal a' and the
//     current a are known when the site starts, so only two entries of each
//     row are needed: the chain's lanes split the chunk's sites (lane p takes
//     positions p, p + LPC, ...) and add J_ij(a', s_j) - J_ij(a, s_j) (lane 0
//     starts from h_i(a') - h_i(a)); at the end of the site a DPP sum over
//     the chain's lanes gives H_i(a') - H_i(a) and lane p = 0 accepts iff
//     u < exp(beta (H_i(a') - H_i(a))).  The staging of the blocks is the
//     same as for the heat-bath draw.
//
// Synchronisation: one workgroup barrier per chunk-step.  Before it, each
// wave waits for its share of the current chunk (vmcnt: at most the A - 1
// younger chunks outstanding) and for its own LDS reads of the previous step
// (lgkmcnt 0).  After it, the slot of the previous step is free for every
// wave and receives the chunk A steps ahead.  A chain's tokens are read and
// written only by its own lanes (one wave, LDS in order), so token updates
// need no barrier.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void_t;

__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

// s_waitcnt vmcnt(N) lgkmcnt(0), N in [0, 63].
template <int N>
__device__ __forceinline__ void wait_vm_lgkm0() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0070);
}

// Lane exchanges inside the aligned 8-lane group of a chain with no LDS
// traffic: DPP quad permutations, row shifts and the half-row mirror; the
// xor-4 exchange by ds_swizzle.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ int dpp_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <- lane 7-i of each 8
constexpr int kDppShr1 = 0x111, kDppShr2 = 0x112, kDppShr4 = 0x114;  // lane i <- lane i-k
constexpr int kDppRor8 = 0x128;       // lane i <- lane (i+8) mod 16 of each 16
__device__ __forceinline__ float swz_xor4(float x) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), 0x101F));
}
// over the V lanes of a quad group (V = 1, 2, 4, 8; groups aligned)
template <int V>
__device__ __forceinline__ float group_max(float x) {
  if (V >= 2) x = fmaxf(x, dpp_f<kDppXor1>(x));
  if (V >= 4) x = fmaxf(x, dpp_f<kDppXor2>(x));
  if (V >= 8) x = fmaxf(x, dpp_f<kDppHalfMirror>(x));
  return x;
}
template <int V>
__device__ __forceinline__ float group_fsum(float x) {
  if (V >= 2) x += dpp_f<kDppXor1>(x);
  if (V >= 4) x += dpp_f<kDppXor2>(x);
  if (V >= 8) x += dpp_f<kDppHalfMirror>(x);
  return x;
}
template <int V>
__device__ __forceinline__ int group_sum(int x) {
  if (V >= 2) x += dpp_i<kDppXor1>(x);
  if (V >= 4) x += dpp_i<kDppXor2>(x);
  if (V >= 8) x += dpp_i<kDppHalfMirror>(x);
  return x;
}
// inclusive prefix sum over v = 0..V-1
template <int V>
__device__ __forceinline__ float group_scan(float x, int v) {
  if (V >= 2) { const float y = dpp_f<kDppShr1>(x); if (v >= 1) x += y; }
  if (V >= 4) { const float y = dpp_f<kDppShr2>(x); if (v >= 2) x += y; }
  if (V >= 8) { const float y = dpp_f<kDppShr4>(x); if (v >= 4) x += y; }
  return x;
}
// value of lane SRC of the group, in every lane of it
template <int V, int SRC>
__device__ __forceinline__ float group_bcast(float x, int v) {
  if constexpr (V == 1) {
    return x;
  } else if constexpr (V == 2) {
    return dpp_f<SRC | (SRC << 2) | ((2 + SRC) << 4) | ((2 + SRC) << 6)>(x);
  } else if constexpr (V == 4) {
    return dpp_f<SRC * 0x55>(x);
  } else {
    const float x1 = dpp_f<(SRC & 3) * 0x55>(x);  // lane SRC%4 of each quad
    const float x2 = dpp_f<kDppHalfMirror>(x1);   // the other quad's
    return ((v & 4) == (SRC & 4)) ? x1 : x2;
  }
}
// sum over the S = LPC / V site groups (lanes with the same v)
template <int V, int LPC>
__device__ __forceinline__ float combine_sites(float x) {
  if (V <= 1) x += dpp_f<kDppXor1>(x);
  if (V <= 2) x += dpp_f<kDppXor2>(x);
  if (V <= 4) x += swz_xor4(x);
  if (LPC == 16) x += dpp_f<kDppRor8>(x);  // lane i <- lane i^8 of each 16
  return x;
}

// Narrow chains (LPC = quads per row, 5..7, one chain per LPC consecutive
// lanes): the draw's cross-lane steps by lane shuffles inside the chain,
// base = first lane of the chain, v = lane - base.  The prefix sum keeps the
// association order of group_scan<8> (add lane v-1, then v-2, then v-4), the
// other steps are exact in any order.
template <int LPC>
__device__ __forceinline__ float narrow_max(float x, int base) {
  float m = __shfl(x, base, kWave);
#pragma unroll
  for (int k = 1; k < LPC; ++k) m = fmaxf(m, __shfl(x, base + k, kWave));
  return m;
}
__device__ __forceinline__ float narrow_scan(float x, int lane, int v) {
  float y = __shfl(x, lane - 1, kWave);
  if (v >= 1) x += y;
  y = __shfl(x, lane - 2, kWave);
  if (v >= 2) x += y;
  y = __shfl(x, lane - 4, kWave);
  if (v >= 4) x += y;
  return x;
}
template <int LPC>
__device__ __forceinline__ int narrow_sum(int x, int base) {
  int t = 0;
#pragma unroll
  for (int k = 0; k < LPC; ++k) t += __shfl(x, base + k, kWave);
  return t;
}

// MAXW: the most waves a workgroup of this instantiation may have (16, or 8
// for plans of at most 8 waves: twice the registers per lane, 256).
template <int Q, int IT, int LPC, bool MH, int MAXW, bool PAIR>
__global__ __launch_bounds__(MAXW * 64) void k_gibbs_gather(
    const float* __restrict__ h, const float* __restrict__ Jt, int8_t* __restrict__ chains,
    int64_t N, int L, int jc, int nchunk, int m4, int ahead, int nload, int slot, int cpb,
    int sweeps, uint32_t k0, uint32_t k1, uint64_t sweep_offset, float beta,
    unsigned long long* flips_out, int32_t* dev_err, const uint64_t* __restrict__ epoch,
    const int32_t* __restrict__ run, const ChainStream* __restrict__ streams,
    const int64_t* __restrict__ count) {
  if (run && *run == 0) return;  // whole grid leaves before any barrier
  // With a live count (a launch sized for N chains of which the first *count
  // are live) the workgroups take chains strided by the grid, chain
  // cb * gridDim.x + blockIdx.x, so a partly filled arena still spreads its
  // live chains over every workgroup; otherwise each takes a contiguous range.
  if (count) {
    const int64_t live = *count;
    if (live < N) N = live;
  }
  if ((count ? (int64_t)blockIdx.x : (int64_t)blockIdx.x * cpb) >= N)
    return;  // no live chain: whole workgroup, before any barrier
  if (epoch) sweep_offset += *epoch * (uint64_t)sweeps;
  constexpr int QP = gather_qp(Q), NQ = QP / 4, V = gather_v(Q), S = gather_s(Q, LPC);
  constexpr int vL = (Q - 1) / 4, eL = (Q - 1) % 4;  // lane and slot of state q-1
  typedef float f4 __attribute__((ext_vector_type(4)));
  extern __shared__ __attribute__((aligned(16))) unsigned char g_smem[];
  // chains per wave: 64 / LPC (narrow chains: the last 64 % LPC lanes of a
  // wave hold no chain)
  constexpr int CPW = 64 / LPC;
  constexpr bool kNarrow = LPC < 8;
  const int T = blockDim.x, CPB = kNarrow ? (T / 64) * CPW : T / LPC;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int p = kNarrow ? lane % LPC : lane & (LPC - 1), u = p / V, v = p % V;
  const bool lane_ok = !kNarrow || lane < CPW * LPC;
  // chain slot in the workgroup (the wide form keeps the plain expression:
  // the per-wave one costs scalar registers that the wide kernels spill)
  const int cb = kNarrow ? wid * CPW + lane / LPC : tid / LPC;
  const int nslot = ahead + 1;
  float* ring = reinterpret_cast<float*>(g_smem);                             // [nslot][slot]
  uint32_t* tokw = reinterpret_cast<uint32_t*>(ring + (size_t)nslot * slot);  // [S][m4][CPB]
  unsigned char* tokb = reinterpret_cast<unsigned char*>(tokw);
  const int64_t c =
      count ? (int64_t)cb * gridDim.x + blockIdx.x : (int64_t)blockIdx.x * cpb + cb;
  const bool has_chain = lane_ok && cb < cpb;
  const bool active = has_chain && (c < N);
  const bool reader = has_chain && v < NQ;
  uint32_t cid = (uint32_t)c;
  if (streams && active) {
    const ChainStream st = streams[c];
    k0 = (uint32_t)st.seed;
    k1 = (uint32_t)(st.seed >> 32);
    cid = st.chain;
    sweep_offset += st.sweep_offset;
  }
  // byte of the token of site j in the chain's token area
  // byte offset of the token of site j (32-bit arithmetic)
  auto tok_off = [&](int j) -> uint32_t {
    const int m = j / S;
    return (uint32_t)((((j % S) * m4 + (m >> 2)) * CPB + cb) * 4 + (m & 3));
  };
  auto tok_at = [&](int j) -> unsigned char* {
    const int m = j / S;
    return tokb + ((size_t)((j % S) * m4 + (m >> 2)) * CPB + cb) * 4 + (m & 3);
  };

  for (int k = lane_ok ? p : S * m4; k < S * m4; k += LPC) {  // dword k = (site group, 4 positions)
    const int uu = k / m4, mq = k % m4;
    uint32_t w = 0;
    for (int e = 0; e < 4; ++e) {
      const int j = S * (4 * mq + e) + uu;
      int t = 0;
      if (active && j < L) t = checked_token(chains[c * L + j], Q, dev_err);
      w |= (uint32_t)t << (8 * e);
    }
    tokw[k * CPB + cb] = w;
  }

  const uint32_t site_bytes = (uint32_t)((size_t)L * Q * QP * sizeof(float));
  const uint32_t chunk_bytes = (uint32_t)((size_t)jc * Q * QP * sizeof(float));
  // Chunk-step (i, k) -> ring slot sl: bytes [k*chunk_bytes, +slot bytes) of
  // site i's run, read through a buffer resource that ends with the run (the
  // hardware returns 0 past it), as 1 KB blocks: loading wave w < nload
  // issues exactly IT of them, blocks w*IT .. w*IT+IT-1, lane l the 16 bytes
  // at 16 l of each.  Bytes past the chunk land in the slot's padding.
  const bool loader = wid < nload;
  auto issue_chunk = [&](int i, int k, int sl) {
    const uint32_t off = (uint32_t)i * site_bytes + (uint32_t)k * chunk_bytes;
    const uint32_t left = site_bytes - (uint32_t)k * chunk_bytes;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(reinterpret_cast<const char*>(Jt) + off), (short)0, (int)left, 0x00020000);
    float* dst0 = ring + (size_t)sl * slot + 256 * IT * wid;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      float* dst = dst0 + 256 * it;  // wave-uniform base; lane adds 16*lane
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void_t*)dst, 16,
                                               1024 * (IT * wid + it) + 16 * lane, 0, 0, 0);
    }
  };

  const int64_t Tn = (int64_t)sweeps * L * nchunk;
  // prefetch cursor: the next chunk-step to issue, as (site, chunk, slot)
  int pi = 0, pk = 0, psl = 0;
  auto advance = [&](int& ii, int& kk, int& sl) {
    if (++kk == nchunk) {
      kk = 0;
      if (++ii == L) ii = 0;
    }
    if (++sl == nslot) sl = 0;
  };
  // chunks in flight before the first step: `ahead` (one barrier per step),
  // or two (paired steps)
  for (int64_t t = 0; t < (PAIR ? 2 : ahead) && t < Tn; ++t) {
    if (loader) issue_chunk(pi, pk, psl);
    advance(pi, pk, psl);
  }

  f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  float hq[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  unsigned long long nflip = 0;
  // one Philox call gives the words of 4 consecutive sites (heat-bath draw)
  // or 2 (Metropolis); sites are drawn in order from i = 0 every sweep.  The
  // words are kept across sites except with 31 loads per wave, where the four
  // extra live registers add spills and cost more than the calls they save.
  constexpr bool kKeepRnd = IT != 31;
  uint4 rnd = make_uint4(0u, 0u, 0u, 0u);
  // Metropolis visit state: current and proposed state, uniform, and this
  // lane's part of H_i(a') - H_i(a)
  int mh_old = 0, mh_prop = 0;
  float mh_u = 0.0f, mh_d = 0.0f;
  // tokens of the next chunk-step's first two positions of this lane, read
  // one step ahead (software pipeline), and their sites
  uint32_t mh_nsv[2] = {0u, 0u};
  int mh_nj[2] = {0, 0};
  const int jcs = jc / S;  // positions per lane per chunk (multiple of 4)
  int i = 0, k = 0, sw = 0, csl = 0;
  // heat-bath draw: the four token dwords the next chunk-step's first group
  // of 16 positions starts with, read one step ahead (software pipeline).
  // In the 16-wave instantiation (128 VGPRs) only with one site group
  // (q > 16): with several, the four live registers cost more in spills than
  // the pipeline saves.
  constexpr bool kPipeTok = !MH && (S == 1 || MAXW <= 8);
  const uint32_t* twl = tokw + (size_t)u * m4 * CPB + cb;
  uint32_t g_tok[4] = {0u, 0u, 0u, 0u};
  if (kPipeTok && reader) {  // first chunk-step (tokens written above by this wave)
#pragma unroll
    for (int d = 0; d < 4; ++d) g_tok[d] = twl[min(d, m4 - 1) * CPB];
  }
  if (MH) {  // tokens of the first chunk-step (written above by this wave)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      mh_nj[e] = min(min(p + LPC * e, jc - 1), L - 1);
      mh_nsv[e] = (uint32_t)tokb[tok_off(mh_nj[e])];
    }
  }
  for (int64_t t = 0; t < Tn; ++t) {
    if constexpr (PAIR) {
      // even steps: chunks t and t + 1 (issued two steps ago) complete in
      // every wave after the barrier, and the slots of t - 2 and t - 1 are
      // free for t + 2 and t + 3; odd steps read chunk t without a barrier
      // (the loads in flight fill the slots of t + 1 and t + 2)
      if ((t & 1) == 0) {
        compiler_fence();
        wait_vm_lgkm0<0>();
        __builtin_amdgcn_s_barrier();
        compiler_fence();
        // the next two chunks' loads go out ahead of the other waves' work
        // (0.5-1.6% shorter launches; in the one-barrier schedule the same
        // raise cost up to 1.4%)
        __builtin_amdgcn_s_setprio(3);
        for (int e = 0; e < 2; ++e) {
          if (t + 2 + e < Tn) {
            if (loader) issue_chunk(pi, pk, psl);
            advance(pi, pk, psl);
          }
        }
        __builtin_amdgcn_s_setprio(0);
      }
    } else {
      // chunk t is complete once at most the younger issued chunks (ahead - 1
      // of them, fewer at the end) are pending
      const int64_t rest = Tn - 1 - t;
      const int younger = rest < ahead - 1 ? (int)rest : ahead - 1;
      compiler_fence();
      if (younger >= 2)
        wait_vm_lgkm0<2 * IT>();
      else if (younger == 1)
        wait_vm_lgkm0<IT>();
      else
        wait_vm_lgkm0<0>();
      __builtin_amdgcn_s_barrier();
      compiler_fence();
      if (t + ahead < Tn) {
        if (loader) issue_chunk(pi, pk, psl);
        advance(pi, pk, psl);
      }
    }
    if (MH && k == 0) {
      // proposal and uniform of this visit; lane 0 starts the difference
      // with h_i(a') - h_i(a)
      const uint32_t sg = (uint32_t)(sweep_offset + (uint64_t)sw);
      if (!kKeepRnd || (i & 1) == 0)
        rnd = philox4x32_10(make_uint4((uint32_t)i >> 1, sg, cid, 3u), k0, k1);
      const uint32_t wp = pick_word(rnd, 2 * (i & 1));
      mh_u = word_to_uniform(pick_word(rnd, 2 * (i & 1) + 1));
      mh_old = (int)*tok_at(i);
      mh_prop = (mh_old + 1 + (int)(((uint64_t)wp * (uint64_t)(Q - 1)) >> 32)) % Q;
      // h_i by scalar loads of the whole row (uniform addresses), then a lane
      // select: a per-lane vector load here would share the counter of the
      // chunk loads in flight and make the wave wait for all of them
      float hs[Q];
#pragma unroll
      for (int a = 0; a < Q; ++a) hs[a] = h[i * Q + a];
      float hp = 0.0f, ho = 0.0f;
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        hp = a == mh_prop ? hs[a] : hp;
        ho = a == mh_old ? hs[a] : ho;
      }
      mh_d = p == 0 ? hp - ho : 0.0f;
    }
    if (!MH && k == 0) {
      // h_i for this lane's quad (scalar loads of the row, lane select)
      float hs[Q];
#pragma unroll
      for (int a = 0; a < Q; ++a) hs[a] = h[i * Q + a];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float x = 0.0f;
#pragma unroll
        for (int vv = 0; vv < NQ; ++vv)
          if (4 * vv + e < Q && v == vv) x = hs[4 * vv + e];
        hq[e] = x;
      }
    }

    // ---- this lane's sites of the chunk: j = k*jc + S*r + u, r < jc/S,
    // token positions m0 + r.  The rows of j = i (zero block) and of j >= L
    // (past the end of the run, loaded as zeros) add nothing, so every
    // position is added unconditionally; positions past the last token dword
    // read any valid token.  Groups of 16 positions: 4 token loads, 16 row
    // loads, the adds (a tail group loads only its positions).
    if (MH && has_chain) {
      // Metropolis needs two entries of each row: the chain's lanes split
      // the chunk's sites (lane p: positions p, p + LPC, ...) and add
      // J_ij(a', s_j) - J_ij(a, s_j); the row of j = i is the zero block.
      // Two positions at a time, without branches: both token reads, then
      // the four entry reads.  Positions past the chunk are clamped and not
      // added; sites past the run read a valid token (clamped to L - 1) and
      // find a zero row (the slot holds zeros past the run end).
      const float* cb0 = ring + (size_t)csl * slot;
      const int j0 = k * jc;
      const int nr = (jc + LPC - 1) / LPC;  // positions per lane, uniform
      for (int r0 = 0; r0 < nr; r0 += 2) {
        uint32_t sv[2];
        int jlv[2];
        bool ok[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int jl = p + LPC * (r0 + e);
          ok[e] = jl < jc;
          jlv[e] = ok[e] ? jl : jc - 1;
          sv[e] = r0 == 0 ? mh_nsv[e] : (uint32_t)tokb[tok_off(min(j0 + jlv[e], L - 1))];
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const float* row = cb0 + __umul24((uint32_t)(jlv[e] * Q) + sv[e], (uint32_t)QP);
          const float x = row[mh_prop] - row[mh_old];
          mh_d += ok[e] ? x : 0.0f;
        }
      }
    }
    if (MH) {
      // read the tokens the next chunk-step starts with (same site, next
      // chunk; or the next site's first chunk)
      const int nk = k + 1 < nchunk ? k + 1 : 0;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int jl = min(p + LPC * e, jc - 1);
        mh_nj[e] = min(nk * jc + jl, L - 1);
        mh_nsv[e] = (uint32_t)tokb[tok_off(mh_nj[e])];
      }
    }
    if (!MH && reader) {
      const float* jb = ring + (size_t)csl * slot + 4 * v;
      const int m0 = k * jcs;  // multiple of 4
      const uint32_t* tw = tokw + (size_t)u * m4 * CPB + cb;
      auto group = [&](int r0, bool tail) {
        // a tail with several site groups (q <= 16, long chunks) skips the
        // loads past its positions; with one (q > 16, at most 16 positions
        // lost) it loads clamped rows, the faster code at protein scale
        constexpr bool kSkip = S > 1;
        uint32_t tk[4];
#pragma unroll
        for (int d = 0; d < 4; ++d)
          tk[d] = (kPipeTok && r0 == 0) ? g_tok[d]  // read one step ahead
                  : (!(kSkip && tail) || 4 * d < jcs - r0)
                      ? tw[min(((m0 + r0) >> 2) + d, m4 - 1) * CPB]
                      : 0u;
        f4 x[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int s = (int)((tk[e >> 2] >> (8 * (e & 3))) & 0xFF);
          // row offset s * QP by a 24-bit multiply (full rate; a 32-bit
          // integer multiply issues at a quarter of the rate)
          const uint32_t so = __umul24((uint32_t)s, (uint32_t)QP);
          if (kSkip) {
            if (!tail || r0 + e < jcs)  // wave-uniform
              x[e] = *reinterpret_cast<const f4*>(jb + (S * (r0 + e) + u) * Q * QP + so);
          } else {
            const int r = tail ? min(r0 + e, jcs - 1) : r0 + e;
            x[e] = *reinterpret_cast<const f4*>(jb + (S * r + u) * Q * QP + so);
          }
        }
#pragma unroll
        for (int e = 0; e < 16; ++e)
          if (!tail || r0 + e < jcs) acc += x[e];
      };
      if (QP < 24 && QP != 16 && jcs % 16 != 0) {
        // Rows of 1-3 or 5 quads (q <= 12, q = 17..20) in chunks whose
        // positions per lane are not a multiple of 16: groups of a
        // compile-time length over the
        // positions of this chunk that can hold a site j < L (a multiple of
        // 4, at most jcs; the rest, past the run in a site's last chunk, are
        // zero rows, and adding +0 to a sum that started at +0 changes no
        // bit), with no clamped or skipped reads in the tail group.  Measured
        // per 10 sweeps: q = 5, L = 400: 23.2 -> 17.4 ms; q = 12, L = 200:
        // 14.5 -> 11.2; q = 17, L = 150: 15.6 -> 10.9.  Where the positions
        // are a multiple of 16 (q = 8, L = 60; q = 13, L = 130) this form was
        // 2-4% slower, so those take the group below; with both forms in the
        // kernel the compiler scheduled the common group of 16-float rows
        // (q = 13..16) worse (5% at q = 13, L = 130), and for rows of 6-8
        // quads (q = 21) the new form itself read 10-13% slower, so those
        // instantiations keep the group below alone.
        const int nv = min(jcs, (((L - k * jc + S - 1) / S) + 3) & ~3);
        auto tgroup = [&](int r1, auto n_c) {
          constexpr int n = decltype(n_c)::value;
          uint32_t tk[n / 4];
#pragma unroll
          for (int d = 0; d < n / 4; ++d)
            tk[d] = (kPipeTok && r1 == 0) ? g_tok[d] : tw[min(((m0 + r1) >> 2) + d, m4 - 1) * CPB];
          f4 x[n];
#pragma unroll
          for (int e = 0; e < n; ++e) {
            const uint32_t so = __umul24((tk[e >> 2] >> (8 * (e & 3))) & 0xFFu, (uint32_t)QP);
            x[e] = *reinterpret_cast<const f4*>(jb + (S * (r1 + e) + u) * Q * QP + so);
          }
#pragma unroll
          for (int e = 0; e < n; ++e) acc += x[e];
        };
        int r1 = 0;
        for (; r1 + 16 <= nv; r1 += 16) tgroup(r1, std::integral_constant<int, 16>{});
        if (nv - r1 == 12)
          tgroup(r1, std::integral_constant<int, 12>{});
        else if (nv - r1 == 8)
          tgroup(r1, std::integral_constant<int, 8>{});
        else if (nv - r1 == 4)
          tgroup(r1, std::integral_constant<int, 4>{});
      } else {
        int r0 = 0;
        for (; r0 + 16 <= jcs; r0 += 16) group(r0, false);
        if (r0 < jcs) group(r0, true);
      }
      if (kPipeTok) {
        // the next chunk-step's first token dwords (same site's next chunk,
        // or the next site's first chunk)
        const int m0n = (k + 1 < nchunk ? k + 1 : 0) * jcs;
#pragma unroll
        for (int d = 0; d < 4; ++d) g_tok[d] = tw[min((m0n >> 2) + d, m4 - 1) * CPB];
      }
    }

    if (k == nchunk - 1) {
      // ---- combine the S site groups, draw, store the token
      if constexpr (MH) {
        float d = group_fsum<8>(mh_d);  // H_i(a') - H_i(a), in every lane of the chain
        if (LPC == 16) d += dpp_f<kDppRor8>(d);
        const bool acc_mh = mh_u < expf(beta * d);
        if (acc_mh) {
          // the next step's tokens were read before this change
#pragma unroll
          for (int e = 0; e < 2; ++e)
            if (mh_nj[e] == i) mh_nsv[e] = (uint32_t)mh_prop;
        }
        if (p == 0 && has_chain && acc_mh) {
          if (active) ++nflip;
          *tok_at(i) = (unsigned char)mh_prop;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = combine_sites<V, LPC>(acc[e]);
        const uint32_t sg = (uint32_t)(sweep_offset + (uint64_t)sw);
        float l[4];
        float mx = -INFINITY;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool ok = v < NQ && 4 * v + e < Q;
          l[e] = ok ? beta * (hq[e] + acc[e]) : -INFINITY;
          mx = fmaxf(mx, l[e]);
        }
        const int nbase = lane - p;  // first lane of the chain (narrow chains)
        if constexpr (kNarrow)
          mx = narrow_max<LPC>(mx, nbase);
        else
          mx = group_max<V>(mx);
        float P[4];
        float run_sum = 0.0f;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool ok = v < NQ && 4 * v + e < Q;
          run_sum += ok ? __expf(l[e] - mx) : 0.0f;
          P[e] = run_sum;
        }
        // inclusive scan of the quad sums over v; exclusive = shifted by one
        float inc, excl, Stot;
        if constexpr (kNarrow) {
          inc = narrow_scan(run_sum, lane, v);
          excl = __shfl(inc, lane - 1, kWave);
          if (v == 0) excl = 0.0f;
          Stot = __shfl(excl + P[eL], nbase + vL, kWave);  // S_{q-1}
        } else {
          inc = group_scan<V>(run_sum, v);
          excl = V > 1 ? dpp_f<kDppShr1>(inc) : 0.0f;
          if (v == 0) excl = 0.0f;
          Stot = group_bcast<V, vL>(excl + P[eL], v);  // S_{q-1}
        }
        if (!kKeepRnd || (i & 3) == 0)
          rnd = philox4x32_10(make_uint4((uint32_t)i >> 2, sg, cid, 0u), k0, k1);
        const float uz = word_to_uniform(pick_word(rnd, i & 3)) * Stot;
        int cnt = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (v < NQ && 4 * v + e < Q - 1 && excl + P[e] <= uz) ++cnt;
        if constexpr (kNarrow)
          cnt = narrow_sum<LPC>(cnt, nbase);
        else
          cnt = group_sum<V>(cnt);
        // every lane of the chain drew the same state: patch the token of
        // site i in the dwords read ahead for the next site's first chunk
        if (kPipeTok && reader && u == i % S) {
          const int mi = i / S;
#pragma unroll
          for (int d = 0; d < 4; ++d)
            if (min(d, m4 - 1) == (mi >> 2))
              g_tok[d] = (g_tok[d] & ~(0xFFu << (8 * (mi & 3)))) | ((uint32_t)cnt << (8 * (mi & 3)));
        }
        if (p == 0 && has_chain) {
          unsigned char* tp = tok_at(i);
          if (active && cnt != (int)*tp) ++nflip;
          *tp = (unsigned char)cnt;
        }
      }
      acc = f4{0.0f, 0.0f, 0.0f, 0.0f};
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
    for (int j = p; j < L; j += LPC) chains[c * L + j] = (int8_t)*tok_at(j);
  if (flips_out) {
    unsigned long long tot = nflip;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, kWave);
    if (lane == 0 && tot) atomicAdd(flips_out, tot);
  }
}

inline int device_cus() {
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

// Launch arguments of a gather-form call.
struct GatherArgs {
  const float* h;
  const float* Jt;
  int8_t* chains;
  int64_t N;
  int L;
  int sweeps;
  uint64_t seed, sweep_offset;
  float beta;
  unsigned long long* flips_out;
  int32_t* dev_err;
  hipStream_t s;
  const DevCtl* ctl;
};

template <int Q, bool MH, int MAXW>
hipError_t launch_gather_shape(const GatherShape& gs, const GatherArgs& a) {
  // lanes per chain: the planner's rule for (q, draw), or narrow chains
  // (heat-bath, 5..7 quads per row) where the planner takes them
  constexpr int LP = gather_lanes(Q, !MH), LN = gather_narrow_lanes(Q, !MH);
  if (gs.lpc != LP && (LN == 0 || gs.lpc != LN)) return hipErrorInvalidValue;
  // the step schedule is a template parameter: with both in one kernel the
  // compiler scheduled each of them worse (up to 9% slower)
  auto pick = [&](auto lanes, auto paired) {
    constexpr int LL = decltype(lanes)::value;
    constexpr bool PP = decltype(paired)::value;
    return gs.items == 31   ? k_gibbs_gather<Q, 31, LL, MH, MAXW, PP>
           : gs.items == 16 ? k_gibbs_gather<Q, 16, LL, MH, MAXW, PP>
                            : k_gibbs_gather<Q, 8, LL, MH, MAXW, PP>;
  };
  using LPt = std::integral_constant<int, LP>;
  decltype(&k_gibbs_gather<Q, 8, LP, MH, MAXW, false>) kern = pick(LPt{}, std::false_type{});
  if (gs.pair) kern = pick(LPt{}, std::true_type{});
  if constexpr (LN > 0) {
    using LNt = std::integral_constant<int, LN>;
    if (gs.lpc == LN) {
      kern = pick(LNt{}, std::false_type{});
      if constexpr (!MH) {
        if (gs.pair) kern = pick(LNt{}, std::true_type{});
      }
    }
  }
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)gs.lds);
  if (e != hipSuccess) return e;
  const DevCtl& ctl = *a.ctl;
  hipLaunchKernelGGL(kern, dim3(gs.blocks), dim3(gs.waves * 64), gs.lds, a.s, a.h, a.Jt, a.chains,
                     a.N, a.L, gs.jc, gs.nchunk, gs.m4, gs.ahead, gs.nload, gs.slot, gs.cpb,
                     a.sweeps, (uint32_t)a.seed, (uint32_t)(a.seed >> 32), a.sweep_offset, a.beta,
                     a.flips_out, a.dev_err, ctl.epoch, ctl.active, ctl.streams, ctl.count);
  return hipGetLastError();
}

template <bool MH, int MAXW>
hipError_t launch_gather_switch(int q, const GatherShape& gs, const GatherArgs& a) {
  switch (q) {
#define BMDCA_GQ(n) \
  case n:           \
    return launch_gather_shape<n, MH, MAXW>(gs, a);
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

// ----- sampler_w8.hip: heat-bath sweeps with MAXW = 8 (q <= 16, plans of at
// most kGSmallWaves waves)
hipError_t launch_gather_heat_w8(int q, const GatherShape& gs, const GatherArgs& a);
// ----- sampler_w12.hip: heat-bath sweeps with MAXW = 12 (q > 16, plans of at
// most kGMidWaves waves)
hipError_t launch_gather_heat_w12(int q, const GatherShape& gs, const GatherArgs& a);

// Sweeps of the gather form over the laid-out blocks Jt (q = 2..32).
template <bool MH>
hipError_t launch_gather_form(const float* h, const float* Jt, int8_t* chains, int64_t N, int L,
                              int q, int sweeps, uint64_t seed, uint64_t sweep_offset, float beta,
                              unsigned long long* flips_out, int32_t* dev_err, hipStream_t s,
                              const DevCtl& ctl) {
  // A launch on a share of the CUs (one of several models running at once)
  // takes workgroups of at most kGShareChains chains: more, smaller
  // workgroups let the largest models spread onto CUs the others free.
  const int64_t cus = ctl.cu_share > 0 ? std::min<int64_t>(ctl.cu_share, device_cus()) : device_cus();
  GatherShape gs = ctl.cu_share > 0 ? gather_plan(N, L, q, cus, kGShareChains, !MH)
                                    : gather_plan(N, L, q, cus, kGMaxWaves * 8, !MH);
  // On a CU share the other models' launches compete for L2 and the MALL, and
  // the third chunk in flight pays more than the halved barriers (64 models
  // trained together: 484.6 ms per epoch with paired steps, 460.7 without)
  if (ctl.cu_share > 0) gs.pair = 0;
  if (gs.waves == 0 || gs.ahead != 3) return hipErrorInvalidValue;
  const GatherArgs a{h, Jt, chains, N, L, sweeps, seed, sweep_offset, beta, flips_out, dev_err,
                     s, &ctl};
  if constexpr (!MH) {
    if (q <= 16 && gs.waves <= kGSmallWaves) return launch_gather_heat_w8(q, gs, a);
    if (q > 16 && gs.waves <= kGMidWaves) return launch_gather_heat_w12(q, gs, a);
  }
  return launch_gather_switch<MH, kGMaxWaves>(q, gs, a);
}

}  // namespace bmdca
