// Launch shape of the gather-form Gibbs sampler: chains per workgroup,
// lanes per chain, chunk length, LDS ring and load counts.  Plain host C++
// (the constexpr helpers are also used by the kernels), so that a CPU
// program can check every planned shape against the kernel's index ranges.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>

namespace bmdca {

constexpr int64_t gp_ceil(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr int kGMaxWaves = 16;   // waves per workgroup at most
constexpr int kGSmallWaves = 8;  // plans with q <= 16 and at most this many waves run a
                                 // kernel bound to 8 waves (256 VGPRs)
constexpr int kGMidWaves = 12;   // heat-bath plans with q > 16 and at most this many waves
                                 // run a kernel bound to 12 waves (168 VGPRs: the 16-wave
                                 // bound of 128 spills two of them to scratch)
constexpr int kGMinWaves = 4;    // and at least
// Chains per workgroup at most for a launch on a share of the CUs (grouped
// training of 64 models over 8 lanes: caps of 32, 64 and 128 chains measured
// 909, 575 and 1163 ms per epoch).
constexpr int kGShareChains = 64;
constexpr size_t kGLds = 160 * 1024 - 256;
constexpr size_t kGAlign = 128;  // chunk boundaries on whole cache lines of the run

// Row pitch of Jt: q rounded up to a multiple of 4 floats (16-byte quads).
constexpr int gather_qp(int q) { return (q + 3) & ~3; }
// Lanes per quad group: quads per row rounded up to a power of two.
constexpr int gather_v(int q) {
  return gather_qp(q) / 4 <= 1 ? 1 : gather_qp(q) / 4 <= 2 ? 2 : gather_qp(q) / 4 <= 4 ? 4 : 8;
}
// Site groups per chain of `lpc` lanes (8 or 16; a narrow chain, one lane
// per quad of its row, has one).
constexpr int gather_s(int q, int lpc) { return lpc >= gather_v(q) ? lpc / gather_v(q) : 1; }

struct GatherShape {
  int lpc;        // lanes per chain (8 or 16)
  int waves;      // waves per workgroup
  int cpb;        // chains per workgroup
  int jc;         // sites per chunk (multiple of 4 S)
  int nchunk;     // chunks per site
  int m4;         // token dwords per (chain, site group)
  int ahead;      // chunks in flight (ring = ahead + 1 slots)
  int items;      // 1 KB loads per loading wave per chunk: 8, 16 or 31, a template
                  // parameter so that every wait is an immediate (31 keeps two
                  // younger chunks within vmcnt's range)
  int nload;      // loading waves (waves 0..nload-1; wave w loads blocks w*items ...)
  int slot;       // floats per ring slot (nload * items KB)
  size_t lds;     // dynamic LDS bytes
  unsigned blocks;
  int pair;       // 1: paired chunk-steps (one barrier per two steps, two chunks in flight)
};

// Token bytes per chain.
inline size_t gather_tok_bytes(int L, int q, int lpc) {
  const int S = gather_s(q, lpc);
  return (size_t)S * (size_t)gp_ceil(gp_ceil(L, S), 4) * 4;
}

// Shape for `cpb` chains per workgroup and a ring of `nslot` slots; waves = 0
// if it does not fit.  `align` asks for chunks on 256-byte boundaries.
inline GatherShape gather_shape_n(int L, int q, int cpb, int nslot, int lpc, bool align) {
  GatherShape g{};
  const int S = gather_s(q, lpc);
  const size_t site_row = (size_t)q * gather_qp(q) * sizeof(float);  // bytes per site of a chunk
  // at least 4 waves, one per SIMD, to spread the chunk loads and barriers
  g.lpc = lpc;
  g.waves = std::max<int>(kGMinWaves, (int)gp_ceil(cpb, 64 / lpc));
  if (g.waves < 1 || g.waves > kGMaxWaves) return GatherShape{};
  const size_t tok = gather_tok_bytes(L, q, lpc) * (size_t)(g.waves * (64 / lpc));
  if (tok >= kGLds) return GatherShape{};
  const size_t per_slot = std::min((kGLds - tok) / nslot, (size_t)31 * g.waves * 1024);
  // Chunks are a multiple of 4 S sites (4 token positions per lane, one
  // token dword) and of kGAlign bytes: a chunk that starts off a 128-byte
  // boundary of the run makes every load of it misaligned (L = 100, q = 21:
  // 17-site chunks, 34272 bytes, took 1.8x the time per sweep of 16-site
  // ones).  A 256-byte rule costs steps for nothing: at q = 21 it takes
  // 8-site chunks where 12 fit (L = 512: 64 chunk-steps per site instead of
  // 43; 39.6 against 25.0 ms per sweep for 10 000 chains on 32 CUs).
  int step = 4 * S;
  while (align && ((size_t)step * site_row) % kGAlign != 0) step += 4 * S;
  const int lcap = (int)gp_ceil(L, 4 * S) * 4 * S;
  // the largest chunk whose padded slots and tokens fit (a chunk of the
  // whole run needs no alignment)
  for (int jc = std::min((int)(per_slot / site_row) / (4 * S) * (4 * S), lcap); jc >= 4 * S;
       jc -= 4 * S) {
    g.nchunk = (int)gp_ceil(L, jc);
    g.jc = (int)gp_ceil(gp_ceil(L, g.nchunk), 4 * S) * 4 * S;  // balanced chunks
    if (g.nchunk > 1) g.jc = (int)gp_ceil(g.jc, step) * step;
    if (g.jc > jc) continue;
    g.nchunk = (int)gp_ceil(L, g.jc);
    g.m4 = (int)gp_ceil(gp_ceil(L, S), 4);
    g.ahead = nslot - 1;
    g.cpb = cpb;
    const int nblk = (int)gp_ceil((size_t)g.jc * site_row, 1024);
    for (int it : {8, 16, 31}) {  // the least padding that the waves can load
      if ((nslot - 2) * it > 63) continue;  // vmcnt range of the younger chunks
      g.items = it;
      g.nload = (int)gp_ceil(nblk, it);
      g.slot = g.nload * it * 256;
      g.lds = (size_t)nslot * g.slot * sizeof(float) + tok;
      if (g.nload <= g.waves && g.lds <= kGLds) return g;
    }
  }
  return GatherShape{};
}

// A ring of 4 slots: three chunks in flight.  Measured at L = 100..512,
// q = 21: 3 slots (larger chunks, two in flight) take 1.4-1.8x as long per
// sweep, 5, 6 or 8 slots (smaller chunks, more steps) 1.5-2.5x.
inline GatherShape gather_shape(int L, int q, int cpb, int lpc) {
  const GatherShape g = gather_shape_n(L, q, cpb, 4, lpc, true);
  // unaligned chunks only where no aligned shape fits (q = 25 or 27 at large
  // L, or large L with many chains' tokens in the LDS)
  return g.waves ? g : gather_shape_n(L, q, cpb, 4, lpc, false);
}

// Lanes per chain (8 or 16): a function of q and the draw alone, never of
// the chain count or the CU share, because the FP32 summation order of a
// chain's local fields follows its lanes -- with this rule a chain draws the
// same bits in bmdca_gibbs, in a grouped epoch on a CU share and in a merged
// bmdca_gibbs_streams launch.  8 lanes for q > 8 (16 cost 1.9x at q = 21:
// the per-wave step overhead doubles).  For q <= 8 (rows of at most two
// quads) the heat-bath draw also takes 8: its 8-wave kernel reads tokens a
// step ahead, which outweighs the halved lanes (q = 5, L = 400, 10 000
// chains: 23.6 against 28.2 ms per 10 sweeps; q = 8, L = 60: 0.78 against
// 1.16; with 4096 chains on the whole device 16 lanes were 13% faster, the
// price of the fixed rule).  Metropolis, which runs the 16-wave kernel,
// takes 16 (q = 5, L = 400, 10 000 chains: 24.0 against 27.2 ms).
constexpr int gather_lanes(int q, bool small) { return (gather_v(q) <= 2 && !small) ? 16 : 8; }

// Narrow heat-bath chains: rows of 5, 6 or 7 quads (q = 17..28) can also run
// with one lane per quad, 12, 10 or 9 chains per wave instead of 8, so no
// lane of the row gathers idles (q = 21: 6 of 8 lanes would).  Each lane adds
// its quad over the positions in the same order as in an 8-lane chain, and
// the draw's cross-lane steps keep the 8-lane association order, so a narrow
// chain draws the same bits as an 8-lane one (checked over whole runs): the
// choice may follow the launch shape.  The planner takes it where it saves
// waves and still leaves at least kGNarrowWaves, two per SIMD (L = 256,
// q = 21, 20 000 chains: 8 waves instead of 10, 33.5 against 39.6 ms per 10
// sweeps; with one wave per SIMD it lost: L = 100, 10 000 chains, 4 instead
// of 5 waves, 5.71 against 5.45 ms; 7 instead of 8 waves was mixed, 16 384
// chains: +2.4% at L = 100, +1.3% at L = 256, -3.9% at L = 512).
constexpr int kGNarrowWaves = 8;
constexpr int gather_narrow_lanes(int q, bool small) {
  return (small && gather_v(q) == 8 && gather_qp(q) / 4 < 8) ? gather_qp(q) / 4 : 0;
}

// Paired chunk-steps: the ring of 4 slots is refilled two chunks at a time,
// one wait and one barrier per two steps, with two chunks in flight instead
// of three.  Where a workgroup holds at least this many chains the row
// gathers dominate a step and the halved barriers pay (L = 256, q = 21,
// 20 000 chains: 33.6 -> 30.2 ms per 10 sweeps; L = 100, 10 000 chains
// 5.46 -> 5.27; q = 12, L = 200 11.4 -> 10.0; q = 5, L = 400 17.8 -> 16.0;
// Metropolis sweeps, whose staging is most of the step: L = 100 4.30 -> 3.96,
// L = 256 24.0 -> 21.9, q = 5, L = 400 24.2 -> 22.4, q = 12, L = 200
// 9.14 -> 8.52);
// with fewer the staging latency dominates and the third chunk in flight
// pays more (L = 512, 4096 chains, 16 per workgroup: 114.7 against 130.8).
// The same holds where the re-laid-out couplings (L^2 q QP 4 bytes) exceed
// the 256 MB last-level cache and the staging comes from HBM, unless the
// workgroup holds at least twice as many chains (10 000 chains, 40 per
// workgroup: L = 400 (323 MB) 71.0 against 79.9 ms, L = 512 (528 MB) 115.3
// against 130.3; L = 300 (181 MB) 41.0 against 40.6; L = 512, 20 000 chains,
// 80 per workgroup: 254.9 against 246.2).  Launches on a share of the CUs
// keep one barrier per step (the launch clears the flag).  The chains draw
// the same bits either way.
constexpr int kGPairChains = 32;
constexpr double kGPairCacheBytes = 256.0 * 1024 * 1024;
inline int gather_pair(int L, int q, int cpb) {
  const double jt = (double)L * L * q * gather_qp(q) * sizeof(float);
  return (cpb >= kGPairChains && (jt <= kGPairCacheBytes || cpb >= 2 * kGPairChains)) ? 1 : 0;
}

// Chains per workgroup for chains of `lpc` lanes: spread the chains over the
// CUs (one workgroup per CU at a time) in as few rounds as the largest
// workgroup that fits allows.
inline GatherShape gather_plan_lanes(int64_t N, int L, int q, int64_t cus, int cap, int lpc) {
  const int cpw = 64 / lpc;  // chains per wave
  int cmax = std::min(cap, kGMaxWaves * cpw);
  while (cmax > cpw && gather_shape(L, q, cmax, lpc).waves == 0) cmax -= cpw;
  const int64_t rounds = gp_ceil(N, cus * cmax);
  const int cpb = (int)std::min<int64_t>(cmax, gp_ceil(N, rounds * cus));
  GatherShape g = gather_shape(L, q, cpb, lpc);
  g.blocks = (unsigned)gp_ceil(N, (int64_t)cpb);
  g.pair = g.waves > 0 ? gather_pair(L, q, g.cpb) : 0;
  return g;
}

inline GatherShape gather_plan(int64_t N, int L, int q, int64_t cus, int cap = kGMaxWaves * 8,
                               bool small = true) {
  GatherShape g = gather_plan_lanes(N, L, q, cus, cap, gather_lanes(q, small));
  const int nl = gather_narrow_lanes(q, small);
  if (nl > 0 && g.waves > kGNarrowWaves) {
    const GatherShape n = gather_plan_lanes(N, L, q, cus, cap, nl);
    if (n.waves >= kGNarrowWaves && n.waves < g.waves && n.blocks <= g.blocks) g = n;
  }
  return g;
}

}  // namespace bmdca
