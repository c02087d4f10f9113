// CPU check of every launch shape the gather-form sampler plans: the index
// ranges the kernel derives from a shape (ring slots, chunk loads, row reads,
// token dwords, LDS total, vmcnt range) stay inside what the shape allocates,
// and the chunks cover every site once.  Exit status 0 when all hold.
#include <cstdio>
#include <set>
#include <vector>

#include "../paper_2501_18456_amd/csrc/gather_plan.hpp"

using namespace bmdca;

static int failures = 0;
#define CHECK(cond, ...)                                              \
  do {                                                                \
    if (!(cond)) {                                                    \
      if (failures < 20) {                                            \
        std::printf("FAIL %s: N=%lld L=%d q=%d cus=%lld cap=%d: ", #cond, (long long)N, L, q, \
                    (long long)cus, cap);                             \
        std::printf(__VA_ARGS__);                                     \
        std::printf("\n");                                            \
      }                                                               \
      ++failures;                                                     \
      return;                                                         \
    }                                                                 \
  } while (0)

static void check(int64_t N, int L, int q, int64_t cus, int cap, bool small) {
  const GatherShape g = gather_plan(N, L, q, cus, cap, small);
  // lanes per chain: fixed by q and the draw (8; 16 for Metropolis at q <= 8),
  // whatever the chain count, CU share and cap
  // or narrow heat-bath chains (one lane per quad, q = 17..28) in plans of at
  // least kGNarrowWaves waves
  const int nq = gather_qp(q) / 4;
  const int want = (gather_v(q) <= 2 && !small) ? 16 : 8;
  const bool narrow_ok = small && gather_v(q) == 8 && nq < 8;
  CHECK(g.lpc == want || (narrow_ok && g.lpc == nq && g.waves >= kGNarrowWaves),
        "lpc %d, expected %d (q %d, cpb %d, small %d)", g.lpc, want, q, g.cpb, (int)small);
  CHECK(g.waves >= kGMinWaves && g.waves <= kGMaxWaves, "waves %d", g.waves);
  CHECK(g.lpc == 8 || g.lpc == 16 || (g.lpc >= 5 && g.lpc <= 7 && g.lpc == nq && small),
        "lpc %d", g.lpc);
  const int S = gather_s(q, g.lpc), QP = gather_qp(q), NQ = QP / 4;
  const int CPW = 64 / g.lpc, CPB = g.waves * CPW;  // chains per wave, per workgroup
  // a narrow chain has one lane per quad and one site group
  if (g.lpc < 8) CHECK(S == 1 && NQ == g.lpc && CPW * g.lpc <= 64, "narrow S %d NQ %d", S, NQ);
  CHECK(g.cpb >= 1 && g.cpb <= CPB && g.cpb <= cap, "cpb %d of %d", g.cpb, CPB);
  CHECK((int64_t)g.blocks * g.cpb >= N && (int64_t)(g.blocks - 1) * g.cpb < N, "blocks %u", g.blocks);
  CHECK(g.ahead == 3, "ahead %d", g.ahead);
  // paired chunk-steps (two chunks in flight, refilled two at a time) in the
  // same ring of ahead + 1 = 4 slots, where the workgroup holds enough chains
  {
    const double jt = (double)L * L * q * QP * 4.0;
    const bool want_pair = g.cpb >= 32 && (jt <= 256.0 * 1024 * 1024 || g.cpb >= 64);
    CHECK(g.pair == (want_pair ? 1 : 0), "pair %d cpb %d small %d jt %.0f", g.pair, g.cpb,
          (int)small, jt);
  }
  CHECK(g.items == 8 || g.items == 16 || g.items == 31, "items %d", g.items);
  CHECK((g.ahead - 1) * g.items <= 63, "vmcnt %d", (g.ahead - 1) * g.items);
  CHECK(g.nload >= 1 && g.nload <= g.waves, "nload %d", g.nload);
  CHECK(g.slot == g.nload * g.items * 256, "slot %d", g.slot);
  CHECK(g.jc % (4 * S) == 0 && g.jc >= 4 * S, "jc %d S %d", g.jc, S);
  CHECK(g.nchunk == (int)gp_ceil(L, g.jc), "nchunk %d", g.nchunk);
  CHECK(g.m4 == (int)gp_ceil(gp_ceil(L, S), 4), "m4 %d", g.m4);
  const size_t tok_dwords = (size_t)S * g.m4 * CPB;
  CHECK(g.lds == (size_t)(g.ahead + 1) * g.slot * 4 + tok_dwords * 4, "lds %zu", g.lds);
  CHECK(g.lds <= kGLds, "lds %zu > %zu", g.lds, kGLds);
  // chunk loads: loading wave w issues blocks w*items .. w*items + items-1 of 1 KB
  const size_t chunk_bytes = (size_t)g.jc * q * QP * 4;
  CHECK(chunk_bytes <= (size_t)g.slot * 4, "chunk %zu slot %d", chunk_bytes, g.slot);
  CHECK((size_t)(g.nload * g.items) * 1024 <= (size_t)g.slot * 4, "loads past the slot");
  // row reads: float (S r + u) q QP + s QP + 4 v + 3 within a slot
  const int jcs = g.jc / S;
  const int64_t last = ((int64_t)(S * (jcs - 1) + S - 1) * q + (q - 1)) * QP + 4 * (NQ - 1) + 3;
  CHECK(last < g.slot, "row read %lld slot %d", (long long)last, g.slot);
  // tokens: every position read (clamped to m4 - 1) lies in the token array,
  // every site j < L is read at a position whose dword exists, once
  std::vector<int> seen(L, 0);
  for (int k = 0; k < g.nchunk; ++k) {
    const int m0 = k * jcs;
    CHECK(m0 % 4 == 0, "m0 %d", m0);
    for (int u = 0; u < S; ++u)
      for (int r = 0; r < jcs; ++r) {
        const int d = std::min((m0 + r) / 4, g.m4 - 1);
        const size_t dw = ((size_t)u * g.m4 + d) * CPB + (CPB - 1);
        CHECK(dw < tok_dwords, "token dword %zu of %zu", dw, tok_dwords);
        const int j = k * g.jc + S * r + u;
        if (j < L) {
          CHECK((m0 + r) / 4 < g.m4, "site %d token dword %d", j, (m0 + r) / 4);
          ++seen[j];
        }
      }
  }
  for (int j = 0; j < L; ++j) CHECK(seen[j] == 1, "site %d read %d times", j, seen[j]);
  // chunks start on kGAlign-byte boundaries of the run unless no aligned shape fits
  const size_t site_row = (size_t)q * QP * 4;
  if (g.nchunk > 1 && (g.jc * site_row) % kGAlign != 0)
    CHECK(gather_shape_n(L, q, g.cpb, 4, g.lpc, true).waves == 0, "misaligned chunk");
}

int main() {
  std::vector<int> Ls;
  for (int L = 1; L <= 40; ++L) Ls.push_back(L);
  for (int L : {50, 64, 99, 100, 101, 127, 128, 200, 255, 256, 257, 300, 385, 400, 511, 512})
    Ls.push_back(L);
  int shapes = 0;
  for (int q = 2; q <= 32; ++q)
    for (int L : Ls) {
      if (gather_shape(L, q, 1, 8).waves == 0) {
        std::printf("FAIL unsupported L=%d q=%d\n", L, q);
        ++failures;
        continue;
      }
      for (int64_t n : {1, 7, 100, 1000, 4096, 10000, 20000, 40000, 100000})
        for (int64_t c : {256, 32})
          for (int cp : {128, kGShareChains})
            for (bool small : {true, false}) {  // heat-bath and Metropolis plans
              check(n, L, q, c, cp, small);
              ++shapes;
            }
    }
  std::printf("%d shapes checked, %d failures\n", shapes, failures);
  return failures == 0 ? 0 : 1;
}
