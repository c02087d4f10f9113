// Launchers shared between the kernel sources and the C-ABI entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace bmdca {

// Random stream of one chain (the public bmdca_chain_stream): the chain
// draws as chain `chain` of a call with key `seed` and `sweep_offset`.
struct ChainStream {
  uint64_t seed;
  uint64_t sweep_offset;
  uint32_t chain;
  uint32_t reserved;
};

// Device-side controls of a launch.  All fields are optional: with the
// defaults a launch behaves as a plain call.
struct DevCtl {
  const uint64_t* epoch = nullptr;  // sampler sweep offset += *epoch * sweeps
  const int32_t* active = nullptr;  // *active == 0: the kernel returns at once
  int cu_share = 0;                 // CUs the sampler grid is sized for (0: all)
  const ChainStream* streams = nullptr;  // per-chain random streams (sampler)
  const int64_t* count = nullptr;   // live chains: only chains < min(N, *count) are swept
  bool keep_layout = false;         // gather form: the workspace already holds the
                                    // re-laid-out couplings of this J
};

// ----- sampler.hip
hipError_t launch_init_chains(int8_t* chains, int64_t N, int L, int q, uint64_t seed,
                              hipStream_t s);
// H[c][r] = h[r] + sum_{k != r/q} J[(k, chains[c][k])][r] for c < N.
// count (optional, device): only chains < min(N, *count).
hipError_t launch_local_fields(const float* h, const float* J, const int8_t* chains, int64_t N,
                               int L, int q, float* H, int32_t* dev_err, hipStream_t s,
                               const int32_t* active = nullptr, const int64_t* count = nullptr);
hipError_t launch_gibbs_sweeps(const float* J, int8_t* chains, float* H, int64_t N, int L, int q,
                               int sweeps, uint64_t seed, uint64_t sweep_offset, float beta,
                               unsigned long long* flips_out, hipStream_t s,
                               const DevCtl& ctl = DevCtl(), bool metropolis = false);
// Gather form (local fields recomputed per visit from LDS-staged coupling
// blocks); needs no field workspace.  metropolis = true: single-site
// Metropolis instead of the heat-bath draw.
bool gather_supported(int L, int q);
size_t gather_ws_bytes(int L, int q);  // re-laid-out coupling blocks
hipError_t launch_gibbs_gather(const float* h, const float* J, int8_t* chains, int64_t N, int L,
                               int q, int sweeps, uint64_t seed, uint64_t sweep_offset, float beta,
                               unsigned long long* flips_out, int32_t* dev_err, void* ws,
                               hipStream_t s, const DevCtl& ctl = DevCtl(),
                               bool metropolis = false);
// ----- sampler_mh.hip: the Metropolis sweeps over laid-out blocks Jt
hipError_t launch_gather_metropolis(const float* h, const float* Jt, int8_t* chains, int64_t N,
                                    int L, int q, int sweeps, uint64_t seed,
                                    uint64_t sweep_offset, float beta,
                                    unsigned long long* flips_out, int32_t* dev_err,
                                    hipStream_t s, const DevCtl& ctl);

// ----- stats.hip
// Workspace carve-up of the one-hot statistics product for M rows.
struct StatsPlan {
  int64_t Mpad;     // rows padded to the K stage
  int ntile;        // output tiles per side
  int nupper;       // upper-triangle tiles
  int splits;       // K splits (FP64 partial planes)
  int64_t kchunk;   // rows per split (multiple of the K stage)
  size_t off_xt, off_whi, off_wlo, off_wf, off_part, off_red, total;
};
StatsPlan plan_stats(int64_t M, int L, int q, int prec);

// X [M][L] -> XT [L][Mpad] (Mpad a multiple of 64); padding rows and invalid
// tokens become -1, invalid tokens also raise BMDCA_DEVERR_TOKEN.
// count (optional, device): rows >= min(M, *count) are treated as padding.
hipError_t launch_transpose_tokens(const int8_t* X, int64_t M, int L, int q, int8_t* XT,
                                  int64_t Mpad, int32_t* dev_err, hipStream_t s,
                                  const int64_t* count = nullptr);

// Statistics product: partial planes P[s][Lq][Lq] (upper tiles only) of
// sum_m w_m [x_mi == a][x_mj == b].  w == nullptr: unit weights.
hipError_t launch_onehot_products(const int8_t* X, const double* w, int64_t M, int L, int q,
                                  int prec, const StatsPlan& plan, void* ws, int32_t* dev_err,
                                  hipStream_t s, const int32_t* active = nullptr);
// Chain counts C[(i,a)][(j,b)] = #{n : s_i(n) = a, s_j(n) = b} (unit weights,
// exact), full symmetric FP64 [Lq][Lq], counted directly in LDS histograms;
// uses the token region of a plan_stats(N, L, q, .) workspace.  q <= 32.
hipError_t launch_pair_counts(const int8_t* X, int64_t N, int L, int q, const StatsPlan& plan,
                              void* ws, double* C, int32_t* dev_err, hipStream_t s,
                              const int32_t* active = nullptr);
// Sum of the partial planes into the full symmetric matrix C (FP64).
hipError_t launch_reduce_partials(const StatsPlan& plan, const void* ws, int Lq, double* C,
                                  hipStream_t s);
// M_eff = sum_m w_m (fixed order) into *meff; unit weights give M exactly.
hipError_t launch_meff(const double* w, int64_t M, double* meff, hipStream_t s);
// f1, f2 with pseudocount from the partial planes.
hipError_t launch_stats_epilogue(const StatsPlan& plan, const void* ws, int L, int q,
                                 const double* meff, double pseudocount, double* f1, double* f2,
                                 hipStream_t s);

// ----- learn.hip
// Pearson coefficient of the connected correlations (Eq. 6); `red` needs
// pearson_red_bytes().
size_t pearson_red_bytes();
hipError_t launch_pearson(const double* f1, const double* f2, const double* C, int64_t N, int L,
                          int q, double* red, double* out, int32_t* dev_err, hipStream_t s);
hipError_t launch_update(float* h, float* J, const double* f1, const double* f2, const double* C,
                         int64_t N, int L, int q, double lr, int32_t* dev_err, hipStream_t s,
                         const int32_t* active = nullptr, const uint8_t* mask = nullptr);
// Group epoch epilogue of one model: if active, epoch += 1 and, with a
// positive target, active = 0 once the Pearson coefficient reaches it.
hipError_t launch_ctl_advance(void* ctl, const double* pearson, hipStream_t s);
// *tick += 1 (one thread): the sweep counter of a replayed sampling launch.
hipError_t launch_tick_advance(uint64_t* tick, hipStream_t s);
// h = (float) log f1 (the profile model's fields).
hipError_t launch_profile_fields(const double* f1, int L, int q, float* h, int32_t* dev_err,
                                 hipStream_t s);

// ----- reweight.hip
struct ReweightPlan {
  int planes, words;
  int64_t Mpad;
  size_t off_planes, off_red, total;
};
ReweightPlan plan_reweight(int64_t M, int L, int q);
hipError_t launch_reweight(const int8_t* msa, int64_t M, int L, int q, int32_t T,
                           const ReweightPlan& plan, void* ws, int32_t* n_sim, double* w,
                           double* meff, int32_t* dev_err, hipStream_t s);

// ----- scoring.hip
// Energy workspace: site-major tokens and per-part FP64 pair sums.
struct EnergyPlan {
  int64_t Bpad;    // sequences padded to 64
  int64_t steps;   // (column chunk, row site) steps over all pairs i < j
  int parts;       // contiguous step ranges (a function of L only)
  size_t off_xt, off_part, total;
};
EnergyPlan plan_energy(int64_t B, int L, int q);
// count (optional, device): only sequences < min(B, *count) are scored (the
// launch is sized for B; E past the count is left as it is).
hipError_t launch_energy(const float* h, const float* J, const int8_t* seqs, int64_t B, int L,
                         int q, float* E, const EnergyPlan& plan, void* ws, int32_t* dev_err,
                         hipStream_t s, const int64_t* count = nullptr);
hipError_t launch_mutant_delta(const float* H, const int8_t* wt, int64_t B, int L, int q,
                               float* dE, hipStream_t s, const int64_t* count = nullptr);
size_t apc_ws_bytes(int L);
hipError_t launch_apc(const float* J, int L, int q, int gap, float* F, float* Fapc, void* ws,
                      hipStream_t s);

// ----- decimation.hip
size_t dec_ws_bytes(int L, int q);
// One edDCA graph update from the chain counts C (FP64 [Lq][Lq]).
hipError_t launch_decimate(float* J, uint8_t* mask, const double* C, int64_t N, int L, int q,
                           double drate, double density, long long* n_active_out, void* ws,
                           hipStream_t s);
// One eaDCA graph update from the chain counts C and the data frequencies f2.
hipError_t launch_activate(uint8_t* mask, const double* C, const double* f2, int64_t N, int L,
                           int q, double factivate, long long* n_active_out, void* ws,
                           int32_t* dev_err, hipStream_t s);

// Coupling graphs: mask = the full graph (full != 0, 1 off the diagonal
// blocks) or the empty one; J = 0 off the graph, active elements r1 < r2
// counted into *n_active (optional).
hipError_t launch_mask_init(uint8_t* mask, int L, int q, int full, hipStream_t s);
hipError_t launch_mask_apply(float* J, const uint8_t* mask, int L, int q, long long* n_active,
                             hipStream_t s);

// ----- equilibrium.hip
size_t draw_ws_bytes(int64_t M);
size_t seqid_ws_bytes();
hipError_t launch_draw_rows(const double* w, int64_t M, int64_t n, uint64_t seed, int32_t* rows,
                            void* ws, int32_t* dev_err, hipStream_t s);
hipError_t launch_gather_rows(const int8_t* X, int64_t M, int L, const int32_t* rows, int64_t n,
                              int8_t* out, int32_t* dev_err, hipStream_t s);
hipError_t launch_seqid(const int8_t* A, const int8_t* B, const int32_t* perm, int64_t N, int L,
                        double* out, void* ws, int32_t* dev_err, hipStream_t s);

}  // namespace bmdca
