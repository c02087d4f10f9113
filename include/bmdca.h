/*
 * bmdca.h -- C ABI of libbmdca, the MI355X (gfx950) implementation of the
 * Boltzmann-machine DCA training hot path of adabmDCA 2.0 (arXiv:2501.18456).
 *
 * Storage conventions (every call):
 *   - Tokens are int8 in 0..q-1; token 0 is the alignment gap (Table 1 lists
 *     the gap first).  Alignments and chains are row-major [rows][L].
 *   - The one-hot vertex (i, a) of Sec. 2.1 has flat index r = i*q + a;
 *     Lq = L*q.
 *   - Fields h: float32 [Lq].  Couplings J: float32 [Lq][Lq], full-symmetric
 *     (J[(i,a),(j,b)] == J[(j,b),(i,a)]) with all-zero diagonal blocks J_ii,
 *     the two constraints stated with Eq. (1).  Every kernel skips j == i, so
 *     a non-zero diagonal block is ignored, never used.
 *   - Energy (Eq. 1): E(s) = -sum_i h_i(s_i) - sum_{i<j} J_ij(s_i, s_j);
 *     each unordered pair is counted once.
 *
 * Memory and streams:
 *   - Every array argument is a DEVICE pointer owned by the caller, unless
 *     its comment says otherwise.  The library allocates nothing: scratch
 *     memory comes in through `ws` (size from bmdca_workspace_bytes).
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Every
 *     call only enqueues work on it and returns; results are ready once the
 *     stream has been synchronised.
 *   - The library keeps no hidden state between calls, apart from the lane
 *     streams of the group calls (created once per device) and graph
 *     handles the caller owns.  Calls on different streams do not share
 *     memory unless the caller passes the same buffers.
 *
 * Errors:
 *   - Host-side validation (null pointers, sizes, q outside 2..32, theta
 *     outside [0,1], non-finite lr, workspace too small) returns a negative
 *     status at once, before anything is enqueued.
 *   - Conditions only the device can see are OR-ed into *dev_err (a device
 *     int32 that the caller zeroes and reads after synchronising):
 *     BMDCA_DEVERR_TOKEN for a token outside 0..q-1 (the caller's duty under
 *     pre-processing step p.1, Sec. 2.3), BMDCA_DEVERR_NONFINITE for a
 *     non-finite parameter or Pearson value.  dev_err may be NULL where noted.
 *   - A failed kernel launch returns BMDCA_EHIP; bmdca_last_error() then
 *     gives the text.  The library never aborts the process.
 */
#ifndef BMDCA_H
#define BMDCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BMDCA_OK = 0,
    BMDCA_EINVAL = -1,     /* bad argument (null pointer, size, range) */
    BMDCA_ETOKEN = -2,     /* reserved for host-checked token errors */
    BMDCA_EWORKSPACE = -3, /* ws_bytes smaller than bmdca_workspace_bytes() */
    BMDCA_EHIP = -4,       /* a HIP call or kernel launch failed */
    BMDCA_ENONFINITE = -5  /* non-finite learning rate or beta */
} bmdca_status;

/* Arithmetic of the two-site statistics product (Eq. 3). */
typedef enum {
    BMDCA_PREC_FP32 = 0,  /* FP32 matrix cores, FP32 weights */
    BMDCA_PREC_BF16X2 = 1 /* BF16 matrix cores; one-hot operands are exact in
                             BF16, each weight is split w = hi + lo into two
                             BF16 parts (two products), FP32 accumulation over
                             chunks of at most 1024 rows flushed into FP64 */
} bmdca_prec;

/* Sampler selection and options, OR-ed into the `flags` argument of
 * bmdca_gibbs, the `prec` argument of bmdca_train_step, and the `prec`
 * argument of bmdca_workspace_bytes for BMDCA_WS_GIBBS / BMDCA_WS_TRAIN_STEP.
 * Without a sampler bit the library picks the gather form whenever the model
 * fits it (L <= 512, q <= 32) and the field form otherwise.  Both forms use
 * the same draw rule and Philox counters; they differ only in FP32 rounding
 * of the local fields. */
#define BMDCA_SAMPLER_FIELDS 0x10 /* per-chain local fields H in HBM, updated
                                     incrementally on every accepted change */
#define BMDCA_SAMPLER_GATHER 0x20 /* local fields recomputed at every visit
                                     from coupling blocks staged in LDS,
                                     chains of a workgroup in lockstep */
#define BMDCA_GIBBS_KEEP_FIELDS 0x40 /* field form only: H_ws already holds
                                        the fields of these chains */
#define BMDCA_GIBBS_KEEP_LAYOUT 0x100 /* gather form only: H_ws already holds
                                        the re-laid-out couplings of this J (left
                                        by a previous call on the same buffers),
                                        so the per-call copy is skipped -- for
                                        repeated sampling of a fixed model */
#define BMDCA_SAMPLER_METROPOLIS 0x80 /* single-site Metropolis instead of the
                                        heat-bath draw, in either form (with
                                        BMDCA_SAMPLER_FIELDS or _GATHER, or
                                        picked as above): at site i in
                                        state a propose a' uniformly among the
                                        q-1 other states, Philox counter
                                        (i/2, sweep, chain, 3), word 2(i%2):
                                        a' = (a + 1 + ((w (q-1)) >> 32)) mod q;
                                        accept iff u < exp(beta (H_i(a') -
                                        H_i(a))), u = (w' >> 8) 2^-24 from word
                                        2(i%2)+1.  The paper names the option
                                        without its rule; this is the textbook
                                        rule. */

/* Chain counts of bmdca_train_step (and its grouped and masked forms): by
 * default they are counted directly, #{n : s_i(n) = a, s_j(n) = b} in
 * integer histograms; with this bit OR-ed into `prec` they come from the
 * one-hot product of that precision instead (for comparing the two product
 * forms).  Both give the same exact integers, so every result is
 * bit-identical either way. */
#define BMDCA_COUNTS_PRODUCT 0x200

/* Bits OR-ed into *dev_err. */
#define BMDCA_DEVERR_TOKEN 1
#define BMDCA_DEVERR_NONFINITE 2
#define BMDCA_DEVERR_INDEX 4 /* a row index or permutation entry out of range */

/* Workspace kinds for bmdca_workspace_bytes. */
typedef enum {
    BMDCA_WS_REWEIGHT = 0,   /* MN = M (alignment rows) */
    BMDCA_WS_STATS = 1,      /* MN = M */
    BMDCA_WS_GIBBS = 2,      /* MN = N (chains) */
    BMDCA_WS_TRAIN_STEP = 3, /* MN = N */
    BMDCA_WS_APC = 4,        /* MN ignored */
    BMDCA_WS_MUTANT = 5,     /* MN = B (wild types) */
    BMDCA_WS_ENERGY = 6,     /* MN = B (sequences) */
    BMDCA_WS_DRAW = 7,       /* MN = M (weights); L, q ignored but must be valid */
    BMDCA_WS_SEQID = 8,      /* MN ignored */
    BMDCA_WS_DECIMATE = 9    /* MN = N (chains) */
} bmdca_ws_kind;

/* Bytes of device scratch memory the call `kind` needs for these sizes
 * (0 for an invalid request).  Any buffer at least this large, 256-byte
 * aligned, may be passed as `ws`. */
size_t bmdca_workspace_bytes(int32_t kind, int64_t MN, int32_t L, int32_t q,
                             int32_t prec);

/* Text of the last non-OK status returned on this host thread. */
const char* bmdca_last_error(void);

/* Integer identity threshold used by bmdca_reweight (host function):
 * T = ceil(theta*L - 1e-6), the number of identical positions at and above
 * which two sequences count as similar (Eq. 7 uses identity >= 0.8 L). */
int32_t bmdca_identity_threshold(double theta, int32_t L);

/* Uniform random chain initialisation, the "chosen uniformly at random"
 * start of the persistent chains (Sec. 2.1).  Token of chain c at site i:
 * (w * q) >> 32 for the Philox4x32-10 word w = out[i % 4] with key = seed
 * (low, high 32 bits) and counter (i / 4, 0, c, 1).
 * chains: int8 [N][L], written. */
int bmdca_init_chains(int8_t* chains, int64_t N, int32_t L, int32_t q,
                      uint64_t seed, void* stream);

/* Importance weights, Eq. (7) (pre-processing step p.2, Sec. 2.3).
 * msa   int8 [M][L] (read)
 * theta identity fraction (0.8 by default in the paper)
 * n_sim int32 [M]  out: N^(m) = #{n : identical positions >= T}, self
 *                  included, T = bmdca_identity_threshold(theta, L);
 *                  bit-exact integer counts, gaps count as symbols
 * w     double [M] out: 1.0 / N^(m) (one IEEE division)
 * meff  double [1] out: sum_m w^(m) (fixed-order reduction)
 * ws    scratch, bmdca_workspace_bytes(BMDCA_WS_REWEIGHT, M, L, q, 0)
 * dev_err optional; BMDCA_DEVERR_TOKEN on a token outside 0..q-1. */
int bmdca_reweight(const int8_t* msa, int64_t M, int32_t L, int32_t q,
                   double theta, int32_t* n_sim, double* w, double* meff,
                   void* ws, size_t ws_bytes, int32_t* dev_err, void* stream);

/* Reweighted one- and two-site frequencies, Eq. (3), with the pseudocount
 * of Eqs. (8)-(9) (pre-processing step p.3, Sec. 2.3).
 * X      int8 [M][L] (read)
 * w      double [M] weights, or NULL for unit weights (M_eff = M)
 * pseudocount  alpha; a negative value selects alpha = 1 / M_eff (the
 *        paper's default), 0 gives the raw frequencies
 * prec   bmdca_prec of the product; with w == NULL both forms are exact
 * f1     double [Lq] out: (1-alpha) f_i(a) + alpha/q
 * f2     double [Lq][Lq] out: (1-alpha) f_ij(a,b) + alpha/q^2 for i != j;
 *        the diagonal blocks hold delta_ab f1[(i,a)]
 * meff_out double [1] out: M_eff = sum_m w_m (fixed-order reduction)
 * ws     scratch, bmdca_workspace_bytes(BMDCA_WS_STATS, M, L, q, prec)
 * dev_err optional; BMDCA_DEVERR_TOKEN on a token outside 0..q-1.
 * With w == NULL the result is the single rounding of count / M, bit-exact. */
int bmdca_stats(const int8_t* X, const double* w, int64_t M, int32_t L,
                int32_t q, double pseudocount, int32_t prec, double* f1,
                double* f2, double* meff_out, void* ws, size_t ws_bytes,
                int32_t* dev_err, void* stream);

/* Gibbs sampling of the persistent chains (Sec. 2.1, "Monte Carlo
 * estimation of the gradient"); one sweep redraws every site once, sites in
 * the order i = 0..L-1, from the conditional P(a) ~ exp(beta * H_i(a)),
 * H_i(a) = h_i(a) + sum_{j != i} J_ij(a, s_j).
 * Draw: l_a = beta*H_i(a); e_a = exp(l_a - max l); S_a = sum_{b<=a} e_b;
 * CDF_a = S_a / S_{q-1}; a_new = #{a in 0..q-2 : CDF_a <= u}, with the
 * uniform u = (w >> 8) * 2^-24 from the Philox4x32-10 word w = out[i % 4],
 * key = seed, counter (i / 4, sweep_offset + s, c, 0) for chain c and sweep s.
 * Two kernels implement it (flags, see BMDCA_SAMPLER_*):
 *  - field form: the local fields are kept per chain in H_ws (float32
 *    [N][Lq], HBM), rebuilt from h, J and the chains at the start of the
 *    call, and updated incrementally on every accepted change,
 *    H += J[(i,new),:] - J[(i,old),:];
 *  - gather form: H_i is recomputed at every visit from a copy of the
 *    coupling blocks that the call re-lays out in H_ws.
 * With BMDCA_SAMPLER_METROPOLIS either form makes Metropolis visits instead
 * (the rule stated at that flag) in the same site order.
 * chains  int8 [N][L] in/out
 * H_ws    scratch of bmdca_workspace_bytes(BMDCA_WS_GIBBS, N, L, q, flags)
 *         bytes
 * flags   BMDCA_SAMPLER_* selection; BMDCA_GIBBS_KEEP_FIELDS (field form):
 *         H_ws already holds the local fields of these chains under these h
 *         and J (left by the previous call on the same buffers), so the
 *         rebuild is skipped -- for sampling in several slices of sweeps.
 * flips_out optional device uint64: the number of accepted changes is added.
 * Arithmetic is FP32; the state is integer. */
int bmdca_gibbs(const float* h, const float* J, int8_t* chains, int64_t N,
                int32_t L, int32_t q, int32_t sweeps, uint64_t seed,
                uint64_t sweep_offset, float beta, float* H_ws,
                size_t H_ws_bytes, int32_t flags,
                unsigned long long* flips_out, void* stream);

/* Random stream of one chain for bmdca_gibbs_streams (24 bytes). */
typedef struct bmdca_chain_stream {
    uint64_t seed;         /* Philox key of the chain's draws */
    uint64_t sweep_offset; /* global sweep index of the call's first sweep */
    uint32_t chain;        /* chain index used in the Philox counter */
    uint32_t reserved;     /* 0 */
} bmdca_chain_stream;

/* bmdca_gibbs over chains that come from different requests: chain c makes
 * exactly the draws of chain streams[c].chain in a bmdca_gibbs call with
 * seed streams[c].seed and sweep_offset streams[c].sweep_offset, so chains
 * of several callers can be swept in one launch with the results each would
 * get alone (same sampler form).  All chains run `sweeps` sweeps.  The
 * random words and draw rules are those of the alone call.  The FP32 local
 * fields of the gather form are summed in an order fixed by L, q and the draw
 * (the lanes per chain are a function of q and the draw alone; heat-bath
 * chains with 5..7 quads per row may run narrow, one lane per quad, where a
 * launch has many chains per CU, and draw the same bits; launches with many
 * chains per workgroup take one barrier per two chunk-steps, which changes no
 * arithmetic), so heat-bath chains are bit-identical to their alone call in
 * any launch.  For
 * Metropolis the order also follows the chunk length, which the chains per
 * workgroup bound where their tokens fill the LDS; where two launches differ
 * in it a chain can part from its alone trajectory at a draw within FP32
 * rounding of the acceptance threshold (as between the two sampler forms).
 * The field form is always bit-identical.
 * streams  device array [N], caller-owned
 * cus      compute units the launch is sized for (0 = the whole device): a
 *          smaller share packs more chains into each workgroup and streams
 *          the couplings fewer times, for launches that share the GPU
 * Other arguments as bmdca_gibbs (seed/sweep_offset come from `streams`). */
int bmdca_gibbs_streams(const float* h, const float* J, int8_t* chains, int64_t N,
                        int32_t L, int32_t q, int32_t sweeps,
                        const bmdca_chain_stream* streams, float beta, float* H_ws,
                        size_t H_ws_bytes, int32_t flags, int32_t cus,
                        unsigned long long* flips_out, void* stream);

/* DCA energies of a batch of sequences, Eq. (1) (Sec. 4.3, "Scoring a
 * sequence set"): E[b] = -sum_i h_i(s_i) - sum_{i<j} J_ij(s_i, s_j), FP32
 * terms summed in FP64, rounded once to float32.  The pair sum of a sequence
 * is formed in an order fixed by L alone, so a sequence's energy does not
 * depend on the other sequences of the batch (bit for bit).
 * seqs int8 [B][L]; E float32 [B] out (both may be NULL when B == 0).
 * ws   scratch, bmdca_workspace_bytes(BMDCA_WS_ENERGY, B, L, q, 0) (may be
 *      NULL when B == 0)
 * dev_err optional; BMDCA_DEVERR_TOKEN on a token outside 0..q-1. */
int bmdca_energy(const float* h, const float* J, const int8_t* seqs, int64_t B,
                 int32_t L, int32_t q, float* E, void* ws, size_t ws_bytes,
                 int32_t* dev_err, void* stream);

/* Bytes of the library's static per-GPU scratch array for
 * bmdca_energy_noalloc (64 MiB). */
#define BMDCA_ENERGY_SCRATCH_BYTES (64u << 20)

/* bmdca_energy with no workspace argument and no device allocation, for
 * callers that cannot allocate: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Results are those of bmdca_energy
 * bit for bit.  Its scratch (the site-major token copy and the FP64 partial
 * pair sums, align256(L Bp) + align256(8 P Bp) bytes with Bp = B rounded up
 * to 64 and P <= 128 pair ranges fixed by L) lives in one static device array
 * of BMDCA_ENERGY_SCRATCH_BYTES per GPU, held from library load to process
 * end; nothing in it needs clearing between calls.  A batch whose scratch
 * exceeds the array returns BMDCA_EINVAL before anything is enqueued (up
 * to 43 648 sequences fit at L = 512, 84 672 at L = 256, 328 960 at
 * L = 100): split it, or call bmdca_energy.  Every call on one GPU uses the
 * same array, so calls
 * that may overlap on that GPU (different streams, or host threads) race and
 * must be serialised by the caller.  The first call on a device looks up the
 * array's device address (not a stream operation); later calls only enqueue
 * kernels.  Other arguments as bmdca_energy. */
int bmdca_energy_noalloc(const float* h, const float* J, const int8_t* seqs, int64_t B,
                         int32_t L, int32_t q, float* E, int32_t* dev_err, void* stream);

/* One epoch of persistent-chain Boltzmann learning (Sec. 2.1):
 *   1. `sweeps` Gibbs sweeps of the chains at beta = 1, global sweep index
 *      epoch*sweeps + s (as bmdca_gibbs);
 *   2. model marginals from the final chains, p = count / N, with the counts
 *      counted directly (exact integers; with BMDCA_COUNTS_PRODUCT, from the
 *      one-hot product of `prec`, the same integers);
 *   3. *pearson = Pearson correlation of C^data = f_ij - f_i f_j and
 *      C^model = p_ij - p_i p_j (Eq. 6) over i < j and all a, b, FP64,
 *      two-pass;
 *   4. the update of Eq. (5) in FP64, rounded once to float32:
 *      J_ij(a,b) += lr (f_ij(a,b) - p_ij(a,b)) for i != j, J_ii stays 0;
 *      h_i(a)    += lr (f_i(a) - p_i(a)).
 * h, J     float32, updated in place
 * chains   int8 [N][L] in/out
 * f1, f2   double data frequencies as produced by bmdca_stats
 * prec     bmdca_prec, OR-ed with BMDCA_SAMPLER_* and BMDCA_COUNTS_PRODUCT
 * pearson  double [1] out (device)
 * flips_out optional device uint64, accepted changes added
 * ws       scratch, bmdca_workspace_bytes(BMDCA_WS_TRAIN_STEP, N, L, q, prec)
 * dev_err  optional; BMDCA_DEVERR_NONFINITE if an updated parameter or the
 *          Pearson value is not finite. */
int bmdca_train_step(float* h, float* J, int8_t* chains, int64_t N, int32_t L,
                     int32_t q, const double* f1, const double* f2, double lr,
                     int32_t sweeps, uint64_t seed, uint64_t epoch,
                     int32_t prec, double* pearson,
                     unsigned long long* flips_out, void* ws, size_t ws_bytes,
                     int32_t* dev_err, void* stream);

/* Fields of the independent-site (profile) model, the starting point of
 * training (eaDCA starts from a profile model, Sec. 2.2; bmDCA here too):
 * h[(i,a)] = log f1[(i,a)] in FP64, rounded once to float32.  With J = 0
 * its one-site marginals are f_i(a) (each f_i sums to 1).
 * f1 double [Lq] (bmdca_stats); h float32 [Lq] out.
 * dev_err optional; BMDCA_DEVERR_NONFINITE where f1 is not positive and
 * finite (that field is not finite). */
int bmdca_profile_fields(const double* f1, int32_t L, int32_t q, float* h, int32_t* dev_err,
                         void* stream);

/* ---- Grouped training (many independent models, one replayable epoch) ----
 *
 * The training loop of Sec. 2.1 run for several independent models at once.
 * The arithmetic of each model is exactly that of bmdca_train_step; what
 * changes is where the epoch number and the stop condition live: in a small
 * device record per model, so that one captured HIP graph can be replayed
 * every epoch with unchanged kernel arguments. */

/* Device-resident control record of one model (24 bytes, caller-owned,
 * device memory; the caller writes it before the first epoch). */
typedef struct bmdca_train_ctl {
    uint64_t epoch;        /* epochs run so far; the next epoch samples sweeps
                              epoch*sweeps .. epoch*sweeps + sweeps - 1 */
    int32_t active;        /* 0: every kernel of this model returns at once
                              (its h, J, chains and counters stay as they are) */
    int32_t converged_at;  /* set to `epoch` when the target was reached */
    double target_pearson; /* > 0: after an epoch whose Pearson coefficient
                              (Eq. 6) is >= this value, active becomes 0 -- the
                              stop criterion of Sec. 2.1 */
} bmdca_train_ctl;

/* One model of a group: the arguments of bmdca_train_step, with the epoch
 * taken from ctl->epoch.  All pointers are device pointers except the record
 * array itself, which is host memory read during the call. */
typedef struct bmdca_train_problem {
    float* h;
    float* J;
    int8_t* chains;
    const double* f1;
    const double* f2;
    double* pearson;
    unsigned long long* flips_out; /* optional */
    int32_t* dev_err;              /* optional */
    bmdca_train_ctl* ctl;          /* required */
    void* ws;                      /* bmdca_workspace_bytes(BMDCA_WS_TRAIN_STEP, ...) */
    size_t ws_bytes;
    int64_t N;
    int32_t L;
    int32_t q;
    double lr;
    uint64_t seed;
    int32_t sweeps;
    int32_t prec; /* bmdca_prec | BMDCA_SAMPLER_* */
    const uint8_t* mask; /* optional coupling graph [Lq][Lq] (1 = active):
                            pruned elements are held at 0 by the update, as
                            bmdca_train_step_masked; NULL = fully connected */
} bmdca_train_problem;

/* Enqueues one epoch of every model of the group on `stream`: the models are
 * spread over `lanes` (1..16) streams forked from `stream` and joined back
 * into it (largest models first, each to the least-loaded lane), so small
 * models run side by side.  Each model runs bmdca_train_step with its epoch
 * read from ctl->epoch, then advances its record: if active, epoch += 1 and
 * the target test above.  Every model's results are the same as its own
 * bmdca_train_step calls with the same epochs (bit for bit; a model with the
 * Metropolis flag in the gather form is subject to the chunk-length
 * exception stated at bmdca_gibbs_streams).
 * The call may be captured into a HIP graph (it allocates no device memory
 * and enqueues no memset); bmdca_train_group_graph does exactly that.  The
 * lane streams are created once per device (default priority) and kept;
 * group calls are serialised by a library lock. */
int bmdca_train_group_step(const bmdca_train_problem* probs, int32_t n,
                           int32_t lanes, void* stream);

/* A captured, instantiated group epoch (opaque, owned by the caller). */
typedef struct bmdca_graph_s* bmdca_graph;

/* Captures bmdca_train_group_step(probs, n, lanes, stream) into a graph and
 * instantiates it; nothing runs.  The problem records are frozen into the
 * graph: the buffers they name must stay allocated while the graph lives.
 * *out receives the handle; on error *out is NULL. */
int bmdca_train_group_graph(const bmdca_train_problem* probs, int32_t n,
                            int32_t lanes, void* stream, bmdca_graph* out);
/* Enqueues one replay (one epoch of every active model) on `stream`. */
int bmdca_graph_launch(bmdca_graph g, void* stream);
/* Frees the graph (NULL is accepted). */
int bmdca_graph_destroy(bmdca_graph g);

/* ---- Sparse models by element decimation (edDCA, Sec. 2.2 and Sec. 3.2) ----
 *
 * A coupling graph is a mask uint8 [Lq][Lq] (device, caller-owned,
 * symmetric; 1 = active element, diagonal blocks ignored). */

/* bmdca_train_step on a sparse graph: Eq. (5) updates active elements only;
 * elements with mask 0 are set to and held at 0.  Other arguments as
 * bmdca_train_step (same workspace). */
int bmdca_train_step_masked(float* h, float* J, const uint8_t* mask, int8_t* chains,
                            int64_t N, int32_t L, int32_t q, const double* f1,
                            const double* f2, double lr, int32_t sweeps,
                            uint64_t seed, uint64_t epoch, int32_t prec,
                            double* pearson, unsigned long long* flips_out,
                            void* ws, size_t ws_bytes, int32_t* dev_err,
                            void* stream);

/* Coupling graph of a model (Sec. 2.2): bmDCA uses the fully connected
 * graph, eaDCA starts from the empty one.  mask uint8 [Lq][Lq] out: with
 * full != 0, 1 for every element of two different sites and 0 on the
 * diagonal blocks; with full == 0, all 0. */
int bmdca_mask_init(uint8_t* mask, int32_t L, int32_t q, int32_t full, void* stream);

/* Restricts couplings to a graph (Sec. 2.2: couplings off the graph are 0):
 * J[r1][r2] = 0 wherever mask is 0 or r1, r2 lie on the same site; J may be
 * NULL to count only.  n_active: optional device int64, set to the number of
 * active elements r1 < r2 of different sites (exact integer count). */
int bmdca_mask_apply(float* J, const uint8_t* mask, int32_t L, int32_t q, long long* n_active,
                     void* stream);

/* One graph update of element decimation: for every active element
 * (r1, r2), r1 < r2 in different sites, with p = (count of chains with
 * s_i = a and s_j = b) / N, the symmetric Kullback-Leibler distance between
 * the model and the model without that element is, from Eq. (1),
 *   D = J (p - p'),  p' = p e^-J / (1 - p + p e^-J)   (D >= 0).
 * With n_act active elements, n_total = L (L-1) q^2 / 2 and n_target =
 * ceil(density n_total), the k = min(max(1, floor(drate n_act)),
 * n_act - n_target) elements with the smallest (D, r1 Lq + r2) are removed
 * (none when n_act <= n_target): mask and J are zeroed on both triangles.
 * The paper's prescription is "remove the drate fraction with the smallest
 * symmetric KL distance"; the count rule and tie order are this library's.
 * chains   int8 [N][L], the model's current chains
 * n_active optional device int64 out: active elements after the update
 * ws       scratch, bmdca_workspace_bytes(BMDCA_WS_DECIMATE, N, L, q, 0)
 * dev_err  optional; BMDCA_DEVERR_TOKEN on a token outside 0..q-1. */
int bmdca_decimate(float* J, uint8_t* mask, const int8_t* chains, int64_t N,
                   int32_t L, int32_t q, double drate, double density,
                   long long* n_active, void* ws, size_t ws_bytes,
                   int32_t* dev_err, void* stream);

/* One graph update of element activation (eaDCA, Sec. 2.2 and Sec. 3.1): among all
 * elements (r1, r2), r1 < r2 in different sites, active or not, the ones
 * whose model marginal p (chain frequency, as above) is farthest from the
 * data frequency f = f2[r1][r2] are set active.  The paper leaves the
 * distance to a citation; this library takes the Kullback-Leibler divergence
 * of the two Bernoulli laws of the element's indicator,
 *   D = f log(f/p) + (1-f) log((1-f)/(1-p))
 * (0 log 0 = 0; +inf where f > 0 = p or f < 1 = p).  With n_inactive
 * elements, the k = max(1, floor(factivate n_inactive)) largest
 * (D, then smallest r1 Lq + r2) get mask 1 on both triangles (k = 0 when
 * none is inactive); selected elements already active add nothing, as the
 * paper notes.  J is not touched: inactive couplings are already 0.
 * mask      uint8 [Lq][Lq] in/out (device, symmetric)
 * chains    int8 [N][L], the model's current chains
 * f2        FP64 [Lq][Lq] data pairwise frequencies (bmdca_stats)
 * factivate fraction in [0, 1]
 * n_active  optional device int64 out: active elements after the update
 * ws        scratch, bmdca_workspace_bytes(BMDCA_WS_DECIMATE, N, L, q, 0)
 * dev_err   optional; BMDCA_DEVERR_TOKEN on a token outside 0..q-1,
 *           BMDCA_DEVERR_NONFINITE on an f2 entry outside [0, 1] (scored 0). */
int bmdca_activate(uint8_t* mask, const int8_t* chains, int64_t N, int32_t L,
                   int32_t q, const double* f2, double factivate,
                   long long* n_active, void* ws, size_t ws_bytes,
                   int32_t* dev_err, void* stream);

/* Single-mutant library (Sec. 4.4): for each of B wild types,
 * dE[b][i*q + a] = E(wild type with site i set to a) - E(wild type)
 *               = -(H_i(a) - H_i(wt_i)),  H_i(a) = h_i(a) + sum_{j!=i} J_ij(a, wt_j);
 * dE is exactly 0 at a = wt_i.
 * wt int8 [B][L]; dE float32 [B][Lq] out.
 * ws scratch, bmdca_workspace_bytes(BMDCA_WS_MUTANT, B, L, q, 0). */
int bmdca_single_mutant_scan(const float* h, const float* J, const int8_t* wt,
                             int64_t B, int32_t L, int32_t q, float* dE,
                             void* ws, size_t ws_bytes, void* stream);

/* Contact scores, Eq. (13) and Sec. 4.2: every block J_ij (i != j) is moved
 * to the zero-sum gauge over all q states, F_ij = sqrt(sum over a, b != gap of
 * the gauged block squared), F_ii = 0, and
 * F_apc[i][j] = F_ij - (sum_k F_ik)(sum_k F_kj) / sum_kl F_kl (0 on the
 * diagonal).  FP64 inside, float32 out.
 * gap  state excluded from the norm (0 for the default alphabets), -1 = none
 * F    float32 [L][L] out (may be NULL); F_apc float32 [L][L] out
 * ws   scratch, bmdca_workspace_bytes(BMDCA_WS_APC, 0, L, q, 0). */
int bmdca_apc_frobenius(const float* J, int32_t L, int32_t q, int32_t gap,
                        float* F, float* F_apc, void* ws, size_t ws_bytes,
                        void* stream);

/* ---- Serving forms: one launch shape, replayed as a HIP graph ----
 *
 * Sampling, scoring and mutant scans of resident trained models (Sec. 4.1,
 * 4.3, 4.4) served to a stream of requests.  Each call below is sized once
 * for a capacity `cap` of items in caller-owned arenas; the number of live
 * items is read at run time from the device int64 *n_live (0 <= *n_live <=
 * cap), which the caller writes before each launch.  Nothing else in the
 * call changes between launches, so a call captured into a HIP graph can be
 * replayed for every batch.  Items past *n_live are not touched; workgroups
 * past it leave at once.  Every live item gets exactly the bits of the plain
 * call (bmdca_energy, bmdca_single_mutant_scan, bmdca_gibbs), whatever else
 * shares the batch. */

/* bmdca_energy over seqs [cap][L] (first *n_live rows live); ws sized by
 * bmdca_workspace_bytes(BMDCA_WS_ENERGY, cap, L, q, 0). */
int bmdca_energy_batch(const float* h, const float* J, const int8_t* seqs, int64_t cap,
                       const int64_t* n_live, int32_t L, int32_t q, float* E, void* ws,
                       size_t ws_bytes, int32_t* dev_err, void* stream);

/* bmdca_single_mutant_scan over wild types wt [cap][L] (first *n_live live);
 * ws sized by bmdca_workspace_bytes(BMDCA_WS_MUTANT, cap, L, q, 0). */
int bmdca_mutant_scan_batch(const float* h, const float* J, const int8_t* wt, int64_t cap,
                            const int64_t* n_live, int32_t L, int32_t q, float* dE, void* ws,
                            size_t ws_bytes, void* stream);

/* One tick of continuous-batching sampling: the chains [0, *n_live) of the
 * arena chains [cap][L] make `sweeps` sweeps in the gather form (heat-bath,
 * or Metropolis with BMDCA_SAMPLER_METROPOLIS), chain c drawing exactly as
 * chain streams[c].chain of a bmdca_gibbs call with key streams[c].seed and
 * sweep offset streams[c].sweep_offset + (*tick) * sweeps; then *tick += 1
 * (device uint64, caller-owned).  A request that joins the arena at tick T0
 * with its own first sweep 0 therefore stores sweep_offset = -T0 * sweeps
 * (mod 2^64), and after k ticks its chains equal its plain bmdca_gibbs call
 * of k * sweeps sweeps.  With BMDCA_GIBBS_KEEP_LAYOUT the couplings are not
 * re-laid out (ws holds them from a previous call with this J).  Needs the
 * gather form (L <= 512, q <= 32); ws as bmdca_gibbs with
 * BMDCA_SAMPLER_GATHER.  cus as bmdca_gibbs_streams. */
int bmdca_sample_tick(const float* h, const float* J, int8_t* chains, int64_t cap,
                      const int64_t* n_live, int32_t L, int32_t q, int32_t sweeps,
                      const bmdca_chain_stream* streams, uint64_t* tick, float beta,
                      float* ws, size_t ws_bytes, int32_t flags, int32_t cus, void* stream);

/* ---- Equilibrium sampling (Sec. 4.1: sampling from a trained model) ----
 *
 * The sampling routine first measures the mixing time: chains start from
 * data sequences drawn according to their weights, and the overlap
 * SeqID(a, b) = (1/L) sum_i [a_i == b_i] is averaged over chain pairs, once
 * against a permutation of the chains (SeqID(t)) and once against the same
 * chains at time t/2 (SeqID(t, t/2)); the mixing time is where the two
 * curves meet.  These calls are its building blocks (with bmdca_gibbs). */

/* n row indices drawn with replacement, row m with probability w_m / W,
 * W = sum of w: with C_m = w_0 + ... + w_m (ascending m), draw k takes the
 * uniform u of Philox counter (k/4, 0, 0, 2), word k%4, u = (word >> 8) 2^-24,
 * key = seed, and returns the first m with C_m > u W.
 * w       double [M] >= 0 (device); rows int32 [n] out
 * ws      scratch, bmdca_workspace_bytes(BMDCA_WS_DRAW, M, 1, 2, 0)
 * dev_err optional; BMDCA_DEVERR_NONFINITE if W is not positive and finite
 *         (every row is then 0). */
int bmdca_draw_rows(const double* w, int64_t M, int64_t n, uint64_t seed,
                    int32_t* rows, void* ws, size_t ws_bytes, int32_t* dev_err,
                    void* stream);

/* out[k][.] = X[rows[k]][.] for k < n (int8 rows of length L).
 * dev_err optional; BMDCA_DEVERR_INDEX for an index outside 0..M-1 (row 0
 * is copied instead). */
int bmdca_gather_rows(const int8_t* X, int64_t M, int32_t L,
                      const int32_t* rows, int64_t n, int8_t* out,
                      int32_t* dev_err, void* stream);

/* Mean and standard deviation of SeqID(A[k], B[perm[k]]) over k < N (B[k]
 * when perm is NULL), from the exact integer sums S1, S2 of the identity
 * counts: out[0] = S1 / (N L), out[1] = sqrt(S2 / (N L^2) - out[0]^2).
 * A, B int8 [N][L]; perm int32 [N] (device, may be NULL); out double [2].
 * ws      scratch, bmdca_workspace_bytes(BMDCA_WS_SEQID, 0, L, 2, 0)
 * dev_err optional; BMDCA_DEVERR_INDEX for a perm entry outside 0..N-1
 *         (that pair is skipped). */
int bmdca_seqid(const int8_t* A, const int8_t* B, const int32_t* perm,
                int64_t N, int32_t L, double* out, void* ws, size_t ws_bytes,
                int32_t* dev_err, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* BMDCA_H */
