/* Host driver that runs every routine of the FP64 oracle once on small seeded
 * inputs (ragged sizes, edge cases), built together with bmdca_oracle.c under
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py:
 * any out-of-bounds access, leak or undefined operation fails the run.  The
 * results are not checked here (the pins do that). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]);
double orc_gibbs_uniform(uint64_t seed, uint64_t c, uint64_t sg, int32_t i);
void orc_init_chains(int8_t* chains, int64_t N, int32_t L, int32_t q, uint64_t seed);
void orc_reweight(const int8_t* msa, int64_t M, int32_t L, double theta, int32_t* n_sim,
                  double* w, double* meff);
void orc_stats(const int8_t* X, const double* w, int64_t M, int32_t L, int32_t q,
               double pseudocount, double* f1, double* f2, double* meff_out);
void orc_energy(const float* h, const float* J, const int8_t* seqs, int64_t B, int32_t L,
                int32_t q, double* E);
void orc_local_fields_all(const float* h, const float* J, const int8_t* s, int32_t L, int32_t q,
                          double* H);
void orc_gibbs_range(const float* h, const float* J, int8_t* chains, int64_t N, int64_t c0,
                     int32_t L, int32_t q, int32_t sweeps, uint64_t seed, uint64_t sweep_offset,
                     double beta, double* margins, int64_t* flips);
double orc_train_step(float* h, float* J, int8_t* chains, int64_t N, int32_t L, int32_t q,
                      const double* f1, const double* f2, double lr, int32_t sweeps,
                      uint64_t seed, uint64_t epoch, double* margins, int64_t* flips);
void orc_mutant_scan(const float* h, const float* J, const int8_t* wt, int32_t L, int32_t q,
                     double* dE);
void orc_apc_frobenius(const float* J, int32_t L, int32_t q, int32_t gap, double* F,
                       double* Fapc);
int orc_enumerate(const float* h, const float* J, int32_t L, int32_t q, double beta, double* p1,
                  double* p2, double* logZ);
void orc_reweight_rows(const int8_t* msa, int64_t M, int32_t L, double theta,
                       const int64_t* rows, int64_t nrows, int32_t* n_sim);
void orc_stats_entries(const int8_t* X, const double* w, int64_t M, int32_t L, int32_t q,
                       double pseudocount, const int64_t* r1, const int64_t* r2, int64_t n,
                       double* out);
void orc_draw_rows(const double* w, int64_t M, int64_t n, uint64_t seed, int32_t* rows,
                   double* margins);
void orc_seqid(const int8_t* A, const int8_t* B, const int32_t* perm, int64_t N, int32_t L,
               double* out);
void orc_metropolis_range(const float* h, const float* J, int8_t* chains, int64_t N, int64_t c0,
                          int32_t L, int32_t q, int32_t sweeps, uint64_t seed,
                          uint64_t sweep_offset, double beta, double* margins, int64_t* flips);
void orc_chain_forced(const float* h, const float* J, int8_t* s, uint64_t c, int32_t L,
                      int32_t q, int32_t sweeps, uint64_t seed, uint64_t sweep_offset,
                      double beta, int32_t metropolis, double tol, const int8_t* force,
                      int8_t* drawn, int8_t* alt_lo, int8_t* alt_hi);
int64_t orc_decimate(float* J, uint8_t* mask, const int8_t* chains, int64_t N, int32_t L,
                     int32_t q, double drate, double density);
int64_t orc_activate(uint8_t* mask, const int8_t* chains, int64_t N, int32_t L, int32_t q,
                     const double* f2, double factivate);
double orc_train_step_masked(float* h, float* J, const uint8_t* mask, int8_t* chains, int64_t N,
                             int32_t L, int32_t q, const double* f1, const double* f2, double lr,
                             int32_t sweeps, uint64_t seed, uint64_t epoch, double* margins,
                             int64_t* flips);
void orc_profile_fields(const double* f1, int32_t L, int32_t q, float* h);
int64_t orc_mask_apply(float* J, const uint8_t* mask, int32_t L, int32_t q);

static uint64_t rs = 88172645463325252ull;
static double urand(void) {
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return (double)(rs >> 11) * (1.0 / 9007199254740992.0);
}

/* symmetric couplings with zero diagonal blocks */
static float* couplings(int L, int q, double s) {
    const int64_t Lq = (int64_t)L * q;
    float* J = calloc((size_t)(Lq * Lq), sizeof(float));
    for (int64_t a = 0; a < Lq; ++a)
        for (int64_t b = a + 1; b < Lq; ++b)
            if (a / q != b / q) J[a * Lq + b] = J[b * Lq + a] = (float)(s * (urand() - 0.5));
    return J;
}

static void run(int L, int q, int64_t N, int64_t M) {
    const int64_t Lq = (int64_t)L * q;
    float* h = malloc(sizeof(float) * (size_t)Lq);
    for (int64_t r = 0; r < Lq; ++r) h[r] = (float)(urand() - 0.5);
    float* J = couplings(L, q, 0.6);
    int8_t* X = malloc((size_t)(M * L));
    orc_init_chains(X, M, L, q, 11);
    int8_t* ch = malloc((size_t)(N * L));
    orc_init_chains(ch, N, L, q, 12);
    int32_t* n = malloc(sizeof(int32_t) * (size_t)M);
    double* w = malloc(sizeof(double) * (size_t)M);
    double meff;
    orc_reweight(X, M, L, 0.8, n, w, &meff);
    double* f1 = malloc(sizeof(double) * (size_t)Lq);
    double* f2 = malloc(sizeof(double) * (size_t)(Lq * Lq));
    orc_stats(X, w, M, L, q, -1.0, f1, f2, &meff);
    orc_stats(X, NULL, M, L, q, 0.0, f1, f2, &meff);
    orc_stats(X, w, M, L, q, -1.0, f1, f2, &meff);
    double* E = malloc(sizeof(double) * (size_t)M);
    orc_energy(h, J, X, M, L, q, E);
    double* H = malloc(sizeof(double) * (size_t)Lq);
    orc_local_fields_all(h, J, ch, L, q, H);
    double* mg = malloc(sizeof(double) * (size_t)(N * 2 * L));
    int64_t flips;
    orc_gibbs_range(h, J, ch, N, 5, L, q, 2, 13, 4, 0.7, mg, &flips);
    orc_metropolis_range(h, J, ch, N, 0, L, q, 2, 14, 0, 1.3, mg, &flips);
    int8_t* force = malloc((size_t)(2 * L));
    int8_t* d = malloc((size_t)(2 * L));
    int8_t* lo = malloc((size_t)(2 * L));
    int8_t* hi = malloc((size_t)(2 * L));
    memset(force, -1, (size_t)(2 * L));
    force[L / 2] = (int8_t)(q - 1);
    orc_chain_forced(h, J, ch, 3, L, q, 2, 15, 1, 1.0, 0, 1e-2, force, d, lo, hi);
    orc_chain_forced(h, J, ch, 3, L, q, 2, 15, 1, 1.0, 1, 1e-2, NULL, d, lo, hi);
    double* dE = malloc(sizeof(double) * (size_t)Lq);
    orc_mutant_scan(h, J, X, L, q, dE);
    double* F = malloc(sizeof(double) * (size_t)(L * L));
    double* Fa = malloc(sizeof(double) * (size_t)(L * L));
    orc_apc_frobenius(J, L, q, 0, F, Fa);
    orc_apc_frobenius(J, L, q, -1, F, Fa);
    int64_t rows[3] = {0, M / 2, M - 1};
    int32_t nr[3];
    orc_reweight_rows(X, M, L, 0.8, rows, 3, nr);
    double ent[3];
    int64_t r1[3] = {0, Lq - 1, Lq / 2}, r2[3] = {Lq - 1, 0, Lq / 2};
    orc_stats_entries(X, w, M, L, q, -1.0, r1, r2, 3, ent);
    int32_t* drawn = malloc(sizeof(int32_t) * 50);
    double* dm = malloc(sizeof(double) * 50);
    orc_draw_rows(w, M, 50, 16, drawn, dm);
    double sq[2];
    int32_t* perm = malloc(sizeof(int32_t) * (size_t)N);
    for (int64_t k = 0; k < N; ++k) perm[k] = (int32_t)(N - 1 - k);
    orc_seqid(ch, ch, perm, N, L, sq);
    orc_seqid(ch, ch, NULL, N, L, sq);
    float* h2 = malloc(sizeof(float) * (size_t)Lq);
    memcpy(h2, h, sizeof(float) * (size_t)Lq);
    orc_train_step(h2, J, ch, N, L, q, f1, f2, 0.05, 2, 17, 3, NULL, &flips);
    uint8_t* mask = malloc((size_t)(Lq * Lq));
    for (int64_t e = 0; e < Lq * Lq; ++e) mask[e] = (uint8_t)((e / Lq) / q != (e % Lq) / q);
    orc_mask_apply(J, mask, L, q);
    orc_decimate(J, mask, ch, N, L, q, 0.1, 0.2);
    orc_train_step_masked(h2, J, mask, ch, N, L, q, f1, f2, 0.05, 1, 18, 4, NULL, NULL);
    memset(mask, 0, (size_t)(Lq * Lq));
    orc_activate(mask, ch, N, L, q, f2, 0.05);
    orc_profile_fields(f1, L, q, h2);
    if (L * log((double)q) < 12.0) {
        double* p1 = malloc(sizeof(double) * (size_t)Lq);
        double* p2 = malloc(sizeof(double) * (size_t)(Lq * Lq));
        double lz;
        orc_enumerate(h, J, L, q, 1.0, p1, p2, &lz);
        free(p1);
        free(p2);
    }
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    orc_philox4x32_10(ctr, key, out);
    (void)orc_gibbs_uniform(7, 8, 9, L - 1);
    free(h); free(J); free(X); free(ch); free(n); free(w); free(f1); free(f2); free(E); free(H);
    free(mg); free(force); free(d); free(lo); free(hi); free(dE); free(F); free(Fa);
    free(drawn); free(dm); free(perm); free(h2); free(mask);
}

int main(void) {
    run(4, 3, 17, 9);
    run(13, 21, 33, 41);
    run(2, 2, 1, 1);
    run(7, 5, 64, 70);
    printf("oracle sanitizer run ok\n");
    return 0;
}
