/*
 * bmdca_oracle.c -- plain, slow, FP64 CPU oracle for the bmDCA training hot
 * path (adabmDCA 2.0, arXiv:2501.18456).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the HIP library; both implement the
 * same written definitions independently.
 *
 * Every routine is the textbook definition written out in double precision:
 * no blocking, no incremental updates, no reordering of any sum beyond the
 * ascending index order stated at each routine.  Build with contraction off
 * (-ffp-contract=off) so that every a*b+c is two roundings.
 *
 * Conventions (shared definitions, restated here):
 *   tokens      int8 0..q-1, token 0 = gap (Table 1 lists the gap first)
 *   flat index  r = i*q + a for site i, state a
 *   h           float32 [L*q]
 *   J           float32 [L*q][L*q], full-symmetric, zero diagonal blocks
 *   energy      E(s) = -sum_i h_i(s_i) - sum_{i<j} J_ij(s_i, s_j)   (Eq. 1)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX2(r1, r2, Lq) ((size_t)(r1) * (size_t)(Lq) + (size_t)(r2))

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator, as defined by Salmon, Moraes, Dror  */
/* and Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten       */
/* rounds of two 32x32->64 multiplies with the round function                 */
/*   (c0,c1,c2,c3) -> (hi(M1*c2)^c1^k0, lo(M1*c2), hi(M0*c0)^c3^k1, lo(M0*c0)) */
/* and a Weyl-sequence key bump between rounds.                               */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* One 32-bit word of the stream: key = seed, counter = (ctr0, ctr1, ctr2,
 * stream), word = output[word_index]. */
static uint32_t philox_word(uint64_t seed, uint32_t ctr0, uint32_t ctr1,
                            uint32_t ctr2, uint32_t stream, int word_index)
{
    uint32_t ctr[4] = {ctr0, ctr1, ctr2, stream};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return out[word_index];
}

/* Uniform used by the Gibbs draw of chain c at site i in global sweep sg:
 * counter (i/4, sg, c, 0), word i%4, u = (word >> 8) * 2^-24 in [0, 1). */
double orc_gibbs_uniform(uint64_t seed, uint64_t c, uint64_t sg, int32_t i)
{
    uint32_t w = philox_word(seed, (uint32_t)i >> 2, (uint32_t)sg, (uint32_t)c,
                             0u, i & 3);
    return (double)(w >> 8) * (1.0 / 16777216.0);
}

/* Uniform random initial chains (the "chosen uniformly at random" start of
 * Sec. 2.1): counter (i/4, 0, c, 1), word i%4, token = (word * q) >> 32. */
void orc_init_chains(int8_t* chains, int64_t N, int32_t L, int32_t q,
                     uint64_t seed)
{
    for (int64_t c = 0; c < N; ++c)
        for (int32_t i = 0; i < L; ++i) {
            uint32_t w = philox_word(seed, (uint32_t)i >> 2, 0u, (uint32_t)c, 1u,
                                     i & 3);
            chains[c * L + i] = (int8_t)(((uint64_t)w * (uint64_t)q) >> 32);
        }
}

/* ------------------------------------------------------------------------ */
/* Pre-processing step p.2: importance weights, Eq. (7).                      */
/* ------------------------------------------------------------------------ */

/* Integer identity threshold: number of identical positions >= theta*L,
 * read as T = ceil(theta*L - 1e-6) so that products such as 0.8*35 that
 * round just above an integer do not raise the threshold by one. */
int32_t orc_identity_threshold(double theta, int32_t L)
{
    return (int32_t)ceil(theta * (double)L - 1e-6);
}

/* N^(m) = #{n : sum_i [a_i^(m) == a_i^(n)] >= T}, self included (Eq. 7);
 * w^(m) = 1 / N^(m); M_eff = sum_m w^(m) in ascending m (the M_eff of the
 * pseudocount paragraph). Gaps count as ordinary symbols. */
void orc_reweight(const int8_t* msa, int64_t M, int32_t L, double theta,
                  int32_t* n_sim, double* w, double* meff)
{
    int32_t T = orc_identity_threshold(theta, L);
    for (int64_t m = 0; m < M; ++m) {
        int32_t count = 0;
        for (int64_t n = 0; n < M; ++n) {
            int32_t same = 0;
            for (int32_t i = 0; i < L; ++i)
                same += (msa[m * L + i] == msa[n * L + i]);
            if (same >= T) count += 1;
        }
        n_sim[m] = count;
    }
    double s = 0.0;
    for (int64_t m = 0; m < M; ++m) {
        w[m] = 1.0 / (double)n_sim[m];
        s += w[m];
    }
    *meff = s;
}

/* ------------------------------------------------------------------------ */
/* Pre-processing step p.3: reweighted frequencies Eq. (3) and pseudocount    */
/* Eqs. (8)-(9).                                                              */
/* ------------------------------------------------------------------------ */

/* f1[i,a] = sum_m w_m [a_i^m == a] / M_eff,
 * f2[(i,a),(j,b)] = sum_m w_m [a_i^m == a][a_j^m == b] / M_eff   (i != j),
 * each sum taken in ascending m.  w == NULL means unit weights (M_eff = M).
 * Pseudocount alpha: alpha < 0 selects alpha = 1/M_eff.
 *   f1' = (1 - alpha) f1 + alpha / q
 *   f2' = (1 - alpha) f2 + alpha / q^2              (i != j)
 *   f2'[(i,a),(i,b)] = delta_ab f1'[i,a]            (diagonal blocks)
 * Outputs f1 [L*q], f2 [Lq*Lq], *meff_out. */
void orc_stats(const int8_t* X, const double* w, int64_t M, int32_t L, int32_t q,
               double pseudocount, double* f1, double* f2, double* meff_out)
{
    const int64_t Lq = (int64_t)L * q;
    double meff = 0.0;
    for (int64_t m = 0; m < M; ++m) meff += (w ? w[m] : 1.0);
    memset(f1, 0, sizeof(double) * (size_t)Lq);
    memset(f2, 0, sizeof(double) * (size_t)Lq * (size_t)Lq);
    /* Accumulate weighted counts; every entry receives its terms in
     * ascending m because m is the outer loop. */
    for (int64_t m = 0; m < M; ++m) {
        const double wm = w ? w[m] : 1.0;
        const int8_t* s = X + m * L;
        for (int32_t i = 0; i < L; ++i) {
            f1[i * q + s[i]] += wm;
            for (int32_t j = 0; j < L; ++j) {
                if (j == i) continue;
                f2[IDX2(i * q + s[i], j * q + s[j], Lq)] += wm;
            }
        }
    }
    double alpha = pseudocount < 0.0 ? 1.0 / meff : pseudocount;
    for (int64_t r = 0; r < Lq; ++r) {
        double f = f1[r] / meff;
        double t1 = (1.0 - alpha) * f;
        double t2 = alpha / (double)q;
        f1[r] = t1 + t2;
    }
    const double qq = (double)q * (double)q;
    for (int32_t i = 0; i < L; ++i)
        for (int32_t a = 0; a < q; ++a)
            for (int32_t j = 0; j < L; ++j)
                for (int32_t b = 0; b < q; ++b) {
                    size_t k = IDX2(i * q + a, j * q + b, Lq);
                    if (i == j) {
                        f2[k] = (a == b) ? f1[i * q + a] : 0.0;
                    } else {
                        double f = f2[k] / meff;
                        double t1 = (1.0 - alpha) * f;
                        double t2 = alpha / qq;
                        f2[k] = t1 + t2;
                    }
                }
    *meff_out = meff;
}

/* ------------------------------------------------------------------------ */
/* Energy of Eq. (1).                                                         */
/* ------------------------------------------------------------------------ */

/* E(s) = -sum_i h_i(s_i) - sum_{i<j} J_ij(s_i,s_j), accumulated in double,
 * fields first (ascending i), then pairs in (i, j) lexicographic order. */
double orc_energy_one(const float* h, const float* J, const int8_t* s, int32_t L,
                      int32_t q)
{
    const int64_t Lq = (int64_t)L * q;
    double e = 0.0;
    for (int32_t i = 0; i < L; ++i) e -= (double)h[i * q + s[i]];
    for (int32_t i = 0; i < L; ++i)
        for (int32_t j = i + 1; j < L; ++j)
            e -= (double)J[IDX2(i * q + s[i], j * q + s[j], Lq)];
    return e;
}

void orc_energy(const float* h, const float* J, const int8_t* seqs, int64_t B,
                int32_t L, int32_t q, double* E)
{
    for (int64_t b = 0; b < B; ++b) E[b] = orc_energy_one(h, J, seqs + b * L, L, q);
}

/* ------------------------------------------------------------------------ */
/* Local field: the log of the conditional of Eq. (1) at site i, up to a     */
/* constant: H_i(a) = h_i(a) + sum_{j != i} J_ij(a, s_j).  From scratch.      */
/* ------------------------------------------------------------------------ */
void orc_local_field(const float* h, const float* J, const int8_t* s, int32_t L,
                     int32_t q, int32_t i, double* Hi)
{
    const int64_t Lq = (int64_t)L * q;
    for (int32_t a = 0; a < q; ++a) {
        double v = (double)h[i * q + a];
        for (int32_t j = 0; j < L; ++j) {
            if (j == i) continue;
            v += (double)J[IDX2(i * q + a, j * q + s[j], Lq)];
        }
        Hi[a] = v;
    }
}

/* All L*q local fields of one configuration (H[i*q + a]). */
void orc_local_fields_all(const float* h, const float* J, const int8_t* s,
                          int32_t L, int32_t q, double* H)
{
    for (int32_t i = 0; i < L; ++i) orc_local_field(h, J, s, L, q, i, H + i * q);
}

/* ------------------------------------------------------------------------ */
/* Gibbs sampling (Sec. 2.1, Monte Carlo estimation of the gradient): one     */
/* sweep proposes a new state at every site; sites are visited in the order  */
/* i = 0..L-1, and site i is redrawn from its exact conditional               */
/* P(a) ~ exp(beta * H_i(a)).                                                 */
/* Draw rule (inverse CDF): e_a = exp(l_a - max l), S_a = sum_{b<=a} e_b in   */
/* ascending b, CDF_a = S_a / S_{q-1}, a_new = #{a in 0..q-2 : CDF_a <= u}.   */
/* The distance from u to the nearest CDF_a (a <= q-2) is the "margin" of the */
/* visit; it is recorded per (chain, sweep, site) when margins != NULL.       */
/* ------------------------------------------------------------------------ */
/* Chains chains[0..N) carry the global chain indices c0 .. c0+N-1 (the
 * chain index is part of the Philox counter), so any contiguous slice of a
 * large set of chains can be advanced on its own. */
/* Draw of one visit from the local fields Hi by the rule above; returns
 * a_new and the visit's margin.  When n_lo / n_hi are given they receive the
 * number of CDF steps a <= q-2 within tol of u at or below u (each of them
 * read the other way lowers a_new by one) and above u (raises it by one). */
static int32_t gibbs_draw(const double* Hi, int32_t q, double beta, double u,
                          double* e, double* cdf, double tol, double* margin,
                          int32_t* n_lo, int32_t* n_hi)
{
    double mx = -INFINITY;
    for (int32_t a = 0; a < q; ++a) {
        double l = beta * Hi[a];
        if (l > mx) mx = l;
    }
    double S = 0.0;
    for (int32_t a = 0; a < q; ++a) {
        e[a] = exp(beta * Hi[a] - mx);
        S += e[a];
        cdf[a] = S; /* running sum, normalised below */
    }
    for (int32_t a = 0; a < q; ++a) cdf[a] = cdf[a] / S;
    int32_t anew = 0, lo = 0, hi = 0;
    double mg = INFINITY;
    for (int32_t a = 0; a < q - 1; ++a) {
        if (cdf[a] <= u) anew += 1;
        double d = fabs(u - cdf[a]);
        if (d < mg) mg = d;
        if (d < tol) {
            if (cdf[a] <= u) lo += 1;
            else hi += 1;
        }
    }
    *margin = mg;
    if (n_lo) *n_lo = lo;
    if (n_hi) *n_hi = hi;
    return anew;
}

/* Chains chains[0..N) carry the global chain indices c0 .. c0+N-1 (the
 * chain index is part of the Philox counter), so any contiguous slice of a
 * large set of chains can be advanced on its own. */
void orc_gibbs_range(const float* h, const float* J, int8_t* chains, int64_t N,
                     int64_t c0, int32_t L, int32_t q, int32_t sweeps,
                     uint64_t seed, uint64_t sweep_offset, double beta,
                     double* margins, int64_t* flips)
{
    int64_t nflip = 0;
    /* Chains are independent.  Built with -fopenmp (the timing build of the
     * CPU baseline) they are spread over threads; every chain's draws are the
     * same in either build. */
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nflip)
    for (int64_t c = 0; c < N; ++c) {
        double* Hi = (double*)malloc(sizeof(double) * (size_t)q);
        double* e = (double*)malloc(sizeof(double) * (size_t)q);
        double* cdf = (double*)malloc(sizeof(double) * (size_t)q);
        int8_t* s = chains + c * L;
        for (int32_t sw = 0; sw < sweeps; ++sw) {
            uint64_t sg = sweep_offset + (uint64_t)sw;
            for (int32_t i = 0; i < L; ++i) {
                orc_local_field(h, J, s, L, q, i, Hi);
                double u = orc_gibbs_uniform(seed, (uint64_t)(c0 + c), sg, i);
                double margin;
                int32_t anew = gibbs_draw(Hi, q, beta, u, e, cdf, 0.0, &margin, NULL, NULL);
                if (margins) margins[((size_t)c * sweeps + sw) * L + i] = margin;
                if (anew != s[i]) nflip += 1;
                s[i] = (int8_t)anew;
            }
        }
        free(Hi);
        free(e);
        free(cdf);
    }
    if (flips) *flips = nflip;
}

void orc_gibbs(const float* h, const float* J, int8_t* chains, int64_t N,
               int32_t L, int32_t q, int32_t sweeps, uint64_t seed,
               uint64_t sweep_offset, double beta, double* margins,
               int64_t* flips)
{
    orc_gibbs_range(h, J, chains, N, 0, L, q, sweeps, seed, sweep_offset, beta,
                    margins, flips);
}

/* ------------------------------------------------------------------------ */
/* Model marginals estimated from N chains (unit weights): p = count / N.     */
/* Diagonal blocks hold delta_ab p_i(a) by the same definition.               */
/* ------------------------------------------------------------------------ */
void orc_chain_freqs(const int8_t* chains, int64_t N, int32_t L, int32_t q,
                     double* p1, double* p2)
{
    const int64_t Lq = (int64_t)L * q;
    memset(p1, 0, sizeof(double) * (size_t)Lq);
    memset(p2, 0, sizeof(double) * (size_t)Lq * (size_t)Lq);
    for (int64_t c = 0; c < N; ++c) {
        const int8_t* s = chains + c * L;
        for (int32_t i = 0; i < L; ++i) {
            p1[i * q + s[i]] += 1.0;
            for (int32_t j = 0; j < L; ++j)
                p2[IDX2(i * q + s[i], j * q + s[j], Lq)] += 1.0;
        }
    }
    for (int64_t r = 0; r < Lq; ++r) p1[r] = p1[r] / (double)N;
    for (int64_t k = 0; k < Lq * Lq; ++k) p2[k] = p2[k] / (double)N;
}

/* ------------------------------------------------------------------------ */
/* Convergence check of Sec. 2.1: Pearson correlation between the connected  */
/* correlations (Eq. 6) C^data = f_ij - f_i f_j and C^model = p_ij - p_i p_j */
/* over all i<j and all a, b, in (i, j, a, b) lexicographic order; two-pass. */
/* ------------------------------------------------------------------------ */
double orc_pearson(const double* f1, const double* f2, const double* p1,
                   const double* p2, int32_t L, int32_t q)
{
    const int64_t Lq = (int64_t)L * q;
    double sx = 0.0, sy = 0.0;
    int64_t n = 0;
    for (int32_t i = 0; i < L; ++i)
        for (int32_t j = i + 1; j < L; ++j)
            for (int32_t a = 0; a < q; ++a)
                for (int32_t b = 0; b < q; ++b) {
                    size_t k = IDX2(i * q + a, j * q + b, Lq);
                    sx += f2[k] - f1[i * q + a] * f1[j * q + b];
                    sy += p2[k] - p1[i * q + a] * p1[j * q + b];
                    n += 1;
                }
    double mx = sx / (double)n, my = sy / (double)n;
    double sxx = 0.0, syy = 0.0, sxy = 0.0;
    for (int32_t i = 0; i < L; ++i)
        for (int32_t j = i + 1; j < L; ++j)
            for (int32_t a = 0; a < q; ++a)
                for (int32_t b = 0; b < q; ++b) {
                    size_t k = IDX2(i * q + a, j * q + b, Lq);
                    double x = f2[k] - f1[i * q + a] * f1[j * q + b] - mx;
                    double y = p2[k] - p1[i * q + a] * p1[j * q + b] - my;
                    sxx += x * x;
                    syy += y * y;
                    sxy += x * y;
                }
    return sxy / sqrt(sxx * syy);
}

/* ------------------------------------------------------------------------ */
/* Boltzmann-learning update, Eq. (5):                                        */
/*   h_i(a)    <- h_i(a)    + lr (f_i(a)    - p_i(a))                         */
/*   J_ij(a,b) <- J_ij(a,b) + lr (f_ij(a,b) - p_ij(a,b))      (i != j)        */
/* in double, rounded once to float; diagonal blocks J_ii stay 0 (Sec. 2.1). */
/* ------------------------------------------------------------------------ */
void orc_update(float* h, float* J, const double* f1, const double* f2,
                const double* p1, const double* p2, int32_t L, int32_t q,
                double lr)
{
    const int64_t Lq = (int64_t)L * q;
    for (int64_t r = 0; r < Lq; ++r) {
        double d = f1[r] - p1[r];
        double t = lr * d;
        h[r] = (float)((double)h[r] + t);
    }
    for (int64_t r1 = 0; r1 < Lq; ++r1)
        for (int64_t r2 = 0; r2 < Lq; ++r2) {
            size_t k = IDX2(r1, r2, Lq);
            if (r1 / q == r2 / q) {
                J[k] = 0.0f;
                continue;
            }
            double d = f2[k] - p2[k];
            double t = lr * d;
            J[k] = (float)((double)J[k] + t);
        }
}

/* One epoch of persistent-chain Boltzmann learning (Sec. 2.1): `sweeps`
 * Gibbs sweeps at beta = 1 with global sweep index epoch*sweeps + s, model
 * marginals from the final chain state, the Pearson check of (f, p), then the
 * update of Eq. (5).  Returns the Pearson coefficient. */
double orc_train_step(float* h, float* J, int8_t* chains, int64_t N, int32_t L,
                      int32_t q, const double* f1, const double* f2, double lr,
                      int32_t sweeps, uint64_t seed, uint64_t epoch,
                      double* margins, int64_t* flips)
{
    const int64_t Lq = (int64_t)L * q;
    orc_gibbs(h, J, chains, N, L, q, sweeps, seed, epoch * (uint64_t)sweeps, 1.0,
              margins, flips);
    double* p1 = (double*)malloc(sizeof(double) * (size_t)Lq);
    double* p2 = (double*)malloc(sizeof(double) * (size_t)Lq * (size_t)Lq);
    orc_chain_freqs(chains, N, L, q, p1, p2);
    double r = orc_pearson(f1, f2, p1, p2, L, q);
    orc_update(h, J, f1, f2, p1, p2, L, q, lr);
    free(p1);
    free(p2);
    return r;
}

/* ------------------------------------------------------------------------ */
/* Single-mutant library (Sec. 4.4): dE[i*q+b] = E(mutant) - E(wild type),   */
/* the mutant being the wild type with site i set to b; two brute-force       */
/* energies per entry (dE = 0 where b is the wild-type state).                */
/* ------------------------------------------------------------------------ */
void orc_mutant_scan(const float* h, const float* J, const int8_t* wt, int32_t L,
                     int32_t q, double* dE)
{
    int8_t* s = (int8_t*)malloc((size_t)L);
    memcpy(s, wt, (size_t)L);
    double e0 = orc_energy_one(h, J, wt, L, q);
    for (int32_t i = 0; i < L; ++i)
        for (int32_t b = 0; b < q; ++b) {
            s[i] = (int8_t)b;
            dE[i * q + b] = orc_energy_one(h, J, s, L, q) - e0;
            s[i] = wt[i];
        }
    free(s);
}

/* ------------------------------------------------------------------------ */
/* Contact score, Eq. (13) and Sec. 4.2: each coupling block J_ij (i != j)   */
/* is moved to the zero-sum gauge over all q states,                          */
/*   J0(a,b) = J(a,b) - mean_b' J(a,b') - mean_a' J(a',b) + mean_a'b' J,      */
/* then F_ij = sqrt(sum_{a,b != gap} J0(a,b)^2), F_ii = 0, and                */
/* F^APC_ij = F_ij - (sum_k F_ik)(sum_k F_kj) / sum_kl F_kl (diagonal = 0).   */
/* gap < 0 keeps every state in the norm.                                     */
/* ------------------------------------------------------------------------ */
void orc_apc_frobenius(const float* J, int32_t L, int32_t q, int32_t gap,
                       double* F, double* Fapc)
{
    const int64_t Lq = (int64_t)L * q;
    double* B = (double*)malloc(sizeof(double) * (size_t)q * (size_t)q);
    double* rm = (double*)malloc(sizeof(double) * (size_t)q);
    double* cm = (double*)malloc(sizeof(double) * (size_t)q);
    for (int32_t i = 0; i < L; ++i)
        for (int32_t j = 0; j < L; ++j) {
            if (i == j) {
                F[(size_t)i * L + j] = 0.0;
                continue;
            }
            double all = 0.0;
            for (int32_t a = 0; a < q; ++a)
                for (int32_t b = 0; b < q; ++b) {
                    B[a * q + b] = (double)J[IDX2(i * q + a, j * q + b, Lq)];
                    all += B[a * q + b];
                }
            all /= (double)q * (double)q;
            for (int32_t a = 0; a < q; ++a) {
                double s = 0.0;
                for (int32_t b = 0; b < q; ++b) s += B[a * q + b];
                rm[a] = s / (double)q;
            }
            for (int32_t b = 0; b < q; ++b) {
                double s = 0.0;
                for (int32_t a = 0; a < q; ++a) s += B[a * q + b];
                cm[b] = s / (double)q;
            }
            double ss = 0.0;
            for (int32_t a = 0; a < q; ++a)
                for (int32_t b = 0; b < q; ++b) {
                    if (a == gap || b == gap) continue;
                    double z = B[a * q + b] - rm[a] - cm[b] + all;
                    ss += z * z;
                }
            F[(size_t)i * L + j] = sqrt(ss);
        }
    double* S = (double*)malloc(sizeof(double) * (size_t)L);
    double tot = 0.0;
    for (int32_t i = 0; i < L; ++i) {
        double s = 0.0;
        for (int32_t k = 0; k < L; ++k) s += F[(size_t)i * L + k];
        S[i] = s;
        tot += s;
    }
    for (int32_t i = 0; i < L; ++i)
        for (int32_t j = 0; j < L; ++j)
            Fapc[(size_t)i * L + j] =
                (i == j) ? 0.0 : F[(size_t)i * L + j] - S[i] * S[j] / tot;
    free(S);
    free(B);
    free(rm);
    free(cm);
}

/* ------------------------------------------------------------------------ */
/* Exact enumeration of all q^L states of a tiny model at inverse            */
/* temperature beta: log Z = log sum_s exp(-beta E(s)) (log-sum-exp), exact  */
/* marginals p1 [L*q] and p2 [Lq*Lq] (diagonal blocks delta_ab p_i(a)).       */
/* Returns 0, or -1 if q^L exceeds 2^24.                                       */
/* ------------------------------------------------------------------------ */
int orc_enumerate(const float* h, const float* J, int32_t L, int32_t q,
                  double beta, double* p1, double* p2, double* logZ)
{
    const int64_t Lq = (int64_t)L * q;
    double nstates_d = pow((double)q, (double)L);
    if (nstates_d > 16777216.0) return -1;
    int64_t nstates = (int64_t)nstates_d;
    int8_t* s = (int8_t*)malloc((size_t)L);
    double* lw = (double*)malloc(sizeof(double) * (size_t)nstates);
    double mx = -INFINITY;
    for (int64_t k = 0; k < nstates; ++k) {
        int64_t t = k;
        for (int32_t i = L - 1; i >= 0; --i) { s[i] = (int8_t)(t % q); t /= q; }
        lw[k] = -beta * orc_energy_one(h, J, s, L, q);
        if (lw[k] > mx) mx = lw[k];
    }
    double Z = 0.0;
    for (int64_t k = 0; k < nstates; ++k) Z += exp(lw[k] - mx);
    *logZ = mx + log(Z);
    memset(p1, 0, sizeof(double) * (size_t)Lq);
    memset(p2, 0, sizeof(double) * (size_t)Lq * (size_t)Lq);
    for (int64_t k = 0; k < nstates; ++k) {
        int64_t t = k;
        for (int32_t i = L - 1; i >= 0; --i) { s[i] = (int8_t)(t % q); t /= q; }
        double p = exp(lw[k] - *logZ);
        for (int32_t i = 0; i < L; ++i) {
            p1[i * q + s[i]] += p;
            for (int32_t j = 0; j < L; ++j) p2[IDX2(i * q + s[i], j * q + s[j], Lq)] += p;
        }
    }
    free(s);
    free(lw);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Single entries of the definitions above, for checks at sizes where the    */
/* full tables are too slow to build here.  Same arithmetic, same order.     */
/* ------------------------------------------------------------------------ */

/* n_sim for the listed rows only (Eq. 7). */
void orc_reweight_rows(const int8_t* msa, int64_t M, int32_t L, double theta,
                       const int64_t* rows, int64_t nrows, int32_t* n_sim)
{
    int32_t T = orc_identity_threshold(theta, L);
    for (int64_t k = 0; k < nrows; ++k) {
        const int64_t m = rows[k];
        int32_t count = 0;
        for (int64_t n = 0; n < M; ++n) {
            int32_t same = 0;
            for (int32_t i = 0; i < L; ++i)
                same += (msa[m * L + i] == msa[n * L + i]);
            if (same >= T) count += 1;
        }
        n_sim[k] = count;
    }
}

/* f2'[(r1),(r2)] for the listed pairs (Eqs. 3, 8, 9), given M_eff as
 * computed by orc_stats (sum of w in ascending m). */
void orc_stats_entries(const int8_t* X, const double* w, int64_t M, int32_t L,
                       int32_t q, double pseudocount, const int64_t* r1,
                       const int64_t* r2, int64_t n, double* out)
{
    double meff = 0.0;
    for (int64_t m = 0; m < M; ++m) meff += (w ? w[m] : 1.0);
    const double alpha = pseudocount < 0.0 ? 1.0 / meff : pseudocount;
    const double qq = (double)q * (double)q;
    for (int64_t k = 0; k < n; ++k) {
        const int32_t i = (int32_t)(r1[k] / q), a = (int32_t)(r1[k] % q);
        const int32_t j = (int32_t)(r2[k] / q), b = (int32_t)(r2[k] % q);
        double s = 0.0;
        if (i == j) {
            for (int64_t m = 0; m < M; ++m)
                if (X[m * L + i] == a) s += (w ? w[m] : 1.0);
            double f1 = s / meff;
            double t1 = (1.0 - alpha) * f1;
            double t2 = alpha / (double)q;
            out[k] = (a == b) ? t1 + t2 : 0.0;
        } else {
            for (int64_t m = 0; m < M; ++m)
                if (X[m * L + i] == a && X[m * L + j] == b) s += (w ? w[m] : 1.0);
            double f = s / meff;
            double t1 = (1.0 - alpha) * f;
            double t2 = alpha / qq;
            out[k] = t1 + t2;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Equilibrium sampling of a trained model (Sec. 4.1, sampling and its       */
/* convergence criterion): chains start from data sequences drawn according  */
/* to their weights and are compared with a permuted copy of themselves      */
/* (SeqID(t)) and with themselves at time t/2 (SeqID(t, t/2)).               */
/* ------------------------------------------------------------------------ */

/* Weighted draw with replacement of n row indices, row m with probability
 * w_m / W.  With the prefix sums C_m = w_0 + ... + w_m (ascending m) and
 * W = C_{M-1}, draw k takes u from counter (k/4, 0, 0, 2), word k%4,
 * u = (word >> 8) 2^-24, and returns the first m with C_m > u W.  When
 * margins != NULL, margins[k] = distance from u W to the nearest C_m. */
void orc_draw_rows(const double* w, int64_t M, int64_t n, uint64_t seed,
                   int32_t* rows, double* margins)
{
    double* C = (double*)malloc(sizeof(double) * (size_t)M);
    double run = 0.0;
    for (int64_t m = 0; m < M; ++m) {
        run += w[m];
        C[m] = run;
    }
    const double W = C[M - 1];
    for (int64_t k = 0; k < n; ++k) {
        uint32_t word = philox_word(seed, (uint32_t)(k >> 2), 0u, 0u, 2u, (int)(k & 3));
        const double t = (double)(word >> 8) * (1.0 / 16777216.0) * W;
        int64_t m = 0;
        while (C[m] <= t) ++m;
        rows[k] = (int32_t)m;
        if (margins) {
            double d = C[m] - t;
            if (m > 0 && t - C[m - 1] < d) d = t - C[m - 1];
            margins[k] = d;
        }
    }
    free(C);
}

/* SeqID(a, b) = (1/L) sum_i [a_i == b_i], the normalised overlap.  Over the
 * N pairs (A[k], B[perm[k]]) (B[k] when perm is NULL): out[0] = the mean
 * SeqID, out[1] = its standard deviation over the pairs, both from the exact
 * integer sums S1 = sum_k n_k and S2 = sum_k n_k^2 of the identity counts
 * n_k: mean = S1 / (N L), var = S2 / (N L^2) - mean^2 (0 if negative). */
void orc_seqid(const int8_t* A, const int8_t* B, const int32_t* perm, int64_t N,
               int32_t L, double* out)
{
    int64_t S1 = 0, S2 = 0;
    for (int64_t k = 0; k < N; ++k) {
        const int8_t* b = B + (int64_t)(perm ? perm[k] : k) * L;
        int64_t same = 0;
        for (int32_t i = 0; i < L; ++i) same += (A[k * L + i] == b[i]);
        S1 += same;
        S2 += same * same;
    }
    const double mean = (double)S1 / ((double)N * (double)L);
    const double m2 = (double)S2 / ((double)N * (double)L * (double)L);
    const double var = m2 - mean * mean;
    out[0] = mean;
    out[1] = sqrt(var > 0.0 ? var : 0.0);
}

/* ------------------------------------------------------------------------ */
/* Metropolis-Hastings sampling (Sec. 2.1 names it beside Gibbs; the          */
/* sampler options of the training and sampling tables).  The paper does not */
/* write the acceptance rule; this is textbook single-site Metropolis with a  */
/* uniform proposal among the other q-1 states: at site i (order 0..L-1) in   */
/* state a, propose a' uniformly from the q-1 states != a and accept with     */
/* probability min(1, exp(beta (H_i(a') - H_i(a)))), which is the ratio       */
/* P(s')/P(s) of Eq. (1) for a single-site change.  Random words: Philox      */
/* counter (i/2, global sweep, chain, 3), words 2(i%2) (proposal) and         */
/* 2(i%2)+1 (acceptance); a' = (a + 1 + ((word * (q-1)) >> 32)) mod q,        */
/* u = (word >> 8) 2^-24, accept iff u < exp(beta (H_i(a') - H_i(a))).  The   */
/* margin of a visit is |u - min(1, exp(beta (H_i(a') - H_i(a))))|.           */
/* ------------------------------------------------------------------------ */
/* One Metropolis visit of site i (rule above) for chain index c in global
 * sweep sg; returns the state after the visit and its margin. */
static int32_t metropolis_visit(const float* h, const float* J, const int8_t* s,
                                int32_t L, int32_t q, int32_t i, uint64_t c,
                                uint64_t sg, uint64_t seed, double beta, double* Hi,
                                double* margin, int32_t* proposal)
{
    orc_local_field(h, J, s, L, q, i, Hi);
    const uint32_t wp = philox_word(seed, (uint32_t)i >> 1, (uint32_t)sg, (uint32_t)c, 3u,
                                    2 * (i & 1));
    const uint32_t wa = philox_word(seed, (uint32_t)i >> 1, (uint32_t)sg, (uint32_t)c, 3u,
                                    2 * (i & 1) + 1);
    const int32_t a = s[i];
    const int32_t ap = (a + 1 + (int32_t)(((uint64_t)wp * (uint64_t)(q - 1)) >> 32)) % q;
    const double u = (double)(wa >> 8) * (1.0 / 16777216.0);
    const double p = exp(beta * (Hi[ap] - Hi[a]));
    const double pc = p < 1.0 ? p : 1.0;
    *margin = fabs(u - pc);
    *proposal = ap;
    return u < p ? ap : a;
}

void orc_metropolis_range(const float* h, const float* J, int8_t* chains, int64_t N,
                          int64_t c0, int32_t L, int32_t q, int32_t sweeps,
                          uint64_t seed, uint64_t sweep_offset, double beta,
                          double* margins, int64_t* flips)
{
    int64_t nflip = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : nflip)
    for (int64_t c = 0; c < N; ++c) {
        double* Hi = (double*)malloc(sizeof(double) * (size_t)q);
        int8_t* s = chains + c * L;
        for (int32_t sw = 0; sw < sweeps; ++sw) {
            uint64_t sg = sweep_offset + (uint64_t)sw;
            for (int32_t i = 0; i < L; ++i) {
                double margin;
                int32_t ap;
                const int32_t anew = metropolis_visit(h, J, s, L, q, i, (uint64_t)(c0 + c), sg,
                                                      seed, beta, Hi, &margin, &ap);
                if (margins) margins[((size_t)c * sweeps + sw) * L + i] = margin;
                if (anew != s[i]) {
                    s[i] = (int8_t)anew;
                    nflip += 1;
                }
            }
        }
        free(Hi);
    }
    if (flips) *flips = nflip;
}

/* ------------------------------------------------------------------------ */
/* Replay of one chain with forced outcomes (Gibbs when metropolis == 0,      */
/* Metropolis otherwise), for parity tests that must tell a boundary event   */
/* (a draw whose uniform lies within tol of its threshold, which FP32 fields */
/* may resolve the other way) from an error.  Visit v = sw*L + i records the */
/* drawn state drawn[v] and the states alt_lo[v]..alt_hi[v] the visit could */
/* take if every comparison within tol of u went the other way (for          */
/* Metropolis: the other outcome of the acceptance test); where nothing is   */
/* that close both equal drawn[v].  force (may be NULL): where force[v] >= 0 */
/* the chain takes that state at visit v instead of the drawn one.  With no  */
/* forced visit the result is exactly that of orc_gibbs_range /              */
/* orc_metropolis_range for the chain with global index c.                   */
/* ------------------------------------------------------------------------ */
void orc_chain_forced(const float* h, const float* J, int8_t* s, uint64_t c, int32_t L,
                      int32_t q, int32_t sweeps, uint64_t seed, uint64_t sweep_offset,
                      double beta, int32_t metropolis, double tol, const int8_t* force,
                      int8_t* drawn, int8_t* alt_lo, int8_t* alt_hi)
{
    double* Hi = (double*)malloc(sizeof(double) * (size_t)q);
    double* e = (double*)malloc(sizeof(double) * (size_t)q);
    double* cdf = (double*)malloc(sizeof(double) * (size_t)q);
    for (int32_t sw = 0; sw < sweeps; ++sw) {
        uint64_t sg = sweep_offset + (uint64_t)sw;
        for (int32_t i = 0; i < L; ++i) {
            const size_t v = (size_t)sw * L + i;
            double margin;
            int32_t anew, lo, hi;
            if (metropolis) {
                int32_t ap;
                const int32_t a = s[i];
                anew = metropolis_visit(h, J, s, L, q, i, c, sg, seed, beta, Hi, &margin, &ap);
                lo = hi = anew;
                if (margin < tol) lo = hi = (anew == ap) ? a : ap;
            } else {
                orc_local_field(h, J, s, L, q, i, Hi);
                const double u = orc_gibbs_uniform(seed, c, sg, i);
                int32_t nlo, nhi;
                anew = gibbs_draw(Hi, q, beta, u, e, cdf, tol, &margin, &nlo, &nhi);
                lo = anew - nlo;
                hi = anew + nhi;
            }
            drawn[v] = (int8_t)anew;
            alt_lo[v] = (int8_t)lo;
            alt_hi[v] = (int8_t)hi;
            s[i] = (int8_t)((force && force[v] >= 0) ? force[v] : anew);
        }
    }
    free(Hi);
    free(e);
    free(cdf);
}

/* ------------------------------------------------------------------------ */
/* Element decimation (edDCA, Sec. 2.2 "Element decimation DCA"): prune the   */
/* active coupling elements whose removal perturbs the model least, measured  */
/* by the symmetric Kullback-Leibler distance between the current model P and */
/* P' = P with the single element J_ij(a,b) set to zero.                     */
/*                                                                          */
/* With x(s) = [s_i == a][s_j == b] and p = E_P[x], Eq. (1) gives             */
/* P'(s) = P(s) exp(-J x(s)) Z / Z', Z'/Z = E_P[exp(-J x)] = 1 - p + p e^-J,  */
/* hence KL(P||P') = J p + log(1 - p + p e^-J), KL(P'||P) = -J p' - log(...), */
/* p' = E_P'[x] = p e^-J / (1 - p + p e^-J), and the symmetric distance is    */
/* J (p - p') >= 0.  p is estimated by the chain frequency count / N.         */
/* ------------------------------------------------------------------------ */
double orc_skl_element(double J, double p)
{
    const double e = exp(-J);
    const double d = 1.0 - p + p * e;
    const double pp = p * e / d;
    return J * (p - pp);
}

typedef struct {
    double score;
    int64_t key; /* r1 * Lq + r2, r1 < r2 */
} orc_scored;

static int orc_scored_cmp(const void* a, const void* b)
{
    const orc_scored* x = (const orc_scored*)a;
    const orc_scored* y = (const orc_scored*)b;
    if (x->score < y->score) return -1;
    if (x->score > y->score) return 1;
    return (x->key < y->key) ? -1 : (x->key > y->key);
}

/* One graph update.  Elements are the unordered pairs of vertices (r1, r2)
 * with r1 < r2 in different sites; mask [Lq][Lq] (1 = active) and J are kept
 * symmetric.  n_total = L (L-1) q^2 / 2; n_target = ceil(density n_total);
 * with n_act active elements, k = min(max(1, floor(drate n_act)), n_act -
 * n_target) elements (none if n_act <= n_target) with the smallest
 * (score, r1 Lq + r2) are removed (mask = 0 and J = 0 on both triangles).
 * Returns the number of active elements afterwards. */
int64_t orc_decimate(float* J, uint8_t* mask, const int8_t* chains, int64_t N, int32_t L,
                     int32_t q, double drate, double density)
{
    const int64_t Lq = (int64_t)L * q;
    double* p1 = (double*)malloc(sizeof(double) * (size_t)Lq);
    double* p2 = (double*)malloc(sizeof(double) * (size_t)Lq * (size_t)Lq);
    orc_chain_freqs(chains, N, L, q, p1, p2);
    const int64_t n_total = (int64_t)L * (L - 1) / 2 * q * q;
    const int64_t n_target = (int64_t)ceil(density * (double)n_total);
    orc_scored* s = (orc_scored*)malloc(sizeof(orc_scored) * (size_t)n_total);
    int64_t n_act = 0;
    for (int64_t r1 = 0; r1 < Lq; ++r1)
        for (int64_t r2 = r1 + 1; r2 < Lq; ++r2) {
            if (r1 / q == r2 / q) continue;
            const size_t k = IDX2(r1, r2, Lq);
            if (!mask[k]) continue;
            s[n_act].score = orc_skl_element((double)J[k], p2[k]);
            s[n_act].key = r1 * Lq + r2;
            ++n_act;
        }
    int64_t kk = 0;
    if (n_act > n_target) {
        kk = (int64_t)floor(drate * (double)n_act);
        if (kk < 1) kk = 1;
        if (kk > n_act - n_target) kk = n_act - n_target;
    }
    qsort(s, (size_t)n_act, sizeof(orc_scored), orc_scored_cmp);
    for (int64_t t = 0; t < kk; ++t) {
        const int64_t r1 = s[t].key / Lq, r2 = s[t].key % Lq;
        mask[IDX2(r1, r2, Lq)] = 0;
        mask[IDX2(r2, r1, Lq)] = 0;
        J[IDX2(r1, r2, Lq)] = 0.0f;
        J[IDX2(r2, r1, Lq)] = 0.0f;
    }
    free(s);
    free(p1);
    free(p2);
    return n_act - kk;
}

/* ------------------------------------------------------------------------ */
/* Element activation (eaDCA, Sec. 2.2 "Element activation DCA"): starting   */
/* from an empty graph, each graph update targets a number of elements equal */
/* to the fraction factivate of the currently inactive ones and activates,   */
/* among all elements (i < j, a, b) -- active ones included, which is why    */
/* fewer may be added -- those whose model pairwise marginal p_ij(a,b) is    */
/* farthest from the data's f_ij(a,b).  The paper leaves the distance to a   */
/* citation; the reading here is the Kullback-Leibler divergence between the */
/* two Bernoulli variables [s_i == a][s_j == b] under the data and under the */
/* model:  D(f || p) = f log(f/p) + (1-f) log((1-f)/(1-p)),                  */
/* with 0 log(0/x) = 0 and +inf where the data has mass the model lacks.     */
/* Count: k = max(1, floor(factivate n_inactive)) (0 when none is inactive); */
/* the k largest (D, then smallest r1 Lq + r2) are set active.               */
/* ------------------------------------------------------------------------ */
double orc_bernoulli_kl(double f, double p)
{
    double d = 0.0;
    if (f > 0.0) d += (p > 0.0) ? f * log(f / p) : INFINITY;
    if (f < 1.0) d += (p < 1.0) ? (1.0 - f) * log((1.0 - f) / (1.0 - p)) : INFINITY;
    return d > 0.0 ? d : 0.0;
}

static int orc_scored_cmp_desc(const void* a, const void* b)
{
    const orc_scored* x = (const orc_scored*)a;
    const orc_scored* y = (const orc_scored*)b;
    if (x->score > y->score) return -1;
    if (x->score < y->score) return 1;
    return (x->key < y->key) ? -1 : (x->key > y->key);
}

int64_t orc_activate(uint8_t* mask, const int8_t* chains, int64_t N, int32_t L, int32_t q,
                     const double* f2, double factivate)
{
    const int64_t Lq = (int64_t)L * q;
    double* p1 = (double*)malloc(sizeof(double) * (size_t)Lq);
    double* p2 = (double*)malloc(sizeof(double) * (size_t)Lq * (size_t)Lq);
    orc_chain_freqs(chains, N, L, q, p1, p2);
    const int64_t n_total = (int64_t)L * (L - 1) / 2 * q * q;
    orc_scored* s = (orc_scored*)malloc(sizeof(orc_scored) * (size_t)n_total);
    int64_t n = 0, n_act = 0;
    for (int64_t r1 = 0; r1 < Lq; ++r1)
        for (int64_t r2 = r1 + 1; r2 < Lq; ++r2) {
            if (r1 / q == r2 / q) continue;
            const size_t k = IDX2(r1, r2, Lq);
            if (mask[k]) ++n_act;
            s[n].score = orc_bernoulli_kl(f2[k], p2[k]);
            s[n].key = r1 * Lq + r2;
            ++n;
        }
    const int64_t n_inact = n_total - n_act;
    int64_t kk = 0;
    if (n_inact > 0) {
        kk = (int64_t)floor(factivate * (double)n_inact);
        if (kk < 1) kk = 1;
    }
    qsort(s, (size_t)n, sizeof(orc_scored), orc_scored_cmp_desc);
    int64_t added = 0;
    for (int64_t t = 0; t < kk; ++t) {
        const int64_t r1 = s[t].key / Lq, r2 = s[t].key % Lq;
        if (!mask[IDX2(r1, r2, Lq)]) ++added;
        mask[IDX2(r1, r2, Lq)] = 1;
        mask[IDX2(r2, r1, Lq)] = 1;
    }
    free(s);
    free(p1);
    free(p2);
    return n_act + added;
}

/* Eq. (5) on a sparse graph: as orc_update, with inactive elements (mask 0)
 * held at zero. */
void orc_update_masked(float* h, float* J, const uint8_t* mask, const double* f1,
                       const double* f2, const double* p1, const double* p2, int32_t L,
                       int32_t q, double lr)
{
    const int64_t Lq = (int64_t)L * q;
    orc_update(h, J, f1, f2, p1, p2, L, q, lr);
    for (int64_t k = 0; k < Lq * Lq; ++k)
        if (!mask[k]) J[k] = 0.0f;
}

/* orc_train_step on a sparse graph (masked update). */
double orc_train_step_masked(float* h, float* J, const uint8_t* mask, int8_t* chains,
                             int64_t N, int32_t L, int32_t q, const double* f1,
                             const double* f2, double lr, int32_t sweeps, uint64_t seed,
                             uint64_t epoch, double* margins, int64_t* flips)
{
    const int64_t Lq = (int64_t)L * q;
    orc_gibbs(h, J, chains, N, L, q, sweeps, seed, epoch * (uint64_t)sweeps, 1.0,
              margins, flips);
    double* p1 = (double*)malloc(sizeof(double) * (size_t)Lq);
    double* p2 = (double*)malloc(sizeof(double) * (size_t)Lq * (size_t)Lq);
    orc_chain_freqs(chains, N, L, q, p1, p2);
    double r = orc_pearson(f1, f2, p1, p2, L, q);
    orc_update_masked(h, J, mask, f1, f2, p1, p2, L, q, lr);
    free(p1);
    free(p2);
    return r;
}

/* ------------------------------------------------------------------------ */
/* Starting point and coupling graphs.                                       */
/* ------------------------------------------------------------------------ */

/* Independent-site (profile) model: h[(i,a)] = (float) log f1[(i,a)]; with
 * J = 0 its one-site marginals are f_i(a) when each f_i sums to 1. */
void orc_profile_fields(const double* f1, int32_t L, int32_t q, float* h)
{
    for (int64_t r = 0; r < (int64_t)L * q; ++r) h[r] = (float)log(f1[r]);
}

/* Couplings restricted to a graph (Sec. 2.2): J = 0 wherever the mask is 0
 * or both indices lie on one site; returns the number of active elements
 * r1 < r2 of different sites. */
int64_t orc_mask_apply(float* J, const uint8_t* mask, int32_t L, int32_t q)
{
    const int64_t Lq = (int64_t)L * q;
    int64_t n = 0;
    for (int64_t r1 = 0; r1 < Lq; ++r1)
        for (int64_t r2 = 0; r2 < Lq; ++r2) {
            const int on = mask[IDX2(r1, r2, Lq)] != 0 && r1 / q != r2 / q;
            if (!on && J) J[IDX2(r1, r2, Lq)] = 0.0f;
            if (on && r1 < r2) n += 1;
        }
    return n;
}
