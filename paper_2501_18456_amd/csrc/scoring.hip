// Downstream scores of a trained model (adabmDCA 2.0, Sec. 4):
//   - energies of a batch of sequences, Eq. (1) (Sec. 4.3);
//   - single-mutant energy differences from the wild type's local fields
//     (Sec. 4.4);
//   - zero-sum-gauge Frobenius norms with the average-product correction,
//     Eq. (13) (Sec. 4.2).
#include "common.hpp"
#include "internal.hpp"

namespace bmdca {

// ---------------------------------------------------------------------------
// Energy, one wave64 per sequence: FP32 terms accumulated in FP64 per lane,
// then a fixed-order wave reduction; rounded once to FP32.
// ---------------------------------------------------------------------------
constexpr int kEnergyWaves = 4;

__global__ __launch_bounds__(kEnergyWaves * 64) void k_energy(const float* __restrict__ h,
                                                              const float* __restrict__ J,
                                                              const int8_t* __restrict__ seqs,
                                                              int64_t B, int L, int q,
                                                              float* __restrict__ E,
                                                              int32_t* dev_err) {
  extern __shared__ int cols_all[];  // per wave: L entries (j*q + s_j)
  const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
  const int64_t b = (int64_t)blockIdx.x * kEnergyWaves + wid;
  if (b >= B) return;
  int* cols = cols_all + wid * L;
  const int Lq = L * q;
  for (int i = lane; i < L; i += 64) cols[i] = i * q + checked_token(seqs[b * L + i], q, dev_err);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
  double acc = 0.0;
  for (int i = lane; i < L; i += 64) acc -= (double)h[cols[i]];
  for (int i = 0; i < L; ++i) {
    const float* __restrict__ row = J + (size_t)cols[i] * Lq;
    for (int j = i + 1 + lane; j < L; j += 64) acc -= (double)row[cols[j]];
  }
  acc = wave_sum_f64(acc);
  if (lane == 0) E[b] = (float)acc;
}

hipError_t launch_energy(const float* h, const float* J, const int8_t* seqs, int64_t B, int L,
                         int q, float* E, int32_t* dev_err, hipStream_t s) {
  hipLaunchKernelGGL(k_energy, dim3((unsigned)ceil_div(B, kEnergyWaves)), dim3(kEnergyWaves * 64),
                     sizeof(int) * L * kEnergyWaves, s, h, J, seqs, B, L, q, E, dev_err);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Single mutants: dE[b][i*q+a] = -(H[b][i*q+a] - H[b][i*q+wt_i]), with H the
// wild type's local fields (h + sum_{j != i} J_ij(., wt_j)).
// ---------------------------------------------------------------------------
__global__ void k_mutant_delta(const float* __restrict__ H, const int8_t* __restrict__ wt,
                               int64_t B, int L, int q, float* __restrict__ dE) {
  const int64_t Lq = (int64_t)L * q;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * Lq) return;
  const int64_t b = idx / Lq;
  const int r = (int)(idx % Lq);
  const int i = r / q;
  int w = wt[b * L + i];
  if (w < 0 || w >= q) w = 0;  // flagged by the field build
  const float* Hb = H + b * Lq;
  dE[idx] = (r == i * q + w) ? 0.0f : -(Hb[r] - Hb[i * q + w]);
}

hipError_t launch_mutant_delta(const float* H, const int8_t* wt, int64_t B, int L, int q,
                               float* dE, hipStream_t s) {
  const int64_t total = B * (int64_t)L * q;
  hipLaunchKernelGGL(k_mutant_delta, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, H, wt,
                     B, L, q, dE);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// APC Frobenius.  k_frob: one workgroup per unordered pair i < j; the q x q
// block is moved to the zero-sum gauge over all states (FP64) and the squares
// of the entries with a, b != gap are summed (fixed tree).  k_apc: row sums
// S_i in ascending k, the total in ascending i, F_apc = F - S_i S_j / S.
// ---------------------------------------------------------------------------
size_t apc_ws_bytes(int L) { return align256(sizeof(double) * ((size_t)L * L + L + 8)); }

__global__ __launch_bounds__(256) void k_frob(const float* __restrict__ J, int L, int q, int gap,
                                              double* __restrict__ F) {
  __shared__ double blk[32 * 32];
  __shared__ double rm[32], cm[32];
  __shared__ double sh[16];
  int t = blockIdx.x, i = 0;
  while (t >= L - 1 - i) {
    t -= L - 1 - i;
    ++i;
  }
  const int j = i + 1 + t;
  const int Lq = L * q;
  for (int k = threadIdx.x; k < q * q; k += blockDim.x) {
    const int a = k / q, b = k % q;
    blk[k] = (double)J[(size_t)(i * q + a) * Lq + j * q + b];
  }
  __syncthreads();
  if (threadIdx.x < q) {
    double s = 0.0;
    for (int b = 0; b < q; ++b) s += blk[threadIdx.x * q + b];
    rm[threadIdx.x] = s / (double)q;
  } else if (threadIdx.x >= 64 && threadIdx.x < 64 + q) {
    const int b = threadIdx.x - 64;
    double s = 0.0;
    for (int a = 0; a < q; ++a) s += blk[a * q + b];
    cm[b] = s / (double)q;
  }
  __syncthreads();
  double all = 0.0;
  for (int a = 0; a < q; ++a) all += rm[a];
  all /= (double)q;
  double ss = 0.0;
  for (int k = threadIdx.x; k < q * q; k += blockDim.x) {
    const int a = k / q, b = k % q;
    if (a == gap || b == gap) continue;
    const double z = blk[k] - rm[a] - cm[b] + all;
    ss += z * z;
  }
  const double tot = block_sum_f64(ss, sh);
  if (threadIdx.x == 0) {
    const double f = sqrt(tot);
    F[(size_t)i * L + j] = f;
    F[(size_t)j * L + i] = f;
  }
}

__global__ __launch_bounds__(1024) void k_apc(double* __restrict__ F, int L,
                                              float* __restrict__ Fout,
                                              float* __restrict__ Fapc) {
  extern __shared__ double S[];  // L + 1
  for (int i = threadIdx.x; i < L; i += blockDim.x) {
    F[(size_t)i * L + i] = 0.0;
    double s = 0.0;
    for (int k = 0; k < L; ++k) s += (k == i) ? 0.0 : F[(size_t)i * L + k];
    S[i] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int i = 0; i < L; ++i) tot += S[i];
    S[L] = tot;
  }
  __syncthreads();
  const double tot = S[L];
  for (size_t k = threadIdx.x; k < (size_t)L * L; k += blockDim.x) {
    const int i = (int)(k / L), j = (int)(k % L);
    const double f = (i == j) ? 0.0 : F[k];
    if (Fout) Fout[k] = (float)f;
    Fapc[k] = (i == j) ? 0.0f : (float)(f - S[i] * S[j] / tot);
  }
}

hipError_t launch_apc(const float* J, int L, int q, int gap, float* F, float* Fapc, void* ws,
                      hipStream_t s) {
  double* Fd = static_cast<double*>(ws);
  const int npairs = L * (L - 1) / 2;
  hipLaunchKernelGGL(k_frob, dim3((unsigned)npairs), dim3(256), 0, s, J, L, q, gap, Fd);
  hipLaunchKernelGGL(k_apc, dim3(1), dim3(1024), sizeof(double) * (L + 1), s, Fd, L, F, Fapc);
  return hipGetLastError();
}

}  // namespace bmdca
