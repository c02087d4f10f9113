// Boltzmann-learning epilogue of one epoch (adabmDCA 2.0, Sec. 2.1):
//   - the convergence check: Pearson correlation between the connected
//     correlations of data and model (Eq. 6), over i < j and all a, b;
//   - the parameter update of Eq. (5).
// Both read the chain counts C (FP64, full symmetric [Lq][Lq], exact
// integers) and form p = C / N in FP64.  Contraction is off for this file, so
// every expression is rounded exactly as written.
#include "common.hpp"
#include "internal.hpp"

namespace bmdca {

constexpr int kPearsonBlocks = 1024;
constexpr int kPearsonThreads = 256;

size_t pearson_red_bytes() { return sizeof(double) * (3 * kPearsonBlocks + 8); }

// Pass 0: per-workgroup sums of x and y; pass 1: of dx^2, dy^2, dx*dy about
// the means.  x = f2 - f1_i f1_j (data), y = p2 - p1_i p1_j (model), over the
// entries (r1, c) with site(r1) < site(c).  Workgroup (column block b, row
// chunk g) owns columns 256 b + t (one per thread: its f1 and p1 stay in
// registers) and rows g, g + G, ...; a row's values are uniform, so the
// reads of f2 and C are coalesced and nothing is divided per entry but C/N.
__global__ __launch_bounds__(kPearsonThreads) void k_pearson_pass(
    const double* __restrict__ f1, const double* __restrict__ f2, const double* __restrict__ C,
    int64_t N, int L, int q, int pass, int nrow_chunks, double* __restrict__ red) {
  __shared__ double sh[16];
  const int Lq = L * q;
  const double dn = (double)N;
  double mx = 0.0, my = 0.0;
  if (pass == 1) {
    mx = red[3 * kPearsonBlocks + 0];
    my = red[3 * kPearsonBlocks + 1];
  }
  const int b = blockIdx.x / nrow_chunks, g = blockIdx.x % nrow_chunks;
  const int c = b * kPearsonThreads + (int)threadIdx.x;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  if (c < Lq) {
    const int rmax = (c / q) * q;  // rows of the sites before c's
    const double f1c = f1[c];
    const double p1c = C[(size_t)c * Lq + c] / dn;
    for (int r1 = g; r1 < rmax; r1 += nrow_chunks) {
      const size_t k = (size_t)r1 * Lq + c;
      const double x = f2[k] - f1[r1] * f1c;
      const double p1r = C[(size_t)r1 * Lq + r1] / dn;
      const double y = C[k] / dn - p1r * p1c;
      if (pass == 0) {
        s0 += x;
        s1 += y;
      } else {
        const double dx = x - mx, dy = y - my;
        s0 += dx * dx;
        s1 += dy * dy;
        s2 += dx * dy;
      }
    }
  }
  const double t0 = block_sum_f64(s0, sh);
  const double t1 = block_sum_f64(s1, sh);
  const double t2 = block_sum_f64(s2, sh);
  if (threadIdx.x == 0) {
    red[3 * blockIdx.x + 0] = t0;
    red[3 * blockIdx.x + 1] = t1;
    red[3 * blockIdx.x + 2] = t2;
  }
}

// Sums the nblk workgroup partials: thread t adds partials t, t + 256, ... in
// order, then a fixed tree over the 256 threads (one workgroup,
// deterministic).  Pass 0: means into red's tail; pass 1: the coefficient
// into *out.
__global__ __launch_bounds__(256) void k_pearson_finish(double* __restrict__ red, int nblk, int L,
                                                        int q, int pass, double* __restrict__ out,
                                                        int32_t* dev_err) {
  __shared__ double part[3][256];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int k = threadIdx.x; k < nblk; k += 256) {
    a += red[3 * k + 0];
    b += red[3 * k + 1];
    c += red[3 * k + 2];
  }
  part[0][threadIdx.x] = a;
  part[1][threadIdx.x] = b;
  part[2][threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      part[0][threadIdx.x] += part[0][threadIdx.x + w];
      part[1][threadIdx.x] += part[1][threadIdx.x + w];
      part[2][threadIdx.x] += part[2][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  a = part[0][0];
  b = part[1][0];
  c = part[2][0];
  if (pass == 0) {
    const double n = (double)L * (double)(L - 1) / 2.0 * (double)q * (double)q;
    red[3 * kPearsonBlocks + 0] = a / n;
    red[3 * kPearsonBlocks + 1] = b / n;
  } else {
    const double r = c / sqrt(a * b);
    *out = r;
    if (!isfinite(r) && dev_err) atomicOr(dev_err, 2);
  }
}

hipError_t launch_pearson(const double* f1, const double* f2, const double* C, int64_t N, int L,
                          int q, double* red, double* out, int32_t* dev_err, hipStream_t s) {
  // column blocks x row chunks, at most kPearsonBlocks partials
  const int Lq = L * q;
  const int ncb = (int)ceil_div(Lq, kPearsonThreads);
  const int nrc = std::max(1, std::min(kPearsonBlocks / ncb, Lq));
  const int nblk = ncb * nrc;
  if (nblk > kPearsonBlocks) return hipErrorInvalidValue;  // Lq > 256 x 1024
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_pearson_pass, dim3(nblk), dim3(kPearsonThreads), 0, s, f1, f2, C, N, L,
                       q, pass, nrc, red);
    hipLaunchKernelGGL(k_pearson_finish, dim3(1), dim3(256), 0, s, red, nblk, L, q, pass, out,
                       dev_err);
  }
  return hipGetLastError();
}

// Eq. (5): J_ij(a,b) += lr (f_ij(a,b) - p_ij(a,b)) for i != j, J_ii = 0;
// h_i(a) += lr (f_i(a) - p_i(a)); FP64, one rounding to FP32.
__global__ void k_update(float* __restrict__ h, float* __restrict__ J,
                         const double* __restrict__ f1, const double* __restrict__ f2,
                         const double* __restrict__ C, int64_t N, int L, int q, double lr,
                         int32_t* dev_err, const int32_t* __restrict__ active,
                         const uint8_t* __restrict__ mask) {
  if (active && *active == 0) return;
  const int Lq = L * q;
  const double dn = (double)N;
  bool bad = false;
  // rows r1 = blockIdx.x, + gridDim.x, ...; the threads stride over the
  // columns, and the diagonal block of row r1 is a column range
  for (int r1 = blockIdx.x; r1 < Lq; r1 += gridDim.x) {
    const int d0 = (r1 / q) * q;
    for (int r2 = threadIdx.x; r2 < Lq; r2 += blockDim.x) {
      const size_t k = (size_t)r1 * Lq + r2;
      if ((r2 >= d0 && r2 < d0 + q) || (mask && !mask[k])) {  // diagonal block or pruned
        J[k] = 0.0f;
        continue;
      }
      const double d = f2[k] - C[k] / dn;
      const double t = lr * d;
      const float v = (float)((double)J[k] + t);
      J[k] = v;
      bad |= !isfinite(v);
    }
  }
  for (size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x; r < (size_t)Lq;
       r += (size_t)gridDim.x * blockDim.x) {
    const double d = f1[r] - C[r * Lq + r] / dn;
    const double t = lr * d;
    const float v = (float)((double)h[r] + t);
    h[r] = v;
    bad |= !isfinite(v);
  }
  if (bad && dev_err) atomicOr(dev_err, 2);
}

hipError_t launch_update(float* h, float* J, const double* f1, const double* f2, const double* C,
                         int64_t N, int L, int q, double lr, int32_t* dev_err, hipStream_t s,
                         const int32_t* active, const uint8_t* mask) {
  const unsigned nb = (unsigned)std::min(L * q, 16384);  // a row per workgroup (and step)
  hipLaunchKernelGGL(k_update, dim3(nb), dim3(256), 0, s, h, J, f1, f2, C, N, L, q, lr, dev_err,
                     active, mask);
  return hipGetLastError();
}

// Layout of the public bmdca_train_ctl record (bmdca.h): epoch u64 at 0,
// active i32 at 8, converged_at i32 at 12, target f64 at 16.
struct CtlRecord {
  uint64_t epoch;
  int32_t active;
  int32_t converged_at;
  double target;
};
static_assert(sizeof(CtlRecord) == 24, "control record layout");

__global__ void k_ctl_advance(CtlRecord* __restrict__ ctl, const double* __restrict__ pearson) {
  if (threadIdx.x != 0 || ctl->active == 0) return;
  ctl->epoch += 1;
  const double r = *pearson;
  if (ctl->target > 0.0 && r >= ctl->target) {
    ctl->active = 0;
    ctl->converged_at = (int32_t)ctl->epoch;
  }
}

hipError_t launch_ctl_advance(void* ctl, const double* pearson, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_advance, dim3(1), dim3(64), 0, s, static_cast<CtlRecord*>(ctl), pearson);
  return hipGetLastError();
}

// Independent-site (profile) model: h_i(a) = log f_i(a) in FP64, rounded
// once to float32.  With J = 0 its one-site marginals are
// exp(h_i(a)) / sum_b exp(h_i(b)) = f_i(a), since each f_i sums to 1.  A
// frequency that is not positive and finite gives a non-finite field and
// raises BMDCA_DEVERR_NONFINITE.
__global__ void k_profile_fields(const double* __restrict__ f1, int Lq, float* __restrict__ h,
                                 int32_t* dev_err) {
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < Lq; r += gridDim.x * blockDim.x) {
    const float v = (float)log(f1[r]);
    h[r] = v;
    if (!isfinite(v) && dev_err) atomicOr(dev_err, 2);
  }
}

hipError_t launch_profile_fields(const double* f1, int L, int q, float* h, int32_t* dev_err,
                                 hipStream_t s) {
  const int Lq = L * q;
  hipLaunchKernelGGL(k_profile_fields, dim3((unsigned)ceil_div(Lq, 256)), dim3(256), 0, s, f1, Lq,
                     h, dev_err);
  return hipGetLastError();
}

__global__ void k_tick_advance(uint64_t* __restrict__ tick) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *tick += 1;
}

hipError_t launch_tick_advance(uint64_t* tick, hipStream_t s) {
  hipLaunchKernelGGL(k_tick_advance, dim3(1), dim3(64), 0, s, tick);
  return hipGetLastError();
}

}  // namespace bmdca
