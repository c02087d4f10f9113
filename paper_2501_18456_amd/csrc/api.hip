// C-ABI entry points of libbmdca (declared in include/bmdca.h): host-side
// validation, workspace carve-up, and the kernel sequence of each call.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/bmdca.h"
#include "common.hpp"
#include "internal.hpp"

using namespace bmdca;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return BMDCA_OK;
  return fail(BMDCA_EHIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr int kMaxL = 1024;
constexpr int kMaxQ = 32;

int check_model(int32_t L, int32_t q) {
  if (L < 1 || L > kMaxL) return fail(BMDCA_EINVAL, "L=%d outside 1..%d", L, kMaxL);
  if (q < 2 || q > kMaxQ) return fail(BMDCA_EINVAL, "q=%d outside 2..%d", q, kMaxQ);
  return BMDCA_OK;
}

#define BMDCA_REQUIRE(cond, ...) \
  do {                           \
    if (!(cond)) return fail(BMDCA_EINVAL, __VA_ARGS__); \
  } while (0)

#define BMDCA_TRY(expr)               \
  do {                                \
    int _rc = (expr);                 \
    if (_rc != BMDCA_OK) return _rc;  \
  } while (0)

size_t gibbs_bytes(int64_t N, int L, int q) { return align256(sizeof(float) * (size_t)N * L * q); }

constexpr int kPrecMask = 0x0F;
constexpr int kSamplerMask = BMDCA_SAMPLER_FIELDS | BMDCA_SAMPLER_GATHER | BMDCA_SAMPLER_METROPOLIS;

// Sampler choice: 1 = gather form, 0 = field form, -1 = invalid request
// (the same for the heat-bath draw and for Metropolis).
int pick_gather(int flags, int L, int q) {
  const int sel = flags & (BMDCA_SAMPLER_FIELDS | BMDCA_SAMPLER_GATHER);
  if (sel == (BMDCA_SAMPLER_FIELDS | BMDCA_SAMPLER_GATHER)) return -1;
  if (sel == BMDCA_SAMPLER_FIELDS) return 0;
  const bool ok = gather_supported(L, q);
  if (sel == BMDCA_SAMPLER_GATHER) return ok ? 1 : -1;
  return ok ? 1 : 0;
}

// Sampler scratch: the local fields (field form) or the re-laid-out
// coupling blocks (gather form).
size_t field_bytes(int64_t N, int L, int q, int flags) {
  return pick_gather(flags, L, q) == 1 ? gather_ws_bytes(L, q) : gibbs_bytes(N, L, q);
}

// Train-step workspace: H, chain-count planes (via the stats plan over N
// rows), full count matrix C, Pearson reductions.
struct TrainPlan {
  StatsPlan sp;
  size_t off_H, off_stats, off_C, off_red, total;
};

TrainPlan plan_train(int64_t N, int L, int q, int prec) {
  TrainPlan t{};
  const size_t Lq = (size_t)L * q;
  t.sp = plan_stats(N, L, q, prec & kPrecMask);
  size_t o = 0;
  t.off_H = o;     o = align256(o + field_bytes(N, L, q, prec));
  t.off_stats = o; o = align256(o + t.sp.total);
  t.off_C = o;     o = align256(o + sizeof(double) * Lq * Lq);
  t.off_red = o;   o = align256(o + pearson_red_bytes());
  t.total = o;
  return t;
}

// Host validation and launches of a sampling call (plain or with per-chain
// streams in ctl).
int gibbs_impl(const float* h, const float* J, int8_t* chains, int64_t N, int32_t L, int32_t q,
               int32_t sweeps, uint64_t seed, uint64_t sweep_offset, float beta, float* H_ws,
               size_t H_ws_bytes, int32_t flags, unsigned long long* flips_out,
               const DevCtl& ctl_in, hipStream_t s) {
  DevCtl ctl = ctl_in;
  ctl.keep_layout = (flags & BMDCA_GIBBS_KEEP_LAYOUT) != 0;
  BMDCA_TRY(check_model(L, q));
  BMDCA_REQUIRE(h && J && chains, "null pointer argument");
  BMDCA_REQUIRE(N >= 1 && N <= (int64_t)1 << 31, "N=%lld outside 1..2^31", (long long)N);
  BMDCA_REQUIRE(sweeps >= 0, "sweeps=%d negative", sweeps);
  if (!std::isfinite(beta)) return fail(BMDCA_ENONFINITE, "beta is not finite");
  const int gather = pick_gather(flags, L, q);
  BMDCA_REQUIRE(gather >= 0, "sampler flags 0x%x not usable for L=%d q=%d", flags, L, q);
  BMDCA_REQUIRE(H_ws, "H_ws is NULL");
  BMDCA_REQUIRE(gather || !(flags & BMDCA_GIBBS_KEEP_LAYOUT),
                "BMDCA_GIBBS_KEEP_LAYOUT needs the gather form");
  if (gather) {
    if (H_ws_bytes < gather_ws_bytes(L, q))
      return fail(BMDCA_EWORKSPACE, "gibbs workspace %zu < %zu bytes", H_ws_bytes,
                  gather_ws_bytes(L, q));
    return hip_status(launch_gibbs_gather(h, J, chains, N, L, q, sweeps, seed, sweep_offset, beta,
                                          flips_out, nullptr, H_ws, s, ctl,
                                          (flags & BMDCA_SAMPLER_METROPOLIS) != 0),
                      "gibbs/gather");
  }
  if (H_ws_bytes < gibbs_bytes(N, L, q))
    return fail(BMDCA_EWORKSPACE, "gibbs workspace %zu < %zu bytes", H_ws_bytes,
                gibbs_bytes(N, L, q));
  if (!(flags & BMDCA_GIBBS_KEEP_FIELDS))
    BMDCA_TRY(hip_status(launch_local_fields(h, J, chains, N, L, q, H_ws, nullptr, s),
                         "gibbs/fields"));
  if (sweeps == 0) return BMDCA_OK;
  return hip_status(launch_gibbs_sweeps(J, chains, H_ws, N, L, q, sweeps, seed, sweep_offset, beta,
                                        flips_out, s, ctl, (flags & BMDCA_SAMPLER_METROPOLIS) != 0),
                    "gibbs/sweeps");
}

static_assert(sizeof(ChainStream) == sizeof(bmdca_chain_stream), "chain stream layout");
static_assert(offsetof(ChainStream, seed) == offsetof(bmdca_chain_stream, seed), "layout");
static_assert(offsetof(ChainStream, sweep_offset) == offsetof(bmdca_chain_stream, sweep_offset),
              "layout");
static_assert(offsetof(ChainStream, chain) == offsetof(bmdca_chain_stream, chain), "layout");

// Host-side validation shared by the single and grouped training calls.
int check_train(const bmdca_train_problem& p) {
  BMDCA_TRY(check_model(p.L, p.q));
  BMDCA_REQUIRE(p.h && p.J && p.chains && p.f1 && p.f2 && p.pearson && p.ws,
                "null pointer argument");
  BMDCA_REQUIRE(p.N >= 1 && p.N < ((int64_t)1 << 24), "N=%lld outside 1..2^24-1", (long long)p.N);
  BMDCA_REQUIRE(p.L >= 2, "train_step needs L >= 2 (got %d)", p.L);
  BMDCA_REQUIRE(p.sweeps >= 0, "sweeps=%d negative", p.sweeps);
  const int pr = p.prec & kPrecMask;
  BMDCA_REQUIRE(pr == BMDCA_PREC_FP32 || pr == BMDCA_PREC_BF16X2, "prec=%d unknown", pr);
  BMDCA_REQUIRE((p.prec & ~(kPrecMask | kSamplerMask | BMDCA_COUNTS_PRODUCT)) == 0,
                "prec flags 0x%x unknown", p.prec);
  BMDCA_REQUIRE(pick_gather(p.prec, p.L, p.q) >= 0, "sampler flags 0x%x not usable for L=%d q=%d",
                p.prec, p.L, p.q);
  if (!std::isfinite(p.lr)) return fail(BMDCA_ENONFINITE, "lr is not finite");
  const TrainPlan plan = plan_train(p.N, p.L, p.q, p.prec);
  if (p.ws_bytes < plan.total)
    return fail(BMDCA_EWORKSPACE, "train_step workspace %zu < %zu bytes", p.ws_bytes, plan.total);
  return BMDCA_OK;
}

// The kernel sequence of one epoch (arguments already validated).  `epoch`
// is used when ctl.epoch is null.
int enqueue_train(const bmdca_train_problem& p, uint64_t epoch, const DevCtl& ctl,
                  hipStream_t s) {
  const int N = (int)p.N, L = p.L, q = p.q;
  const int pr = p.prec & kPrecMask;
  const int gather = pick_gather(p.prec, L, q);
  const TrainPlan plan = plan_train(p.N, L, q, p.prec);
  char* base = static_cast<char*>(p.ws);
  float* H = reinterpret_cast<float*>(base + plan.off_H);
  void* sws = base + plan.off_stats;
  double* C = reinterpret_cast<double*>(base + plan.off_C);
  double* red = reinterpret_cast<double*>(base + plan.off_red);
  const int Lq = L * q;
  const uint64_t sweep0 = ctl.epoch ? 0 : epoch * (uint64_t)p.sweeps;
  if (gather) {
    BMDCA_TRY(hip_status(launch_gibbs_gather(p.h, p.J, p.chains, N, L, q, p.sweeps, p.seed, sweep0,
                                             1.0f, p.flips_out, p.dev_err, H, s, ctl,
                                             (p.prec & BMDCA_SAMPLER_METROPOLIS) != 0),
                         "train_step/gather"));
  } else {
    BMDCA_TRY(hip_status(launch_local_fields(p.h, p.J, p.chains, N, L, q, H, p.dev_err, s,
                                             ctl.active),
                         "train_step/fields"));
    if (p.sweeps > 0)
      BMDCA_TRY(hip_status(launch_gibbs_sweeps(p.J, p.chains, H, N, L, q, p.sweeps, p.seed, sweep0,
                                               1.0f, p.flips_out, s, ctl,
                                               (p.prec & BMDCA_SAMPLER_METROPOLIS) != 0),
                           "train_step/sweeps"));
  }
  if (p.prec & BMDCA_COUNTS_PRODUCT) {
    BMDCA_TRY(hip_status(launch_onehot_products(p.chains, nullptr, N, L, q, pr, plan.sp, sws,
                                                p.dev_err, s, ctl.active),
                         "train_step/counts"));
    BMDCA_TRY(hip_status(launch_reduce_partials(plan.sp, sws, Lq, C, s), "train_step/reduce"));
  } else {
    BMDCA_TRY(hip_status(launch_pair_counts(p.chains, N, L, q, plan.sp, sws, C, p.dev_err, s,
                                            ctl.active),
                         "train_step/counts"));
  }
  BMDCA_TRY(hip_status(launch_pearson(p.f1, p.f2, C, N, L, q, red, p.pearson, p.dev_err, s),
                       "train_step/pearson"));
  return hip_status(launch_update(p.h, p.J, p.f1, p.f2, C, N, L, q, p.lr, p.dev_err, s,
                                  ctl.active, p.mask),
                    "train_step/update");
}

// ----- grouped epochs: lane streams forked from and joined into the caller's
constexpr int kMaxLanes = 16;

struct LanePool {
  int device = -1;
  hipStream_t lanes[kMaxLanes] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kMaxLanes] = {};
  int created = 0;
};

std::mutex g_group_mu;
LanePool g_pools[64];  // per device ordinal

LanePool* pool_for_current() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  LanePool* lp = &g_pools[dev];
  lp->device = dev;
  return lp;
}

hipError_t ensure_lanes_locked(int lanes) {
  LanePool* lp = pool_for_current();
  if (!lp) return hipErrorInvalidDevice;
  if (!lp->fork) {
    hipError_t e = hipEventCreateWithFlags(&lp->fork, hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  while (lp->created < lanes) {
    const int k = lp->created;
    hipError_t e = hipStreamCreateWithFlags(&lp->lanes[k], hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipEventCreateWithFlags(&lp->join[k], hipEventDisableTiming);
    if (e != hipSuccess) return e;
    ++lp->created;
  }
  return hipSuccess;
}

hipError_t ensure_lanes(int lanes) {
  std::lock_guard<std::mutex> lock(g_group_mu);
  return ensure_lanes_locked(lanes);
}

// Relative cost of one model's epoch: site visits times the local-field
// work per visit, plus the count product.
double model_cost(const bmdca_train_problem& p) {
  const double Lq = (double)p.L * p.q;
  return (double)p.N * p.L * (p.sweeps > 0 ? p.sweeps : 1) * Lq + (double)p.N * Lq * Lq / 64.0;
}

int enqueue_group(const bmdca_train_problem* probs, int n, int lanes, hipStream_t s) {
  std::lock_guard<std::mutex> lock(g_group_mu);
  BMDCA_TRY(hip_status(ensure_lanes_locked(lanes), "group lanes"));
  LanePool* lp = pool_for_current();
  // Largest first, each to the least-loaded lane (ties: lowest lane).
  std::vector<int> order(n);
  for (int k = 0; k < n; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return model_cost(probs[a]) > model_cost(probs[b]);
  });
  std::vector<double> load(lanes, 0.0);
  std::vector<int> lane_of(n, 0);
  for (int k : order) {
    int best = 0;
    for (int l = 1; l < lanes; ++l)
      if (load[l] < load[best]) best = l;
    lane_of[k] = best;
    load[best] += model_cost(probs[k]);
  }
  // CU share of each model's sampler grid: the lane's share of the chip.
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int share = std::max(1, cus / lanes);
  BMDCA_TRY(hip_status(hipEventRecord(lp->fork, s), "group fork"));
  for (int l = 0; l < lanes; ++l)
    BMDCA_TRY(hip_status(hipStreamWaitEvent(lp->lanes[l], lp->fork, 0), "group fork"));
  for (int k : order) {
    const bmdca_train_problem& p = probs[k];
    hipStream_t ls = lp->lanes[lane_of[k]];
    DevCtl ctl;
    auto* rec = reinterpret_cast<char*>(p.ctl);
    ctl.epoch = reinterpret_cast<const uint64_t*>(rec + offsetof(bmdca_train_ctl, epoch));
    ctl.active = reinterpret_cast<const int32_t*>(rec + offsetof(bmdca_train_ctl, active));
    ctl.cu_share = lanes > 1 ? share : 0;
    BMDCA_TRY(enqueue_train(p, 0, ctl, ls));
    BMDCA_TRY(hip_status(launch_ctl_advance(p.ctl, p.pearson, ls), "group ctl"));
  }
  for (int l = 0; l < lanes; ++l) {
    BMDCA_TRY(hip_status(hipEventRecord(lp->join[l], lp->lanes[l]), "group join"));
    BMDCA_TRY(hip_status(hipStreamWaitEvent(s, lp->join[l], 0), "group join"));
  }
  return BMDCA_OK;
}

// Decimation workspace: chain-count planes, the count matrix, select state.
struct DecimatePlan {
  StatsPlan sp;
  size_t off_stats, off_C, off_dec, total;
};

DecimatePlan plan_decimate(int64_t N, int L, int q) {
  DecimatePlan d{};
  const size_t Lq = (size_t)L * q;
  d.sp = plan_stats(N, L, q, BMDCA_PREC_BF16X2);
  size_t o = 0;
  d.off_stats = o; o = align256(o + d.sp.total);
  d.off_C = o;     o = align256(o + sizeof(double) * Lq * Lq);
  d.off_dec = o;   o = align256(o + dec_ws_bytes(L, q));
  d.total = o;
  return d;
}

}  // namespace

// ----- Allocation-free energies: the scratch of bmdca_energy_noalloc lives in
// a file-scope device array (each GPU holds its own copy from module load to
// process end).  Host code never passes the array's name to a kernel: its
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kEnergyScratchBytes = (size_t)BMDCA_ENERGY_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kEnergyScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call there).
static int scratch_address(void** out) {
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e, "energy_noalloc: current device");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(BMDCA_EINVAL, "energy_noalloc: device %d outside 0..%d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t g = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (g != hipSuccess) return hip_status(g, "energy_noalloc: scratch address");
    if (!p) return fail(BMDCA_EHIP, "energy_noalloc: scratch address is NULL");
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return BMDCA_OK;
}

struct bmdca_graph_s {
  hipGraphExec_t exec = nullptr;
};

extern "C" {

const char* bmdca_last_error(void) { return g_err.c_str(); }

int32_t bmdca_identity_threshold(double theta, int32_t L) {
  return (int32_t)std::ceil(theta * (double)L - 1e-6);
}

size_t bmdca_workspace_bytes(int32_t kind, int64_t MN, int32_t L, int32_t q, int32_t prec) {
  if (L < 1 || L > kMaxL || q < 2 || q > kMaxQ) return 0;
  switch (kind) {
    case BMDCA_WS_REWEIGHT:
      if (MN < 1 || L > 512) return 0;
      return plan_reweight(MN, L, q).total;
    case BMDCA_WS_STATS:
      if (MN < 1) return 0;
      return plan_stats(MN, L, q, prec).total;
    case BMDCA_WS_GIBBS:
      if (MN < 1 || pick_gather(prec, L, q) < 0) return 0;
      return field_bytes(MN, L, q, prec);
    case BMDCA_WS_TRAIN_STEP:
      if (MN < 1 || pick_gather(prec, L, q) < 0) return 0;
      return plan_train(MN, L, q, prec).total;
    case BMDCA_WS_APC:
      return apc_ws_bytes(L);
    case BMDCA_WS_MUTANT:
      if (MN < 1) return 0;
      return gibbs_bytes(MN, L, q);
    case BMDCA_WS_ENERGY:
      if (MN < 0) return 0;
      return plan_energy(MN, L, q).total;
    case BMDCA_WS_DRAW:
      if (MN < 1) return 0;
      return draw_ws_bytes(MN);
    case BMDCA_WS_SEQID:
      return seqid_ws_bytes();
    case BMDCA_WS_DECIMATE:
      if (MN < 1) return 0;
      return plan_decimate(MN, L, q).total;
    default:
      return 0;
  }
}

int bmdca_init_chains(int8_t* chains, int64_t N, int32_t L, int32_t q, uint64_t seed,
                      void* stream) {
  BMDCA_TRY(check_model(L, q));
  BMDCA_REQUIRE(chains, "chains is NULL");
  BMDCA_REQUIRE(N >= 1 && N <= (int64_t)1 << 31, "N=%lld outside 1..2^31", (long long)N);
  return hip_status(launch_init_chains(chains, N, L, q, seed, (hipStream_t)stream), "init_chains");
}

int bmdca_reweight(const int8_t* msa, int64_t M, int32_t L, int32_t q, double theta,
                   int32_t* n_sim, double* w, double* meff, void* ws, size_t ws_bytes,
                   int32_t* dev_err, void* stream) {
  BMDCA_TRY(check_model(L, q));
  BMDCA_REQUIRE(L <= 512, "reweight supports L <= 512 (got %d)", L);
  BMDCA_REQUIRE(msa && n_sim && w && meff && ws, "null pointer argument");
  BMDCA_REQUIRE(M >= 1 && M <= (int64_t)1 << 31, "M=%lld outside 1..2^31", (long long)M);
  BMDCA_REQUIRE(theta >= 0.0 && theta <= 1.0, "theta=%g outside [0,1]", theta);
  const ReweightPlan plan = plan_reweight(M, L, q);
  if (ws_bytes < plan.total)
    return fail(BMDCA_EWORKSPACE, "reweight workspace %zu < %zu bytes", ws_bytes, plan.total);
  const int32_t T = bmdca_identity_threshold(theta, L);
  return hip_status(launch_reweight(msa, M, L, q, T, plan, ws, n_sim, w, meff, dev_err,
                                    (hipStream_t)stream),
                    "reweight");
}

int bmdca_stats(const int8_t* X, const double* w, int64_t M, int32_t L, int32_t q,
                double pseudocount, int32_t prec, double* f1, double* f2, double* meff_out,
                void* ws, size_t ws_bytes, int32_t* dev_err, void* stream) {
  BMDCA_TRY(check_model(L, q));
  BMDCA_REQUIRE(X && f1 && f2 && meff_out && ws, "null pointer argument");
  BMDCA_REQUIRE(M >= 1 && M < ((int64_t)1 << 24), "M=%lld outside 1..2^24-1", (long long)M);
  BMDCA_REQUIRE(prec == BMDCA_PREC_FP32 || prec == BMDCA_PREC_BF16X2, "prec=%d unknown", prec);
  BMDCA_REQUIRE(std::isfinite(pseudocount) && pseudocount <= 1.0, "pseudocount=%g invalid",
                pseudocount);
  const StatsPlan plan = plan_stats(M, L, q, prec);
  if (ws_bytes < plan.total)
    return fail(BMDCA_EWORKSPACE, "stats workspace %zu < %zu bytes", ws_bytes, plan.total);
  hipStream_t s = (hipStream_t)stream;
  BMDCA_TRY(hip_status(launch_meff(w, M, meff_out, s), "stats/meff"));
  BMDCA_TRY(hip_status(launch_onehot_products(X, w, M, L, q, prec, plan, ws, dev_err, s),
                       "stats/product"));
  return hip_status(launch_stats_epilogue(plan, ws, L, q, meff_out, pseudocount, f1, f2, s),
                    "stats/epilogue");
}

int bmdca_gibbs(const float* h, const float* J, int8_t* chains, int64_t N, int32_t L, int32_t q,
                int32_t sweeps, uint64_t seed, uint64_t sweep_offset, float beta, float* H_ws,
                size_t H_ws_bytes, int32_t flags, unsigned long long* flips_out,
                void* stream) {
  return gibbs_impl(h, J, chains, N, L, q, sweeps, seed, sweep_offset, beta, H_ws, H_ws_bytes,
                    flags, flips_out, DevCtl(), (hipStream_t)stream);
}

int bmdca_gibbs_streams(const float* h, const float* J, int8_t* chains, int64_t N, int32_t L,
                        int32_t q, int32_t sweeps, const bmdca_chain_stream* streams, float beta,
                        float* H_ws, size_t H_ws_bytes, int32_t flags, int32_t cus,
                        unsigned long long* flips_out, void* stream) {
  BMDCA_REQUIRE(streams, "streams is NULL");
  BMDCA_REQUIRE(cus >= 0, "cus=%d negative", cus);
  DevCtl ctl;
  ctl.streams = reinterpret_cast<const ChainStream*>(streams);
  ctl.cu_share = cus;
  return gibbs_impl(h, J, chains, N, L, q, sweeps, 0, 0, beta, H_ws, H_ws_bytes, flags, flips_out,
                    ctl, (hipStream_t)stream);
}

int bmdca_energy(const float* h, const float* J, const int8_t* seqs, int64_t B, int32_t L,
                 int32_t q, float* E, void* ws, size_t ws_bytes, int32_t* dev_err, void* stream) {
  BMDCA_TRY(check_model(L, q));
  BMDCA_REQUIRE(B >= 0 && B <= (int64_t)1 << 31, "B=%lld outside 0..2^31", (long long)B);
  if (B == 0) return BMDCA_OK;  // nothing to score; seqs, E and ws may be NULL
  BMDCA_REQUIRE(h && J && seqs && E && ws, "null pointer argument");
  const EnergyPlan plan = plan_energy(B, L, q);
  if (ws_bytes < plan.total)
    return fail(BMDCA_EWORKSPACE, "energy workspace %zu < %zu bytes", ws_bytes, plan.total);
  return hip_status(launch_energy(h, J, seqs, B, L, q, E, plan, ws, dev_err, (hipStream_t)stream),
                    "energy");
}

int bmdca_energy_noalloc(const float* h, const float* J, const int8_t* seqs, int64_t B,
                         int32_t L, int32_t q, float* E, int32_t* dev_err, void* stream) {
  BMDCA_TRY(check_model(L, q));
  BMDCA_REQUIRE(B >= 0 && B <= (int64_t)1 << 31, "B=%lld outside 0..2^31", (long long)B);
  if (B == 0) return BMDCA_OK;  // nothing to score; seqs and E may be NULL
  BMDCA_REQUIRE(h && J && seqs && E, "null pointer argument");
  const EnergyPlan plan = plan_energy(B, L, q);
  if (plan.total > kEnergyScratchBytes)
    return fail(BMDCA_EINVAL,
                "energy_noalloc: B=%lld at L=%d needs %zu bytes of scratch, more than the "
                "%zu-byte static array; split the batch or use bmdca_energy",
                (long long)B, L, plan.total, kEnergyScratchBytes);
  void* ws = nullptr;
  BMDCA_TRY(scratch_address(&ws));
  return hip_status(launch_energy(h, J, seqs, B, L, q, E, plan, ws, dev_err, (hipStream_t)stream),
                    "energy_noalloc");
}

int bmdca_energy_batch(const float* h, const float* J, const int8_t* seqs, int64_t cap,
                       const int64_t* n_live, int32_t L, int32_t q, float* E, void* ws,
                       size_t ws_bytes, int32_t* dev_err, void* stream) {
  BMDCA_TRY(check_model(L, q));
  BMDCA_REQUIRE(cap >= 1 && cap <= (int64_t)1 << 31, "cap=%lld outside 1..2^31", (long long)cap);
  BMDCA_REQUIRE(h && J && seqs && E && ws && n_live, "null pointer argument");
  const EnergyPlan plan = plan_energy(cap, L, q);
  if (ws_bytes < plan.total)
    return fail(BMDCA_EWORKSPACE, "energy workspace %zu < %zu bytes", ws_bytes, plan.total);
  return hip_status(launch_energy(h, J, seqs, cap, L, q, E, plan, ws, dev_err,
                                  (hipStream_t)stream, n_live),
                    "energy_batch");
}

int bmdca_mutant_scan_batch(const float* h, const float* J, const int8_t* wt, int64_t cap,
                            const int64_t* n_live, int32_t L, int32_t q, float* dE, void* ws,
                            size_t ws_bytes, void* stream) {
  BMDCA_TRY(check_model(L, q));
  BMDCA_REQUIRE(cap >= 1 && cap <= (int64_t)1 << 31, "cap=%lld outside 1..2^31", (long long)cap);
  BMDCA_REQUIRE(h && J && wt && dE && ws && n_live, "null pointer argument");
  if (ws_bytes < gibbs_bytes(cap, L, q))
    return fail(BMDCA_EWORKSPACE, "mutant workspace %zu < %zu bytes", ws_bytes,
                gibbs_bytes(cap, L, q));
  hipStream_t s = (hipStream_t)stream;
  float* H = static_cast<float*>(ws);
  BMDCA_TRY(hip_status(launch_local_fields(h, J, wt, cap, L, q, H, nullptr, s, nullptr, n_live),
                       "mutant_batch/fields"));
  return hip_status(launch_mutant_delta(H, wt, cap, L, q, dE, s, n_live), "mutant_batch/delta");
}

int bmdca_sample_tick(const float* h, const float* J, int8_t* chains, int64_t cap,
                      const int64_t* n_live, int32_t L, int32_t q, int32_t sweeps,
                      const bmdca_chain_stream* streams, uint64_t* tick, float beta,
                      float* ws, size_t ws_bytes, int32_t flags, int32_t cus, void* stream) {
  BMDCA_TRY(check_model(L, q));
  BMDCA_REQUIRE(streams && tick && n_live, "null pointer argument");
  BMDCA_REQUIRE(cus >= 0, "cus=%d negative", cus);
  BMDCA_REQUIRE(gather_supported(L, q), "sample_tick needs the gather form (L=%d q=%d)", L, q);
  BMDCA_REQUIRE((flags & ~(BMDCA_GIBBS_KEEP_LAYOUT | BMDCA_SAMPLER_METROPOLIS |
                           BMDCA_SAMPLER_GATHER)) == 0,
                "sample_tick flags 0x%x: only KEEP_LAYOUT, METROPOLIS, GATHER", flags);
  DevCtl ctl;
  ctl.streams = reinterpret_cast<const ChainStream*>(streams);
  ctl.cu_share = cus;
  ctl.epoch = tick;
  ctl.count = n_live;
  hipStream_t s = (hipStream_t)stream;
  BMDCA_TRY(gibbs_impl(h, J, chains, cap, L, q, sweeps, 0, 0, beta, ws, ws_bytes,
                       flags | BMDCA_SAMPLER_GATHER, nullptr, ctl, s));
  return hip_status(launch_tick_advance(tick, s), "sample_tick/advance");
}

int bmdca_draw_rows(const double* w, int64_t M, int64_t n, uint64_t seed, int32_t* rows,
                    void* ws, size_t ws_bytes, int32_t* dev_err, void* stream) {
  BMDCA_REQUIRE(M >= 1 && M < ((int64_t)1 << 31), "M=%lld outside 1..2^31-1", (long long)M);
  BMDCA_REQUIRE(n >= 0 && n < ((int64_t)1 << 34), "n=%lld outside 0..2^34-1", (long long)n);
  BMDCA_REQUIRE(w && ws && (rows || n == 0), "null pointer argument");
  if (ws_bytes < draw_ws_bytes(M))
    return fail(BMDCA_EWORKSPACE, "draw workspace %zu < %zu bytes", ws_bytes, draw_ws_bytes(M));
  return hip_status(launch_draw_rows(w, M, n, seed, rows, ws, dev_err, (hipStream_t)stream),
                    "draw_rows");
}

int bmdca_gather_rows(const int8_t* X, int64_t M, int32_t L, const int32_t* rows, int64_t n,
                      int8_t* out, int32_t* dev_err, void* stream) {
  BMDCA_REQUIRE(M >= 1 && L >= 1 && L <= kMaxL, "M=%lld, L=%d invalid", (long long)M, L);
  BMDCA_REQUIRE(n >= 0 && n * (int64_t)L < ((int64_t)1 << 40), "n=%lld invalid", (long long)n);
  if (n == 0) return BMDCA_OK;
  BMDCA_REQUIRE(X && rows && out, "null pointer argument");
  return hip_status(launch_gather_rows(X, M, L, rows, n, out, dev_err, (hipStream_t)stream),
                    "gather_rows");
}

int bmdca_seqid(const int8_t* A, const int8_t* B, const int32_t* perm, int64_t N, int32_t L,
                double* out, void* ws, size_t ws_bytes, int32_t* dev_err, void* stream) {
  BMDCA_REQUIRE(N >= 1 && N < ((int64_t)1 << 31), "N=%lld outside 1..2^31-1", (long long)N);
  BMDCA_REQUIRE(L >= 1 && L <= kMaxL, "L=%d outside 1..%d", L, kMaxL);
  BMDCA_REQUIRE(A && B && out && ws, "null pointer argument");
  if (ws_bytes < seqid_ws_bytes())
    return fail(BMDCA_EWORKSPACE, "seqid workspace %zu < %zu bytes", ws_bytes, seqid_ws_bytes());
  return hip_status(launch_seqid(A, B, perm, N, L, out, ws, dev_err, (hipStream_t)stream),
                    "seqid");
}

int bmdca_train_step(float* h, float* J, int8_t* chains, int64_t N, int32_t L, int32_t q,
                     const double* f1, const double* f2, double lr, int32_t sweeps, uint64_t seed,
                     uint64_t epoch, int32_t prec, double* pearson, unsigned long long* flips_out,
                     void* ws, size_t ws_bytes, int32_t* dev_err, void* stream) {
  bmdca_train_problem p{};
  p.h = h;
  p.J = J;
  p.chains = chains;
  p.f1 = f1;
  p.f2 = f2;
  p.pearson = pearson;
  p.flips_out = flips_out;
  p.dev_err = dev_err;
  p.ws = ws;
  p.ws_bytes = ws_bytes;
  p.N = N;
  p.L = L;
  p.q = q;
  p.lr = lr;
  p.seed = seed;
  p.sweeps = sweeps;
  p.prec = prec;
  BMDCA_TRY(check_train(p));
  return enqueue_train(p, epoch, DevCtl(), (hipStream_t)stream);
}

int bmdca_train_step_masked(float* h, float* J, const uint8_t* mask, int8_t* chains, int64_t N,
                            int32_t L, int32_t q, const double* f1, const double* f2, double lr,
                            int32_t sweeps, uint64_t seed, uint64_t epoch, int32_t prec,
                            double* pearson, unsigned long long* flips_out, void* ws,
                            size_t ws_bytes, int32_t* dev_err, void* stream) {
  BMDCA_REQUIRE(mask, "mask is NULL");
  bmdca_train_problem p{};
  p.h = h;
  p.J = J;
  p.chains = chains;
  p.f1 = f1;
  p.f2 = f2;
  p.pearson = pearson;
  p.flips_out = flips_out;
  p.dev_err = dev_err;
  p.ws = ws;
  p.ws_bytes = ws_bytes;
  p.N = N;
  p.L = L;
  p.q = q;
  p.lr = lr;
  p.seed = seed;
  p.sweeps = sweeps;
  p.prec = prec;
  p.mask = mask;
  BMDCA_TRY(check_train(p));
  return enqueue_train(p, epoch, DevCtl(), (hipStream_t)stream);
}

int bmdca_decimate(float* J, uint8_t* mask, const int8_t* chains, int64_t N, int32_t L, int32_t q,
                   double drate, double density, long long* n_active, void* ws, size_t ws_bytes,
                   int32_t* dev_err, void* stream) {
  BMDCA_TRY(check_model(L, q));
  BMDCA_REQUIRE(L >= 2, "decimation needs L >= 2 (got %d)", L);
  BMDCA_REQUIRE(J && mask && chains && ws, "null pointer argument");
  BMDCA_REQUIRE(N >= 1 && N < ((int64_t)1 << 24), "N=%lld outside 1..2^24-1", (long long)N);
  BMDCA_REQUIRE(drate >= 0.0 && drate <= 1.0, "drate=%g outside [0, 1]", drate);
  BMDCA_REQUIRE(density >= 0.0 && density <= 1.0, "density=%g outside [0, 1]", density);
  const DecimatePlan plan = plan_decimate(N, L, q);
  if (ws_bytes < plan.total)
    return fail(BMDCA_EWORKSPACE, "decimate workspace %zu < %zu bytes", ws_bytes, plan.total);
  hipStream_t s = (hipStream_t)stream;
  char* base = static_cast<char*>(ws);
  void* sws = base + plan.off_stats;
  double* C = reinterpret_cast<double*>(base + plan.off_C);
  BMDCA_TRY(hip_status(launch_pair_counts(chains, N, L, q, plan.sp, sws, C, dev_err, s),
                       "decimate/counts"));
  return hip_status(launch_decimate(J, mask, C, N, L, q, drate, density, n_active,
                                    base + plan.off_dec, s),
                    "decimate/select");
}

int bmdca_activate(uint8_t* mask, const int8_t* chains, int64_t N, int32_t L, int32_t q,
                   const double* f2, double factivate, long long* n_active, void* ws,
                   size_t ws_bytes, int32_t* dev_err, void* stream) {
  BMDCA_TRY(check_model(L, q));
  BMDCA_REQUIRE(L >= 2, "activation needs L >= 2 (got %d)", L);
  BMDCA_REQUIRE(mask && chains && f2 && ws, "null pointer argument");
  BMDCA_REQUIRE(N >= 1 && N < ((int64_t)1 << 24), "N=%lld outside 1..2^24-1", (long long)N);
  BMDCA_REQUIRE(factivate >= 0.0 && factivate <= 1.0, "factivate=%g outside [0, 1]", factivate);
  const DecimatePlan plan = plan_decimate(N, L, q);
  if (ws_bytes < plan.total)
    return fail(BMDCA_EWORKSPACE, "activate workspace %zu < %zu bytes", ws_bytes, plan.total);
  hipStream_t s = (hipStream_t)stream;
  char* base = static_cast<char*>(ws);
  void* sws = base + plan.off_stats;
  double* C = reinterpret_cast<double*>(base + plan.off_C);
  BMDCA_TRY(hip_status(launch_pair_counts(chains, N, L, q, plan.sp, sws, C, dev_err, s),
                       "activate/counts"));
  return hip_status(launch_activate(mask, C, f2, N, L, q, factivate, n_active,
                                    base + plan.off_dec, dev_err, s),
                    "activate/select");
}

int bmdca_profile_fields(const double* f1, int32_t L, int32_t q, float* h, int32_t* dev_err,
                         void* stream) {
  BMDCA_TRY(check_model(L, q));
  BMDCA_REQUIRE(f1 && h, "null pointer argument");
  return hip_status(launch_profile_fields(f1, L, q, h, dev_err, (hipStream_t)stream),
                    "profile_fields");
}

int bmdca_mask_init(uint8_t* mask, int32_t L, int32_t q, int32_t full, void* stream) {
  BMDCA_TRY(check_model(L, q));
  BMDCA_REQUIRE(mask, "null pointer argument");
  return hip_status(launch_mask_init(mask, L, q, full != 0, (hipStream_t)stream), "mask_init");
}

int bmdca_mask_apply(float* J, const uint8_t* mask, int32_t L, int32_t q, long long* n_active,
                     void* stream) {
  BMDCA_TRY(check_model(L, q));
  BMDCA_REQUIRE(mask, "null pointer argument");
  return hip_status(launch_mask_apply(J, mask, L, q, n_active, (hipStream_t)stream),
                    "mask_apply");
}

int bmdca_train_group_step(const bmdca_train_problem* probs, int32_t n, int32_t lanes,
                           void* stream) {
  BMDCA_REQUIRE(probs && n >= 1, "group needs at least one problem");
  BMDCA_REQUIRE(lanes >= 1 && lanes <= kMaxLanes, "lanes=%d outside 1..%d", lanes, kMaxLanes);
  for (int32_t k = 0; k < n; ++k) {
    const int rc = check_train(probs[k]);
    if (rc != BMDCA_OK) return fail(rc, "problem %d: %s", k, g_err.c_str());
    if (!probs[k].ctl) return fail(BMDCA_EINVAL, "problem %d: ctl is required", k);
  }
  return enqueue_group(probs, n, lanes, (hipStream_t)stream);
}

int bmdca_train_group_graph(const bmdca_train_problem* probs, int32_t n, int32_t lanes,
                            void* stream, bmdca_graph* out) {
  BMDCA_REQUIRE(out, "null pointer argument");
  *out = nullptr;
  BMDCA_REQUIRE(probs && n >= 1, "group needs at least one problem");
  BMDCA_REQUIRE(lanes >= 1 && lanes <= kMaxLanes, "lanes=%d outside 1..%d", lanes, kMaxLanes);
  for (int32_t k = 0; k < n; ++k) {
    const int rc = check_train(probs[k]);
    if (rc != BMDCA_OK) return fail(rc, "problem %d: %s", k, g_err.c_str());
    if (!probs[k].ctl) return fail(BMDCA_EINVAL, "problem %d: ctl is required", k);
  }
  BMDCA_REQUIRE(stream, "graph capture needs a created stream (not NULL)");
  hipStream_t s = (hipStream_t)stream;
  // Lanes are created before capture begins.
  BMDCA_TRY(hip_status(ensure_lanes(lanes), "group lanes"));
  BMDCA_TRY(hip_status(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture"));
  const int rc = enqueue_group(probs, n, lanes, s);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(s, &graph);
  if (rc != BMDCA_OK) {
    if (graph) hipGraphDestroy(graph);
    return rc;
  }
  BMDCA_TRY(hip_status(ec, "end capture"));
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  BMDCA_TRY(hip_status(ei, "graph instantiate"));
  auto* g = new (std::nothrow) bmdca_graph_s;
  if (!g) {
    hipGraphExecDestroy(exec);
    return fail(BMDCA_EINVAL, "out of host memory");
  }
  g->exec = exec;
  *out = g;
  return BMDCA_OK;
}

int bmdca_graph_launch(bmdca_graph g, void* stream) {
  BMDCA_REQUIRE(g && g->exec, "null graph");
  return hip_status(hipGraphLaunch(g->exec, (hipStream_t)stream), "graph launch");
}

int bmdca_graph_destroy(bmdca_graph g) {
  if (!g) return BMDCA_OK;
  const hipError_t e = g->exec ? hipGraphExecDestroy(g->exec) : hipSuccess;
  delete g;
  return hip_status(e, "graph destroy");
}

int bmdca_single_mutant_scan(const float* h, const float* J, const int8_t* wt, int64_t B,
                             int32_t L, int32_t q, float* dE, void* ws, size_t ws_bytes,
                             void* stream) {
  BMDCA_TRY(check_model(L, q));
  BMDCA_REQUIRE(h && J && wt && dE && ws, "null pointer argument");
  BMDCA_REQUIRE(B >= 1 && B <= (int64_t)1 << 31, "B=%lld outside 1..2^31", (long long)B);
  if (ws_bytes < gibbs_bytes(B, L, q))
    return fail(BMDCA_EWORKSPACE, "mutant workspace %zu < %zu bytes", ws_bytes,
                gibbs_bytes(B, L, q));
  hipStream_t s = (hipStream_t)stream;
  float* H = static_cast<float*>(ws);
  BMDCA_TRY(hip_status(launch_local_fields(h, J, wt, B, L, q, H, nullptr, s), "mutant/fields"));
  return hip_status(launch_mutant_delta(H, wt, B, L, q, dE, s), "mutant/delta");
}

int bmdca_apc_frobenius(const float* J, int32_t L, int32_t q, int32_t gap, float* F,
                        float* F_apc, void* ws, size_t ws_bytes, void* stream) {
  BMDCA_TRY(check_model(L, q));
  BMDCA_REQUIRE(L >= 2, "apc_frobenius needs L >= 2 (got %d)", L);
  BMDCA_REQUIRE(J && F_apc && ws, "null pointer argument");
  BMDCA_REQUIRE(gap >= -1 && gap < q, "gap=%d outside -1..q-1", gap);
  if (ws_bytes < apc_ws_bytes(L))
    return fail(BMDCA_EWORKSPACE, "apc workspace %zu < %zu bytes", ws_bytes, apc_ws_bytes(L));
  return hip_status(launch_apc(J, L, q, gap, F, F_apc, ws, (hipStream_t)stream), "apc_frobenius");
}

}  // extern "C"
