"""Benchmark of the bmDCA training hot path on one MI355X.

Default workload (the precision form): L = 256 sites, q = 21 states, an
alignment of M = 100 000 synthetic sequences (phylogeny-like, seeded) with
non-uniform weights w = 1 - U[0, 1) in (0, 1], N = 20 000 persistent chains,
10 Gibbs sweeps per epoch, lr 0.05.  One step = one training epoch through
bmdca_train_step (sweeps in the gather form, chain counts on the matrix
cores, FP64 Pearson check and FP64 update), timed in the plain FP32 form
(`value`); beside it the mixed (BF16 hi+lo) epoch, the weighted two-site
statistics in both forms with their maximum error against the FP64 oracle on
sampled entries, the sweep kernels alone, and the protein-scale workload
(L = 100, N = 10 000) as context.  Inputs are synthetic and resident in HBM
before the timed region.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gibbs site-updates/s + epoch time, BF16 vs FP32 at ≤1e-5 stat err; p99 latency"
HBM_PEAK_GBS = 8000.0
# LDS read peak per CU and clock on gfx950: 256 bytes (twice the previous
# generation's 128; a 64-lane read of contiguous 16-byte quads, 16 waves per
# CU, sustains 213 B/clk on MI355X)
LDS_BYTES_PER_CLK = 256

# HBM bytes per 10-sweep launch of the gather sweep kernel: rocprofv3
# FETCH_SIZE and WRITE_SIZE of that launch (KiB per dispatch), each scaled by
# what the same counter reads for a 512 MiB device copy in the same run.
# Valid only for the sources they were taken with (the SHA-256 of the files
# below); for other sources the line reports null.
GATHER_TRAFFIC_SOURCES = ("paper_2501_18456_amd/csrc/gather_kernel.hpp",
                          "paper_2501_18456_amd/csrc/gather_plan.hpp",
                          "paper_2501_18456_amd/csrc/sampler.hip",
                          "paper_2501_18456_amd/csrc/sampler_w12.hip",
                          "paper_2501_18456_amd/csrc/common.hpp")
# workload -> bytes per launch: the gather kernel's 10-sweep launch and the
# field kernel's 5-sweep launch of the precision form (L = 256, N = 20 000)
GATHER_TRAFFIC = {"sha256": "6e43891342b19d2558b6b03d0016c4c6009e47f97f3cd79fd6103f12122d2941",
                  "bytes": {"precision": 1.05827e10,           # 1.05775e10 read + 5.18e6 written
                            "precision-fields": 1.98177e+12}}  # 1.45992e+12 read + 5.2185e+11


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in GATHER_TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def gather_traffic(workload):
    """The profiled HBM bytes per launch if the kernel sources are unchanged."""
    if GATHER_TRAFFIC["sha256"] != sources_digest():
        return None
    return GATHER_TRAFFIC["bytes"].get(workload)


def cpu_info():
    """Host cores this process may use, nproc and the CPU model name."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", usable) or usable)
    return {"nproc": os.cpu_count(), "usable": usable, "omp_threads": min(threads, usable),
            "model": model}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gather_lds_bytes(N, L, q, sweeps, cus, row_bytes=None):
    """LDS traffic of a gather-form sweep launch: every visit reads row_bytes
    of each of L-1 coupling rows (the q-vector, 4q bytes, for the heat-bath
    draw; the two entries of a and a', 8 bytes, for Metropolis); every
    workgroup stages site i's L-1 blocks of q x q once per visit of site i
    (workgroups as the library sizes them: chains spread over the CUs in as
    few rounds as workgroups of at most 128 chains allow; at L = 100 the
    tokens never limit that size)."""
    rounds = -(-N // (cus * 128))
    cpb = min(128, -(-N // (rounds * cus)))
    nwg = -(-N // cpb)
    rb = 4 * q if row_bytes is None else row_bytes
    return N * L * sweeps * (L - 1) * rb + nwg * sweeps * L * (L - 1) * q * q * 4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "bf16x2"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (counter calibration)")
    ap.add_argument("--cpu-chains", type=int, default=1000,
                    help="chains in the oracle's timed sample epoch")
    ap.add_argument("--no-oracle-errors", action="store_true",
                    help="precision: skip the FP64 oracle entries of the statistics errors")
    ap.add_argument("--no-protein", action="store_true",
                    help="precision: skip the protein-scale context figures")
    ap.add_argument("--workload", default="precision",
                    choices=["protein", "small", "precision", "scoring", "group", "serve", "next"],
                    help="precision (default): training epochs at L=256, M=1e5 weighted rows, "
                         "N=2e4 chains, FP32 form timed, BF16 hi+lo beside it, statistics "
                         "errors vs the FP64 oracle; protein: one model at protein scale; "
                         "small: the whole "
                         "plain-bmDCA run at CPU-seconds size (L=20) on the GPU and in the "
                         "oracle; scoring: "
                         "reweighting at M=1e5 and energies, mutant scans, contact scores of an "
                         "L=512 model; group: 64 "
                         "uneven models trained together in one captured graph per epoch; "
                         "serve: request loop over 8 resident models at three arrival rates; "
                         "next: equilibrium sampling with the mixing time, Metropolis sweeps, "
                         "element decimation and activation at protein scale")
    ap.add_argument("--lanes", type=int, default=8, help="group/serve: concurrent lane streams")
    ap.add_argument("--serve-requests", type=int, default=2000, help="serve: requests per rate")
    ap.add_argument("--serve-budget-gib", type=float, default=32.0,
                    help="serve: HBM budget for requests in flight")
    ap.add_argument("--serve-chunk", type=int, default=1,
                    help="serve: sweeps per sampling tick (the batching boundary)")
    ap.add_argument("--serve-cus", type=int, default=64,
                    help="serve: compute units a sampling tick is sized for (0: all)")
    return ap.parse_args()


class Timer:
    """HIP events on the current stream (the stream the library launches on)."""

    def __init__(self):
        import torch
        self.a = torch.cuda.Event(enable_timing=True)
        self.b = torch.cuda.Event(enable_timing=True)

    def start(self):
        self.a.record()

    def stop_ms(self):
        import torch
        self.b.record()
        self.b.synchronize()
        return self.a.elapsed_time(self.b)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 (the "
                                   "library has no multi-GPU path)"}))
        sys.exit(2)
    fn = {"precision": bench_precision_epoch, "protein": bench_protein, "small": bench_small,
          "next": bench_next, "scoring": bench_scoring, "group": bench_group,
          "serve": bench_serve}[args.workload]
    return fn(args)


def bench_protein(args, emit=True):
    """Protein scale: L = 100, q = 21, N = 10 000 chains, planted sparse-contact
    model (3L random pairs with N(0, 0.5) blocks, gap holding 15% of the
    independent-site mass), M = 20 000 sequences drawn from it by 200 Gibbs
    sweeps and reweighted at 80% identity, FP32 statistics.  One step = one
    epoch.  With emit=False returns the line's dict (the default workload
    reports it as context)."""
    import numpy as np
    import torch

    from paper_2501_18456_amd import api, synth
    from paper_2501_18456_amd import _lib as B

    torch.cuda.set_device(0)
    if emit:
        calibration_copy(args)
    L, q, N, M, sweeps, lr = 100, 21, 10000, 20000, 10, 0.05
    Lq = L * q
    seed_model, seed_msa, seed_chain = 1002, 2002, 3002
    log(f"workload L={L} q={q} N={N} M={M} sweeps={sweeps} prec={args.prec}")

    # ---------------- synthetic inputs (not timed)
    h_true, J_true = synth.planted_sparse(L, q, seed=seed_model, sigma_J=0.5, gap_mass=0.15)
    ht = torch.from_numpy(h_true).cuda()
    Jt = torch.from_numpy(J_true).cuda()
    msa = api.init_chains(M, L, q, seed=seed_msa)
    api.gibbs(ht, Jt, msa, sweeps=200, seed=seed_msa)
    torch.cuda.synchronize()
    log("alignment drawn (200 sweeps of the planted model)")
    t = Timer()
    t.start()
    _, w, meff = api.reweight(msa, q, 0.8)
    rw_ms = t.stop_ms()
    t.start()
    f1, f2, _ = api.stats(msa, q, w, -1.0, args.prec)
    st_ms = t.stop_ms()
    log(f"reweight {rw_ms:.2f} ms, M_eff={float(meff.cpu()[0]):.1f}; stats {st_ms:.2f} ms")

    # initial model: independent-site fields log f_i(a), no couplings
    h = api.profile_fields(f1, L, q)
    J = torch.zeros((Lq, Lq), dtype=torch.float32, device="cuda")
    chains = api.init_chains(N, L, q, seed=seed_chain)
    h0, J0, c0 = h.clone(), J.clone(), chains.clone()
    ws = api.workspace(B.WS_TRAIN_STEP, N, L, q, args.prec)
    pearson = torch.zeros(1, dtype=torch.float64, device="cuda")
    flips = torch.zeros(1, dtype=torch.int64, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")

    for ep in range(args.warmup):
        api.train_step(h, J, chains, f1, f2, lr, sweeps, seed_chain, ep, args.prec, ws, pearson,
                       flips, err)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} epochs done, pearson={float(pearson.cpu()[0]):.4f}")

    # ---------------- timed region: exactly K epochs
    flips.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        api.train_step(h, J, chains, f1, f2, lr, sweeps, seed_chain, args.warmup + k, args.prec,
                       ws, pearson, flips, err)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed * 1e3 / args.steps
    site_updates = N * L * sweeps * args.steps
    value = site_updates / elapsed
    flip_frac = float(flips.cpu()[0]) / site_updates
    assert int(err.cpu()[0]) == 0, "device error flag raised"
    log(f"timed {args.steps} epochs: {ms_step:.2f} ms/epoch, {value:.3e} site-updates/s, "
        f"flip fraction {flip_frac:.3f}, pearson {float(pearson.cpu()[0]):.4f}")

    # ---------------- the two sweep kernels alone, same chains and model
    reps = 5
    visits = N * L * sweeps
    ck = chains.clone()
    Wg = api.workspace(B.WS_GIBBS, N, L, q, B.SAMPLER_GATHER)
    kflips = torch.zeros(1, dtype=torch.int64, device="cuda")
    api.gibbs(h, J, ck, 1, seed_chain, sweep_offset=10**6 - 1, H_ws=Wg, sampler="gather")
    t.start()
    for r in range(reps):
        api.gibbs(h, J, ck, sweeps, seed_chain, sweep_offset=10**6 + r * sweeps, H_ws=Wg,
                  flips=kflips, sampler="gather")
    g_all = t.stop_ms() / reps
    t.start()
    for r in range(reps):  # the per-call coupling re-layout and token pass alone
        api.gibbs(h, J, ck, 0, seed_chain, H_ws=Wg, sampler="gather")
    g_fix = t.stop_ms() / reps
    g_ms = g_all - g_fix
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    lds_bytes = gather_lds_bytes(N, L, q, sweeps, cus)
    lds_gbs = lds_bytes / (g_ms * 1e-3) / 1e9
    lds_peak = cus * LDS_BYTES_PER_CLK * 2.4e9 / 1e9  # GB/s at 2.4 GHz
    # the row gathers alone in this launch's pattern (8-lane chains, as many
    # waves per workgroup as the planner gives these chains: at least 4, 8
    # chains per wave), measured on this device
    import ctypes
    pk = ctypes.CDLL(os.path.join(ROOT, "paper_2501_18456_amd", "libbmdca_peaks.so"))
    pk.bmdca_probe_lds_rows.restype = ctypes.c_double
    pk.bmdca_probe_lds_rows.argtypes = [ctypes.c_int] * 4
    row_rate = N * L * sweeps * (L - 1) / (g_ms * 1e-3)
    p_waves = max(4, -(-(-(-N // cus)) // 8))
    row_probe = pk.bmdca_probe_lds_rows(8, p_waves, 20000, cus) if q == 21 else None
    log(f"gather sweep kernel: {g_ms:.3f} ms per launch ({sweeps} sweeps; +{g_fix:.3f} ms re-layout), "
        f"{visits / (g_ms * 1e-3):.3e} site-updates/s, LDS {lds_gbs:.0f} GB/s of {lds_peak:.0f}; "
        f"{row_rate:.3e} row gathers/s"
        + (f" ({100 * row_rate / row_probe:.0f}% of the {row_probe:.3e}/s of the gathers alone "
           f"with {p_waves} waves)" if row_probe else ""))

    ck = chains.clone()
    H = api.workspace(B.WS_GIBBS, N, L, q, B.SAMPLER_FIELDS)
    api.gibbs(h, J, ck, 0, seed_chain, H_ws=H, sampler="fields")  # build the fields once
    kflips.zero_()
    t.start()
    for r in range(reps):
        api.gibbs(h, J, ck, sweeps, seed_chain, sweep_offset=10**6 + r * sweeps, H_ws=H,
                  flips=kflips, keep_fields=True, sampler="fields")
    k_ms = t.stop_ms() / reps
    kf = float(kflips.cpu()[0]) / reps
    alg_bytes = visits * 4 * q + kf * 8 * (Lq - q) + 2 * N * L
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    log(f"field sweep kernel: {k_ms:.2f} ms per launch ({sweeps} sweeps), flips/launch {kf:.3e}, "
        f"algorithmic HBM bytes {alg_bytes / 1e9:.2f} GB -> {achieved:.0f} GB/s")

    # ---------------- BF16 vs FP32 statistics on the same alignment
    extras = {"epoch_ms": ms_step, "flip_fraction": flip_frac,
              "pearson_after": float(pearson.cpu()[0]), "reweight_ms": rw_ms,
              "gather_kernel": {"ms_per_launch": g_ms, "relayout_ms": g_fix,
                                "site_updates_per_s": visits / (g_ms * 1e-3),
                                "lds_GBps": lds_gbs, "lds_frac": lds_gbs / lds_peak,
                                "row_gathers_per_s": row_rate, "row_probe_per_s": row_probe,
                                "row_probe_frac": row_rate / row_probe if row_probe else None},
              "field_kernel": {"ms_per_launch": k_ms, "site_updates_per_s": visits / (k_ms * 1e-3),
                               "alg_hbm_GBps": achieved, "hbm_frac": achieved / HBM_PEAK_GBS}}
    other = "bf16x2" if args.prec == "fp32" else "fp32"
    stat_ms = {args.prec: st_ms}
    t.start()
    g1, g2, _ = api.stats(msa, q, w, -1.0, other)
    stat_ms[other] = t.stop_ms()
    for p in ("fp32", "bf16x2"):  # warm timings
        t.start()
        api.stats(msa, q, w, -1.0, p)
        stat_ms[p] = t.stop_ms()
    extras["stats_ms"] = stat_ms
    extras["stats_bf16x2_vs_fp32_maxabs"] = {
        "f1": float((g1 - f1).abs().max()), "f2": float((g2 - f2).abs().max())}
    # epoch time in the other precision (same start state)
    hb, Jb, cb = h0.clone(), J0.clone(), c0.clone()
    wsb = api.workspace(B.WS_TRAIN_STEP, N, L, q, other)
    api.train_step(hb, Jb, cb, f1, f2, lr, sweeps, seed_chain, 0, other, wsb)
    t.start()
    for k in range(3):
        api.train_step(hb, Jb, cb, f1, f2, lr, sweeps, seed_chain, 1 + k, other, wsb)
    extras[f"epoch_ms_{other}"] = t.stop_ms() / 3
    extras[f"epoch_ms_{args.prec}"] = ms_step

    out = {
        "metric": METRIC, "value": value, "unit": "site-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (planted sparse Potts model; alignment sampled from it)",
        "config": {"workload": "bmDCA training epoch at protein scale", "L": L, "q": q,
                   "chains": N, "msa_rows": M, "sweeps_per_step": sweeps, "lr": lr,
                   "stats_precision": args.prec, "reweight_identity": 0.8},
        "roofline": {"kernel": "k_gibbs_gather (Gibbs sweeps, gather form)", "bound": "lds",
                     "achieved": lds_gbs, "peak": lds_peak, "unit": "GB/s",
                     "frac": lds_gbs / lds_peak, "traffic": gather_traffic("protein"),
                     "launch_ms": g_ms, "alg_bytes_per_launch": lds_bytes},
        "extras": extras,
    }

    # ---------------- oracle on the host cores (bounded sample)
    if emit and not args.no_cpu_baseline:
        from oracle import oracle as O
        n_s = min(args.cpu_chains, N)
        hh, JJ = h0.cpu().numpy(), J0.cpu().numpy()
        cc = c0[:n_s].cpu().numpy()
        F1, F2 = f1.cpu().numpy(), f2.cpu().numpy()
        log(f"oracle sample epoch: {n_s} chains ...")
        t1 = time.perf_counter()
        O.train_step(hh, JJ, cc, F1, F2, q, lr, sweeps, seed_chain, 0)
        cpu_s = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": n_s * L * sweeps / cpu_s, "unit": "site-updates/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"one epoch of the same workload with {n_s} of the "
                                         f"{N} chains ({cpu_s:.1f} s, single thread)"}
        log(f"oracle: {cpu_s:.1f} s")
    if emit:
        print(json.dumps(out), flush=True)
    return out


def bench_small(args):
    """Plain bmDCA at CPU-seconds size (L = 20, q = 21): planted dense model
    (h ~ N(0, 1), J ~ N(0, 0.1) on all pairs), M = 500 sequences drawn by 200
    sweeps, 80% identity weights, N = 500 chains, 10 sweeps per epoch, 20
    epochs, lr 0.05, FP32 statistics.  The whole run (alignment draw,
    reweighting, statistics, 20 epochs) is timed on the GPU and, with the same
    seeds, in the oracle on one host core; the trained parameters of the two
    are compared.  The epochs are also replayed from one captured graph: that
    takes as long as the eager calls, so the epoch is not launch-bound; at this
    size each site is one chunk and a sweep launch is 200 dependent chunk-steps
    of a few microseconds.  No roofline line at this size."""
    import numpy as np
    import torch

    from oracle import oracle as O
    from paper_2501_18456_amd import api, synth
    from paper_2501_18456_amd import _lib as B

    torch.cuda.set_device(0)
    L, q, M, N, sweeps, lr, epochs = 20, 21, 500, 500, 10, 0.05, 20
    h_true, J_true = synth.planted_dense(L, q, seed=1001, sigma_J=0.1)
    log(f"small: L={L} q={q} M={M} N={N} sweeps={sweeps} epochs={epochs} lr={lr} fp32")

    def gpu_run():
        ht, Jt = torch.from_numpy(h_true).cuda(), torch.from_numpy(J_true).cuda()
        msa = api.init_chains(M, L, q, seed=2001)
        api.gibbs(ht, Jt, msa, sweeps=200, seed=2001)
        _, w, _ = api.reweight(msa, q, 0.8)
        f1, f2, _ = api.stats(msa, q, w, -1.0, "fp32")
        h = torch.log(f1).float().reshape(L, q).contiguous()
        J = torch.zeros((L * q, L * q), dtype=torch.float32, device="cuda")
        ch = api.init_chains(N, L, q, seed=3001)
        ws = api.workspace(B.WS_TRAIN_STEP, N, L, q, "fp32")
        return h, J, ch, f1, f2, ws, msa

    for _ in range(max(args.warmup, 1)):  # warm: library load, kernel first calls
        gpu_run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h, J, ch, f1, f2, ws, msa_g = gpu_run()
    torch.cuda.synchronize()
    t_pre = time.perf_counter() - t0
    t = Timer()
    t.start()
    for e in range(epochs):
        pr = api.train_step(h, J, ch, f1, f2, lr, sweeps, 3001, e, "fp32", ws)
    ep_ms = t.stop_ms() / epochs
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    visits = N * L * sweeps
    log(f"GPU: preprocessing {t_pre * 1e3:.2f} ms, epoch {ep_ms:.3f} ms "
        f"({visits / (ep_ms * 1e-3):.3e} site-updates/s), whole run {t_all * 1e3:.1f} ms")
    # the same 20 epochs as replays of one captured epoch (a graph of one
    # model): the launch overhead of the small kernels goes away; the trained
    # parameters must equal the eager run's bit for bit
    hg, Jg, chg, f1g, f2g, wsg, _ = gpu_run()
    model = api.TrainModel(hg, Jg, chg, f1g, f2g, lr, sweeps, 3001, "fp32", ws=wsg)
    graph = api.TrainGroupGraph([model], lanes=1)
    torch.cuda.synchronize()
    t.start()
    for e in range(epochs):
        graph.launch()
    gep_ms = t.stop_ms() / epochs
    torch.cuda.synchronize()
    same = bool(torch.equal(Jg, J) and torch.equal(hg, h) and torch.equal(chg, ch))
    graph.close()
    log(f"GPU, graph-replayed epochs: {gep_ms:.3f} ms per epoch "
        f"({visits / (gep_ms * 1e-3):.3e} site-updates/s); parameters equal to the eager run: "
        f"{same}")
    out = {
        "metric": METRIC, "value": visits / (ep_ms * 1e-3), "unit": "site-updates/s",
        "n_gpus": 1, "steps": epochs, "warmup": max(args.warmup, 1), "ms_per_step": ep_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (planted dense Potts model; alignment sampled from it)",
        "config": {"workload": "plain bmDCA at CPU-seconds size", "L": L, "q": q, "chains": N,
                   "msa_rows": M, "sweeps_per_step": sweeps, "epochs": epochs, "lr": lr,
                   "stats_precision": "fp32", "reweight_identity": 0.8},
        "roofline": None,
        "extras": {"gpu_whole_run_ms": t_all * 1e3, "gpu_preprocessing_ms": t_pre * 1e3,
                   "pearson_after": float(pr.cpu()[0]), "graph_epoch_ms": gep_ms,
                   "graph_run_equals_eager": same},
    }
    if not args.no_cpu_baseline:
        t1 = time.perf_counter()
        msa = O.gibbs(h_true, J_true, O.init_chains(M, L, q, seed=2001), q, sweeps=200,
                      seed=2001)[0]
        _, w, _ = O.reweight(msa, 0.8)
        F1, F2, _ = O.stats(msa, q, w, -1.0)
        hh = np.log(F1).astype(np.float32).reshape(L, q)
        JJ = np.zeros((L * q, L * q), np.float32)
        cc = O.init_chains(N, L, q, seed=3001)
        for e in range(epochs):
            hh, JJ, cc, _, _, _ = O.train_step(hh, JJ, cc, F1, F2, q, lr, sweeps, 3001, e)
        cpu_s = time.perf_counter() - t1
        dJ = float(np.abs(J.cpu().numpy() - JJ).max())
        rows = int((msa_g.cpu().numpy() != msa).any(axis=1).sum())
        out["cpu_baseline"] = {"value": epochs * visits / cpu_s, "unit": "site-updates/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"the whole run ({cpu_s:.2f} s, single thread: "
                                         f"alignment draw, reweighting, statistics, "
                                         f"{epochs} epochs)"}
        out["extras"]["oracle_whole_run_s"] = cpu_s
        out["extras"]["max_abs_J_gpu_minus_oracle"] = dJ
        out["extras"]["alignment_rows_differing"] = rows
        log(f"oracle: whole run {cpu_s:.2f} s; alignment rows that differ: {rows} of {M}; "
            f"max |J_gpu - J_oracle| = {dJ:.3g} (both are 0 unless a draw fell within 1e-5 of "
            "a CDF step, after which the trajectories part)")
    print(json.dumps(out), flush=True)


def bench_next(args):
    """The next items at protein scale (L = 100, q = 21, planted sparse model as
    the trained model, alignment of M = 20 000 drawn by 200 sweeps, 80% identity
    weights): (1) the mixing time of Sec. 4.1 from 10 000 data-started chains
    and equilibrium sampling of 10 000 chains for 2 t_mix sweeps; (2)
    Metropolis sweeps of 10 000 chains (proposal uniform over the other q - 1
    states) in the gather and the field form; (3) one edDCA graph update
    (symmetric KL scores of every element, selection of the smallest 1%), one
    masked epoch, and one eaDCA graph update (Bernoulli KL scores of every
    element, the largest 0.1% of the inactive count activated).  The line's value is the gather-form Metropolis sweep
    rate; its roofline is that kernel's LDS traffic."""
    import numpy as np
    import torch

    from paper_2501_18456_amd import api, sampling, synth
    from paper_2501_18456_amd import _lib as B

    torch.cuda.set_device(0)
    L, q, M, N, sweeps, lr = 100, 21, 20000, 10000, 10, 0.05
    Lq = L * q
    h_true, J_true = synth.planted_sparse(L, q, seed=1002, sigma_J=0.5, gap_mass=0.15)
    h, J = torch.from_numpy(h_true).cuda(), torch.from_numpy(J_true).cuda()
    msa = api.init_chains(M, L, q, seed=2002)
    api.gibbs(h, J, msa, sweeps=200, seed=2002)
    _, w, _ = api.reweight(msa, q, 0.8)
    f1, f2, _ = api.stats(msa, q, w, -1.0, "bf16x2")
    torch.cuda.synchronize()
    log(f"next items: L={L} q={q} M={M} N={N}")
    extras = {}

    # (1) mixing time and equilibrium sampling
    sampling.mixing_time(h, J, msa, w, 1000, seed=7, max_sweeps=8)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_mix, rec, _ = sampling.mixing_time(h, J, msa, w, N, seed=7, max_sweeps=4096)
    torch.cuda.synchronize()
    mix_s = time.perf_counter() - t0
    last = rec[-1][0]
    t0 = time.perf_counter()
    chains, t_mix2, _ = sampling.sample_equilibrium(h, J, msa, w, N, N, seed=7, nmix=2,
                                                    max_sweeps=4096)
    torch.cuda.synchronize()
    eq_s = time.perf_counter() - t0
    extras["mixing"] = {"t_mix": t_mix, "checkpoints": len(rec) - 1, "last_sweep": last,
                        "ms": mix_s * 1e3, "site_updates_per_s": N * L * last / mix_s,
                        "equilibrium_sample_ms": eq_s * 1e3,
                        "records": [[r[0], r[1], r[3]] for r in rec]}
    log(f"mixing time {t_mix} sweeps ({len(rec) - 1} checkpoints, {mix_s * 1e3:.1f} ms, "
        f"{N * L * last / mix_s:.3e} site-updates/s with the SeqID read-backs); "
        f"equilibrium sample of {N} chains (mixing time + {2 * (t_mix or 0)} sweeps): "
        f"{eq_s * 1e3:.1f} ms")

    # (2) Metropolis sweeps: gather form (the default where the model fits)
    # and field form, on the same start chains
    t = Timer()
    reps = max(args.steps, 3)
    visits = N * L * sweeps
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    ch = api.init_chains(N, L, q, seed=3002)
    Wg = api.workspace(B.WS_GIBBS, N, L, q, B.SAMPLER_METROPOLIS | B.SAMPLER_GATHER)
    flips = torch.zeros(1, dtype=torch.int64, device="cuda")
    api.gibbs(h, J, ch, 1, 3002, H_ws=Wg, sampler="metropolis-gather")  # warm
    flips.zero_()
    t.start()
    for r in range(reps):
        api.gibbs(h, J, ch, sweeps, 3002, sweep_offset=1 + r * sweeps, H_ws=Wg, flips=flips,
                  sampler="metropolis-gather")
    mg_all = t.stop_ms() / reps
    acc_g = float(flips.cpu()[0]) / reps / visits
    t.start()
    for r in range(reps):  # the per-call coupling re-layout and token pass alone
        api.gibbs(h, J, ch, 0, 3002, H_ws=Wg, sampler="metropolis-gather")
    mg_fix = t.stop_ms() / reps
    mg_ms = mg_all - mg_fix
    lds_bytes = gather_lds_bytes(N, L, q, sweeps, cus, row_bytes=8)
    lds_gbs = lds_bytes / (mg_ms * 1e-3) / 1e9
    lds_peak = cus * LDS_BYTES_PER_CLK * 2.4e9 / 1e9
    log(f"Metropolis, gather form: {mg_ms:.2f} ms per {sweeps} sweeps (+{mg_fix:.3f} ms re-layout; "
        f"{visits / (mg_ms * 1e-3):.3e} site-updates/s), acceptance {acc_g:.3f}, "
        f"LDS {lds_gbs:.0f} GB/s of {lds_peak:.0f}")

    ch = api.init_chains(N, L, q, seed=3002)
    H = api.workspace(B.WS_GIBBS, N, L, q, B.SAMPLER_METROPOLIS | B.SAMPLER_FIELDS)
    api.gibbs(h, J, ch, 1, 3002, H_ws=H, sampler="metropolis-fields")  # builds the fields
    flips.zero_()
    t.start()
    for r in range(reps):
        api.gibbs(h, J, ch, sweeps, 3002, sweep_offset=1 + r * sweeps, H_ws=H, flips=flips,
                  keep_fields=True, sampler="metropolis-fields")
    m_ms = t.stop_ms() / reps
    acc = float(flips.cpu()[0]) / reps
    m_bytes = visits * 8 + acc * 8 * (Lq - q) + 2 * N * L
    m_gbs = m_bytes / (m_ms * 1e-3) / 1e9
    log(f"Metropolis, field form: {m_ms:.2f} ms per {sweeps} sweeps ({visits / (m_ms * 1e-3):.3e} "
        f"site-updates/s), acceptance {acc / visits:.3f}, algorithmic HBM {m_gbs:.0f} GB/s")
    g_ch = api.init_chains(N, L, q, seed=3002)
    t.start()
    for r in range(reps):
        api.gibbs(h, J, g_ch, sweeps, 3002, sweep_offset=r * sweeps)
    g_ms = t.stop_ms() / reps
    extras["metropolis"] = {"gather_ms_per_launch": mg_ms, "gather_relayout_ms": mg_fix,
                            "gather_acceptance": acc_g, "gather_lds_GBps": lds_gbs,
                            "fields_ms_per_launch": m_ms, "fields_acceptance": acc / visits,
                            "fields_alg_hbm_GBps": m_gbs,
                            "gibbs_ms_per_launch_same_chains": g_ms}

    # (3) element decimation: one graph update and one masked epoch
    mask = api.full_mask(L, q)
    J2 = J.clone() * mask.to(J.dtype)
    h2 = h.clone()
    ch2 = chains.clone()
    wsd = api.workspace(B.WS_DECIMATE, N, L, q, 0)
    n_act = torch.empty(1, dtype=torch.int64, device="cuda")
    api.decimate(J2.clone(), mask.clone(), ch2, q, 0.01, 0.0, ws=wsd, n_active=n_act)  # warm
    t.start()
    api.decimate(J2, mask, ch2, q, 0.01, 0.0, ws=wsd, n_active=n_act)
    d_ms = t.stop_ms()
    wst = api.workspace(B.WS_TRAIN_STEP, N, L, q, "bf16x2")
    api.train_step_masked(h2, J2, mask, ch2, f1, f2, lr, sweeps, 3003, 0, "bf16x2", wst)
    t.start()
    for e in range(3):
        api.train_step_masked(h2, J2, mask, ch2, f1, f2, lr, sweeps, 3003, 1 + e, "bf16x2", wst)
    me_ms = t.stop_ms() / 3
    total = L * (L - 1) // 2 * q * q
    extras["decimation"] = {"graph_update_ms": d_ms, "masked_epoch_ms": me_ms,
                            "active_after": int(n_act.cpu()[0]), "elements": total}
    log(f"edDCA: graph update {d_ms:.2f} ms ({total} elements scored, "
        f"{int(n_act.cpu()[0])} left), masked epoch {me_ms:.2f} ms")
    # element activation: one graph update from the empty graph (factivate 0.001)
    empty = torch.zeros((Lq, Lq), dtype=torch.uint8, device="cuda")
    api.activate(empty.clone(), ch2, f2, q, 0.001, ws=wsd, n_active=n_act)  # warm
    t.start()
    api.activate(empty, ch2, f2, q, 0.001, ws=wsd, n_active=n_act)
    a_ms = t.stop_ms()
    extras["activation"] = {"graph_update_ms": a_ms, "active_after": int(n_act.cpu()[0])}
    log(f"eaDCA: graph update {a_ms:.2f} ms ({total} elements scored, "
        f"{int(n_act.cpu()[0])} active)")

    out = {
        "metric": METRIC, "value": visits / (mg_ms * 1e-3), "unit": "site-updates/s",
        "n_gpus": 1, "steps": reps, "warmup": 1, "ms_per_step": mg_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (planted sparse Potts model; alignment sampled from it)",
        "config": {"workload": "equilibrium sampling, Metropolis sweeps, element "
                               "decimation and activation at protein scale", "L": L, "q": q, "chains": N,
                   "msa_rows": M, "sweeps_per_step": sweeps},
        "roofline": {"kernel": "k_gibbs_gather (Metropolis sweeps, gather form)",
                     "bound": "lds", "achieved": lds_gbs, "peak": lds_peak, "unit": "GB/s",
                     "frac": lds_gbs / lds_peak, "traffic": None, "launch_ms": mg_ms,
                     "alg_bytes_per_launch": lds_bytes},
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


def calibration_copy(args):
    """A plain device copy of known size first, when asked: its FETCH_SIZE /
    WRITE_SIZE counters scale the sweep kernel's in the same profiled run."""
    import torch
    if args.profile_copy_mib:
        n = args.profile_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst


def stats_product_flops(M, Lq, prec):
    """Dense MFMA work of the statistics product: 128-wide output tiles on or
    above the diagonal (64 x 128 for BF16 hi+lo, two products), K = M rows
    padded to 64."""
    Mpad = -(-M // 64) * 64
    if prec == "bf16x2":
        tiles64 = sum(-(-Lq // 128) - (ti * 64) // 128 for ti in range(-(-Lq // 64)))
        return 2.0 * 2 * Mpad * 64 * 128 * tiles64
    tiles128 = (-(-Lq // 128)) * (-(-Lq // 128) + 1) // 2
    return 2.0 * Mpad * 128 * 128 * tiles128


def bench_precision_epoch(args):
    """The precision form (the default line): training epochs at L = 256,
    q = 21, N = 20 000 chains on an alignment of M = 100 000 weighted
    sequences; FP32 form timed for `value`, BF16 hi+lo beside it."""
    import numpy as np
    import torch

    from paper_2501_18456_amd import api, synth
    from paper_2501_18456_amd import _lib as B

    torch.cuda.set_device(0)
    calibration_copy(args)
    L, q, M, N, sweeps, lr = 256, 21, 100000, 20000, 10, 0.05
    Lq = L * q
    seed_chain = 3003
    t_in = time.perf_counter()
    X_h = synth.clustered_msa(M, L, q, seed=2003, n_families=200, mut_rate=0.3)
    w_h = synth.weights_open_unit(M, 4003)
    msa = torch.from_numpy(X_h).cuda()
    w = torch.from_numpy(w_h).cuda()
    torch.cuda.synchronize()
    log(f"precision form: L={L} q={q} M={M} (phylogeny-like alignment, weights 1 - U[0,1)) "
        f"N={N} sweeps={sweeps}; inputs {time.perf_counter() - t_in:.1f} s")
    t = Timer()
    extras = {}

    # ---------------- weighted two-site statistics, both forms (run once per training)
    stats, st_ms, st_tf, st_frac = {}, {}, {}, {}
    peaks = {"bf16x2": 2500.0, "fp32": 157.3}
    for prec in ("bf16x2", "fp32"):
        ws = api.workspace(B.WS_STATS, M, L, q, prec)
        out = (torch.empty(Lq, dtype=torch.float64, device="cuda"),
               torch.empty((Lq, Lq), dtype=torch.float64, device="cuda"),
               torch.empty(1, dtype=torch.float64, device="cuda"))
        api.stats(msa, q, w, -1.0, prec, ws=ws, out=out)
        reps = max(3, min(args.steps, 10))
        t.start()
        for _ in range(reps):
            api.stats(msa, q, w, -1.0, prec, ws=ws, out=out)
        st_ms[prec] = t.stop_ms() / reps
        st_tf[prec] = stats_product_flops(M, Lq, prec) / (st_ms[prec] * 1e-3) / 1e12
        st_frac[prec] = st_tf[prec] / peaks[prec]
        stats[prec] = out
        del ws
        torch.cuda.empty_cache()
    # error against the FP64 oracle: every f1 entry and 2000 sampled f2 entries
    err = {}
    if not args.no_oracle_errors:
        from oracle import oracle as O
        g = np.random.default_rng(8)
        r1, r2 = g.integers(0, Lq, 2000), g.integers(0, Lq, 2000)
        d = np.arange(Lq)
        t1 = time.perf_counter()
        ref1 = O.stats_entries(X_h, q, d, d, w_h, -1.0)
        ref2 = O.stats_entries(X_h, q, r1, r2, w_h, -1.0)
        sel = torch.from_numpy(r1 * Lq + r2).cuda()
        for prec, (f1p, f2p, _) in stats.items():
            g1 = f1p.cpu().numpy()
            g2 = f2p.reshape(-1)[sel].cpu().numpy()
            nz1, nz2 = ref1 != 0, ref2 != 0
            err[prec] = {"f1_maxabs": float(np.abs(g1 - ref1).max()),
                         "f1_maxrel": float((np.abs(g1 - ref1)[nz1] / np.abs(ref1[nz1])).max()),
                         "f2_maxabs": float(np.abs(g2 - ref2).max()),
                         "f2_maxrel": float((np.abs(g2 - ref2)[nz2] / np.abs(ref2[nz2])).max()),
                         "entries": {"f1": int(Lq), "f2": 2000},
                         "f2_zero_entries_exact": bool((g2[~nz2] == 0).all())}
        log(f"oracle entries for the statistics errors: {time.perf_counter() - t1:.1f} s")
    for prec in ("bf16x2", "fp32"):
        e = err.get(prec, {})
        log(f"stats {prec}: {st_ms[prec]:.2f} ms, {st_tf[prec]:.0f} TFLOP/s dense tile work "
            f"({100 * st_frac[prec]:.0f}% of {peaks[prec]:.0f}); max |f - f_FP64| "
            f"f1 {e.get('f1_maxabs', float('nan')):.2e} f2 {e.get('f2_maxabs', float('nan')):.2e}")
    extras["stats"] = {"ms": st_ms, "tflops": st_tf, "mfma_frac": st_frac,
                       "peak_tflops": peaks, "error_vs_fp64_oracle": err,
                       "alg_flops_per_call": {p: stats_product_flops(M, Lq, p) for p in peaks}}

    # ---------------- training epochs: FP32 form timed for `value`, then BF16 hi+lo;
    # chain counts counted directly (the library default), and for the comparison
    # of the two product forms also from the one-hot product of each precision
    epoch_ms, pear, flipf = {}, {}, {}
    forms = {"fp32": B.PREC_FP32, "bf16x2": B.PREC_BF16X2,
             "fp32_product_counts": B.PREC_FP32 | B.COUNTS_PRODUCT,
             "bf16x2_product_counts": B.PREC_BF16X2 | B.COUNTS_PRODUCT}
    for form, prec in forms.items():
        f1, f2, _ = stats[form.split("_")[0]]
        h = api.profile_fields(f1, L, q)
        J = torch.zeros((Lq, Lq), dtype=torch.float32, device="cuda")
        ch = api.init_chains(N, L, q, seed=seed_chain)
        wst = api.workspace(B.WS_TRAIN_STEP, N, L, q, prec)
        pearson = torch.zeros(1, dtype=torch.float64, device="cuda")
        flips = torch.zeros(1, dtype=torch.int64, device="cuda")
        derr = torch.zeros(1, dtype=torch.int32, device="cuda")
        for ep in range(args.warmup):
            api.train_step(h, J, ch, f1, f2, lr, sweeps, seed_chain, ep, prec, wst, pearson,
                           flips, derr)
        flips.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            api.train_step(h, J, ch, f1, f2, lr, sweeps, seed_chain, args.warmup + k, prec, wst,
                           pearson, flips, derr)
        torch.cuda.synchronize()
        epoch_ms[form] = (time.perf_counter() - t0) * 1e3 / args.steps
        pear[form] = float(pearson.item())
        flipf[form] = float(flips.item()) / (N * L * sweeps * args.steps)
        assert int(derr.item()) == 0, "device error flag raised"
        log(f"epoch {form}: {epoch_ms[form]:.2f} ms ({N * L * sweeps / (epoch_ms[form] * 1e-3):.3e} "
            f"site-updates/s), flip fraction {flipf[form]:.3f}, pearson {pear[form]:.4f}")
        if form == "fp32":
            h_run, J_run, ch_run = h, J, ch
        else:
            del h, J, ch
        del wst
        torch.cuda.empty_cache()
    value = N * L * sweeps / (epoch_ms["fp32"] * 1e-3)
    extras["epoch_ms"] = epoch_ms
    extras["site_updates_per_s"] = {p: N * L * sweeps / (v * 1e-3) for p, v in epoch_ms.items()}
    extras["mixed_speedup_over_fp32"] = epoch_ms["fp32"] / epoch_ms["bf16x2"]
    extras["mixed_speedup_over_fp32_product_counts"] = (epoch_ms["fp32_product_counts"] /
                                                       epoch_ms["bf16x2_product_counts"])
    extras["pearson_after"] = pear
    extras["flip_fraction"] = flipf

    # ---------------- the sweep kernels alone on the trained model and its chains
    reps = 5
    visits = N * L * sweeps
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    ck = ch_run.clone()
    Wg = api.workspace(B.WS_GIBBS, N, L, q, B.SAMPLER_GATHER)
    api.gibbs(h_run, J_run, ck, 1, seed_chain, sweep_offset=10**6 - 1, H_ws=Wg, sampler="gather")
    t.start()
    for r in range(reps):
        api.gibbs(h_run, J_run, ck, sweeps, seed_chain, sweep_offset=10**6 + r * sweeps, H_ws=Wg,
                  sampler="gather")
    g_all = t.stop_ms() / reps
    t.start()
    for r in range(reps):  # the per-call coupling re-layout alone
        api.gibbs(h_run, J_run, ck, 0, seed_chain, H_ws=Wg, sampler="gather")
    g_fix = t.stop_ms() / reps
    g_ms = g_all - g_fix
    lds_bytes = gather_lds_bytes(N, L, q, sweeps, cus)
    lds_gbs = lds_bytes / (g_ms * 1e-3) / 1e9
    lds_peak = cus * LDS_BYTES_PER_CLK * 2.4e9 / 1e9
    # the rate of the row gathers alone in the narrow-chain pattern at q = 21
    # (10 chains of 6 lanes per wave, one 8-wave workgroup per CU, random rows of
    # a 16-site chunk) on this device: a probe without staging, draws or barriers
    import ctypes
    pk = ctypes.CDLL(os.path.join(ROOT, "paper_2501_18456_amd", "libbmdca_peaks.so"))
    pk.bmdca_probe_lds_rows.restype = ctypes.c_double
    pk.bmdca_probe_lds_rows.argtypes = [ctypes.c_int] * 4
    row_rate = N * L * sweeps * (L - 1) / (g_ms * 1e-3)  # coupling rows gathered per second
    row_probe = pk.bmdca_probe_lds_rows(6, 8, 20000, cus) if q == 21 else None
    log(f"gather sweep kernel: {g_ms:.2f} ms per launch ({sweeps} sweeps; +{g_fix:.3f} ms "
        f"re-layout), {visits / (g_ms * 1e-3):.3e} site-updates/s, LDS {lds_gbs:.0f} GB/s of "
        f"{lds_peak:.0f}; {row_rate:.3e} row gathers/s"
        + (f" ({100 * row_rate / row_probe:.0f}% of the {row_probe:.3e}/s that the gathers alone "
           f"reach in the same pattern)" if row_probe else ""))
    del Wg
    ck = ch_run.clone()
    H = api.workspace(B.WS_GIBBS, N, L, q, B.SAMPLER_FIELDS)
    api.gibbs(h_run, J_run, ck, 0, seed_chain, H_ws=H, sampler="fields")
    kfl = torch.zeros(1, dtype=torch.int64, device="cuda")
    fs = 5  # sweeps
    t.start()
    api.gibbs(h_run, J_run, ck, fs, seed_chain, sweep_offset=2 * 10**6, H_ws=H, flips=kfl,
              keep_fields=True, sampler="fields")
    f_ms = t.stop_ms()
    fv = N * L * fs
    fl = float(kfl.item())
    f_bytes = fv * 4 * q + fl * 8 * (Lq - q) + 2 * N * L
    f_gbs = f_bytes / (f_ms * 1e-3) / 1e9
    log(f"field sweep kernel: {f_ms:.1f} ms per {fs} sweeps, flip fraction {fl / fv:.3f}, "
        f"algorithmic HBM {f_gbs:.0f} GB/s ({100 * f_gbs / HBM_PEAK_GBS:.0f}% of peak; H = "
        f"{N * Lq * 4 / 1e6:.0f} MB, beyond the 256 MB last-level cache)")
    del H
    torch.cuda.empty_cache()
    extras["gather_kernel"] = {"ms_per_launch": g_ms, "sweeps_per_launch": sweeps,
                               "relayout_ms": g_fix,
                               "site_updates_per_s": visits / (g_ms * 1e-3),
                               "alg_lds_bytes_per_launch": lds_bytes, "lds_GBps": lds_gbs,
                               "lds_frac": lds_gbs / lds_peak}
    extras["field_kernel"] = {"ms_per_launch": f_ms, "sweeps_per_launch": fs,
                              "flip_fraction": fl / fv, "alg_hbm_bytes_per_launch": f_bytes,
                              "alg_hbm_GBps": f_gbs, "hbm_frac": f_gbs / HBM_PEAK_GBS,
                              "site_updates_per_s": fv / (f_ms * 1e-3),
                              "traffic": gather_traffic("precision-fields")}

    # ---------------- protein scale as context
    if not args.no_protein:
        del ch_run, J_run, h_run
        torch.cuda.empty_cache()
        pa = argparse.Namespace(**vars(args))
        pa.steps, pa.warmup = 10, 2
        po = bench_protein(pa, emit=False)
        extras["protein_scale"] = {"config": po["config"], "ms_per_step": po["ms_per_step"],
                                   "site_updates_per_s": po["value"],
                                   "gather_kernel": po["extras"]["gather_kernel"],
                                   "field_kernel": po["extras"]["field_kernel"],
                                   "gather_traffic": po["roofline"]["traffic"]}

    out = {
        "metric": METRIC, "value": value, "unit": "site-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": epoch_ms["fp32"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (phylogeny-like alignment of seeded ancestors and mutations; "
                "weights 1 - U[0,1); model trained from the profile start)",
        "config": {"workload": "precision form: bmDCA training epoch at L=256, q=21, "
                               "M=100000 weighted rows, N=20000 chains",
                   "L": L, "q": q, "msa_rows": M, "chains": N, "sweeps_per_step": sweeps,
                   "lr": lr, "step_form": "fp32 (BF16 hi+lo epoch in extras)"},
        "roofline": {"kernel": "k_gibbs_gather (Gibbs sweeps, gather form)", "bound": "lds",
                     "achieved": lds_gbs, "peak": lds_peak, "unit": "GB/s",
                     "frac": lds_gbs / lds_peak, "traffic": gather_traffic("precision"),
                     "launch_ms": g_ms, "alg_bytes_per_launch": lds_bytes,
                     "row_gathers_per_s": row_rate, "row_probe_per_s": row_probe,
                     "row_probe_frac": row_rate / row_probe if row_probe else None},
        "extras": extras,
    }

    # ---------------- oracle on the host cores (bounded sample, extrapolated)
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        info = cpu_info()
        n_s = min(args.cpu_chains, N)
        f1, f2, _ = stats["fp32"]
        F1, F2 = f1.cpu().numpy(), f2.cpu().numpy()
        hh = np.log(F1).astype(np.float32).reshape(L, q)
        JJ = np.zeros((Lq, Lq), np.float32)
        cc = O.init_chains(n_s, L, q, seed_chain)
        res = {}
        for label, threads in (("single_thread", False), ("all_cores", True)):
            log(f"oracle sample epoch ({label}): {n_s} of {N} chains ...")
            t1 = time.perf_counter()
            O.train_step(hh, JJ, cc, F1, F2, q, lr, sweeps, seed_chain, 0, threads=threads)
            cpu_s = time.perf_counter() - t1
            res[label] = {"value": n_s * L * sweeps / cpu_s, "seconds": cpu_s,
                          "cores": info["omp_threads"] if threads else 1}
            log(f"oracle ({label}): {cpu_s:.1f} s")
        allc = res["all_cores"]
        out["cpu_baseline"] = {
            "value": allc["value"], "unit": "site-updates/s", "cores": allc["cores"],
            "kind": "oracle",
            "sample": f"one epoch (10 sweeps, chain statistics, Pearson, update) of {n_s} of the "
                      f"{N} chains at L={L}, q={q}, timed and extrapolated per site-update "
                      f"({allc['seconds']:.1f} s on {allc['cores']} threads; single thread "
                      f"{res['single_thread']['seconds']:.1f} s)",
            "extrapolated": True, "single_thread": res["single_thread"],
            "nproc": info["nproc"], "usable_cores": info["usable"], "cpu_model": info["model"]}
    print(json.dumps(out), flush=True)


def bench_scoring(args):
    """Pre-processing and scoring kernels at their largest workload sizes:
    reweighting of M = 100 000 rows at L = 256 (integer pair counts), and for a
    resident L = 512, q = 21 model: energies of 100 000 sequences, mutant scans
    of 64 wild types, the APC contact map."""
    import numpy as np
    import torch

    from paper_2501_18456_amd import api, synth
    from paper_2501_18456_amd import _lib as B

    torch.cuda.set_device(0)
    calibration_copy(args)
    t = Timer()
    # ---- reweighting: L = 256, q = 21, M = 100 000 rows drawn from a planted model
    L, q, M = 256, 21, 100000
    h_true, J_true = synth.planted_dense(L, q, seed=1003, sigma_J=0.05)
    msa = api.init_chains(M, L, q, seed=2003)
    api.gibbs(torch.from_numpy(h_true).cuda(), torch.from_numpy(J_true).cuda(), msa, 50, 2003)
    ws = api.workspace(B.WS_REWEIGHT, M, L, q, 0)
    api.reweight(msa, q, 0.8, ws=ws)
    t.start()
    for _ in range(args.steps):
        n_sim, w, meff = api.reweight(msa, q, 0.8, ws=ws)
    rw_ms = t.stop_ms() / args.steps
    P, W = 5, -(-L // 32)
    # every unordered pair is compared once: M(M-1)/2 pairs (plus the M self
    # pairs); per pair one three-input bit operation per plane word ((a ^ b) |
    # c, the first plane a plain XOR), one popcount-accumulate per word,
    # threshold test and count, and the column side's ballot and popcount
    ops_pair = W * P + W + 4
    rw_pairs = M * (M - 1) / 2 + M
    rw_ops = rw_pairs * ops_pair
    # integer VALU peak measured on this device by a probe of the same
    # operation mix (8 independent chains per lane, 1M lanes)
    import ctypes
    pk = ctypes.CDLL(os.path.join(ROOT, "paper_2501_18456_amd", "libbmdca_peaks.so"))
    pk.bmdca_probe_int_valu.restype = ctypes.c_double
    pk.bmdca_probe_int_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    int_peak = pk.bmdca_probe_int_valu(1, 20000, 4096)
    int_peak_bitop = pk.bmdca_probe_int_valu(0, 20000, 4096)
    nominal = 256 * 64 * 2.4e9  # one wave64 instruction per CU and clock
    log(f"integer VALU probe: {int_peak / 1e12:.1f} T lane-ops/s (pair-count mix), "
        f"{int_peak_bitop / 1e12:.1f} T (bit operations only); 256 CU x 64 lanes x 2.4 GHz = "
        f"{nominal / 1e12:.1f} T")
    log(f"reweight M={M} L={L}: {rw_ms:.1f} ms, {rw_pairs / (rw_ms * 1e-3):.3e} unordered pairs/s, "
        f"{rw_ops / (rw_ms * 1e-3) / 1e12:.2f} Tops/s ({100 * rw_ops / (rw_ms * 1e-3) / int_peak:.1f}% "
        f"of the probed integer VALU rate); max n_sim {int(n_sim.max())}, "
        f"M_eff {float(meff.item()):.1f}")
    del msa, ws, n_sim, w
    torch.cuda.empty_cache()
    # ---- scoring of a resident L = 512 model
    L, q = 512, 21
    Lq = L * q
    h, J = synth.planted_dense(L, q, seed=5007, sigma_J=0.02)
    hg, Jg = torch.from_numpy(h).cuda(), torch.from_numpy(J).cuda()
    Bn = 100000
    S = torch.from_numpy(synth.random_sequences(Bn, L, q, 6)).cuda()
    wse = api.workspace(B.WS_ENERGY, Bn, L, q, 0)
    E = torch.empty(Bn, dtype=torch.float32, device="cuda")
    api.energy(hg, Jg, S, out=E, ws=wse)
    t.start()
    for _ in range(args.steps):
        api.energy(hg, Jg, S, out=E, ws=wse)
    en_ms = t.stop_ms() / args.steps
    pairs = Bn * L * (L - 1) / 2
    blocks = -(-Bn // (2048 if q > 8 else 1024))  # sequences per workgroup
    tiles = sum(min(16 * jc + 15, L - 1) for jc in range(-(-L // 16)))
    lds_bytes = pairs * 4 + blocks * tiles * q * 16 * q * 4  # lookups + staged tiles
    lds_peak = 256 * LDS_BYTES_PER_CLK * 2.4e9
    # the rate that random 4-byte LDS lookups of the same address pattern reach
    # on this device (a probe without tile staging, token loads or step
    # bookkeeping), at the kernel's tile row pitch: 16 q floats plus the pad
    # of 0, 4, 8 or 12 whose largest per-bank share of the q^2 (row, column)
    # pairs is smallest, then the smallest sum of squared shares, among the
    # pads that keep the workgroups per CU
    def energy_pitch(qq):
        thr = 512 if qq > 8 else 256
        cap = 32 // (thr // 64)
        wgs = lambda b: min(163840 // b, cap)
        wg0 = wgs(2 * qq * 16 * qq * 4)
        best = None
        for pad in (0, 4, 8, 12):
            P_ = 16 * qq + pad
            if wgs(2 * qq * P_ * 4) < wg0:
                continue
            cnt = [0] * 64
            for a in range(qq):
                for b in range(qq):
                    cnt[(P_ * a + b) % 64] += 1
            key = (max(cnt), sum(x * x for x in cnt))
            if best is None or key < best[0]:
                best = (key, P_)
        return best[1]
    pk.bmdca_probe_lds_lookups.restype = ctypes.c_double
    pk.bmdca_probe_lds_lookups.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lk_pitch = energy_pitch(q)
    lk_peak = pk.bmdca_probe_lds_lookups(lk_pitch, 2000, 4096)
    lk_rate = pairs / (en_ms * 1e-3)
    log(f"energy B={Bn} L={L}: {en_ms:.2f} ms, {Bn / (en_ms * 1e-3):.3e} sequences/s, "
        f"{pairs / (en_ms * 1e-3):.3e} pair terms/s, LDS {lds_bytes / (en_ms * 1e-3) / 1e12:.1f} TB/s; "
        f"random-lookup probe at pitch {lk_pitch}: {lk_peak:.3e} lookups/s "
        f"({100 * lk_rate / lk_peak:.0f}% reached)")
    del S, wse, E
    torch.cuda.empty_cache()
    nw = 64
    WT = torch.from_numpy(synth.random_sequences(nw, L, q, 7)).cuda()
    wsm = api.workspace(B.WS_MUTANT, nw, L, q, 0)
    dE = torch.empty((nw, Lq), dtype=torch.float32, device="cuda")
    api.single_mutant_scan(hg, Jg, WT, ws=wsm, out=dE)
    t.start()
    for _ in range(args.steps):
        api.single_mutant_scan(hg, Jg, WT, ws=wsm, out=dE)
    mu_ms = t.stop_ms() / args.steps
    mu_bytes = nw * (L * Lq * 4 + 2 * Lq * 4)  # L coupling rows per wild type, fields, output
    # wild types that share a residue at a site read the same coupling row: the
    # distinct rows are the bytes that HBM has to deliver at least once
    wt_np = WT.cpu().numpy()
    mu_rows = sum(len(set(wt_np[:, j].tolist())) for j in range(L))
    mu_hbm = mu_rows * Lq * 4 + nw * 2 * Lq * 4
    log(f"mutant scans {nw} wild types L={L}: {mu_ms:.2f} ms, rows as read "
        f"{mu_bytes / (mu_ms * 1e-3) / 1e9:.0f} GB/s, distinct rows {mu_hbm / (mu_ms * 1e-3) / 1e9:.0f} GB/s")
    wsa = api.workspace(B.WS_APC, 0, L, q, 0)
    api.apc_frobenius(Jg, L, q, 0, ws=wsa)
    t.start()
    for _ in range(args.steps):
        F, Fa = api.apc_frobenius(Jg, L, q, 0, ws=wsa)
    apc_ms = t.stop_ms() / args.steps
    apc_bytes = Lq * Lq * 4 // 2  # J is symmetric: the blocks j > i are read once
    log(f"APC Frobenius L={L}: {apc_ms:.2f} ms, {apc_bytes / (apc_ms * 1e-3) / 1e9:.0f} GB/s")
    out = {
        "metric": METRIC, "value": Bn / (en_ms * 1e-3), "unit": "sequences/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": en_ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (planted models; uniform random sequences)",
        "config": {"workload": "scoring of an L=512, q=21 model (energies of 100000 sequences, "
                               "64 mutant scans, APC) and reweighting of 100000 rows at L=256"},
        "roofline": {"kernel": "k_energy_pairs (energies)", "bound": "lds",
                     "achieved": lds_bytes / (en_ms * 1e-3) / 1e9, "peak": lds_peak / 1e9,
                     "unit": "GB/s", "frac": lds_bytes / (en_ms * 1e-3) / lds_peak,
                     "traffic": None, "call_ms": en_ms, "alg_bytes_per_call": lds_bytes,
                     "lookups_per_s": lk_rate, "lookup_probe_per_s": lk_peak,
                     "lookup_probe_frac": lk_rate / lk_peak, "tile_pitch_floats": lk_pitch},
        "extras": {
            "reweight": {"ms": rw_ms, "unordered_pairs_per_s": rw_pairs / (rw_ms * 1e-3),
                         "ops_per_pair": ops_pair, "int_ops_per_s": rw_ops / (rw_ms * 1e-3),
                         "alu_probe_ops_per_s": int_peak, "alu_probe_bitop_ops_per_s":
                         int_peak_bitop, "alu_nominal_ops_per_s": nominal,
                         "alu_frac": rw_ops / (rw_ms * 1e-3) / int_peak, "M": M, "L": 256},
            "mutant_scan": {"ms": mu_ms, "wild_types": nw,
                            "rows_read_GBps": mu_bytes / (mu_ms * 1e-3) / 1e9,
                            "distinct_rows": mu_rows,
                            "GBps": mu_hbm / (mu_ms * 1e-3) / 1e9,
                            "hbm_frac": mu_hbm / (mu_ms * 1e-3) / 8e12},
            "apc": {"ms": apc_ms, "GBps": apc_bytes / (apc_ms * 1e-3) / 1e9,
                    "hbm_frac": apc_bytes / (apc_ms * 1e-3) / 8e12},
        },
    }
    print(json.dumps(out), flush=True)


def bench_group(args):
    """64 planted models of uneven size trained together: one captured graph
    replays one epoch of every model (lane streams side by side)."""
    import numpy as np
    import torch

    from paper_2501_18456_amd import api, synth
    from paper_2501_18456_amd import _lib as B

    torch.cuda.set_device(0)
    n_models, N, sweeps, lr, msa_sweeps = 64, 4096, 10, 0.05, 20
    rng = np.random.default_rng(4000)
    Ls = rng.integers(50, 401, size=n_models)
    qs = np.array([21] * 48 + [5] * 16)
    rng.shuffle(qs)
    Ms = rng.integers(5000, 50001, size=n_models)
    log(f"group workload: {n_models} models, L {Ls.min()}..{Ls.max()}, "
        f"{int((qs == 21).sum())} with q=21 and {int((qs == 5).sum())} with q=5, N={N}")
    models = []
    t_setup = time.perf_counter()
    for k in range(n_models):
        L, q, M = int(Ls[k]), int(qs[k]), int(Ms[k])
        h_true, J_true = synth.planted_sparse(L, q, seed=1000 + k, sigma_J=0.5, gap_mass=0.15)
        ht, Jt = torch.from_numpy(h_true).cuda(), torch.from_numpy(J_true).cuda()
        msa = api.init_chains(M, L, q, seed=2000 + k)
        api.gibbs(ht, Jt, msa, sweeps=msa_sweeps, seed=2000 + k)
        _, w, _ = api.reweight(msa, q, 0.8)
        f1, f2, _ = api.stats(msa, q, w, -1.0, "bf16x2")
        h = torch.log(f1).to(torch.float32).reshape(L, q).contiguous()
        J = torch.zeros((L * q, L * q), dtype=torch.float32, device="cuda")
        chains = api.init_chains(N, L, q, seed=3000 + k)
        models.append(api.TrainModel(h, J, chains, f1, f2, lr, sweeps, 3000 + k, "bf16x2"))
        del ht, Jt, msa, w
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"setup (alignments by {msa_sweeps} sweeps, reweighting, BF16 statistics) "
        f"{time.perf_counter() - t_setup:.1f} s, "
        f"{torch.cuda.memory_allocated() / 2**30:.1f} GiB resident")
    graph = api.TrainGroupGraph(models, lanes=args.lanes)
    for _ in range(args.warmup):
        graph.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.launch()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed * 1e3 / args.steps
    per_epoch = sum(m.N * m.L * sweeps for m in models)
    value = per_epoch * args.steps / elapsed
    pear = [float(m.pearson.item()) for m in models]
    log(f"group epoch {ms_step:.1f} ms, {value:.3e} site-updates/s, "
        f"Pearson {min(pear):.3f}..{max(pear):.3f}")
    # the same epochs run model after model on one stream (no graph, no lanes)
    t = Timer()
    t.start()
    for m in models:
        api.train_step(m.h, m.J, m.chains, m.f1, m.f2, lr, sweeps, 3000, 10**6, m.prec,
                       m.ws, m.pearson)
    solo_ms = t.stop_ms()
    log(f"sum of the 64 solo epochs {solo_ms:.1f} ms -> group speedup {solo_ms / ms_step:.2f}x")
    out = {
        "metric": METRIC, "value": value, "unit": "site-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (64 planted sparse Potts models; alignments sampled from them)",
        "config": {"workload": "grouped bmDCA training, 64 uneven models, one captured graph "
                               "per epoch", "models": n_models, "L_range": [int(Ls.min()),
                                                                              int(Ls.max())],
                   "q21_models": int((qs == 21).sum()), "q5_models": int((qs == 5).sum()),
                   "chains_per_model": N, "msa_rows_range": [int(Ms.min()), int(Ms.max())],
                   "sweeps_per_step": sweeps, "stats_precision": "bf16x2", "lanes": args.lanes},
        "roofline": None,
        "extras": {"solo_sum_ms": solo_ms, "group_speedup_vs_solo_sum": solo_ms / ms_step,
                   "site_updates_per_epoch": per_epoch,
                   "resident_GiB": torch.cuda.memory_allocated() / 2**30},
    }
    graph.close()
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Poisson request streams against 8 resident models at three rates: light
    (0.3x), knee (0.8x) and saturating (1.3x) of the measured capacity.  Every
    batch is one replay of its engine's captured graph."""
    import numpy as np
    import torch

    from paper_2501_18456_amd import serve

    torch.cuda.set_device(0)
    Ls, q = (64, 128, 200, 256, 320, 400, 450, 512), 21
    models = serve.resident_models(Ls, q)
    budget = int(args.serve_budget_gib * 2**30)
    mix = (0.4, 0.4, 0.2)
    t0 = time.perf_counter()
    srv = serve.Server(models, budget, lanes=args.lanes, chunk_sweeps=args.serve_chunk,
                       sample_cus=args.serve_cus)
    log(f"engines: {len(srv.engines)} captured graphs, arenas {srv.stats.arena_bytes / 2**30:.2f} "
        f"GiB of the {args.serve_budget_gib:.0f} GiB budget, built in "
        f"{time.perf_counter() - t0:.1f} s")
    # warmup: every kind on every model once
    warm = serve.poisson_requests(48, 1e6, Ls, q, seed=7, mix=(1, 1, 1),
                                  energy_range=(1000, 2000), chain_range=(100, 200))
    srv.run(warm, realtime=False)
    torch.cuda.synchronize()
    # capacity: a burst of requests all present at once
    n_cap = max(100, args.serve_requests // 10)
    burst = serve.poisson_requests(n_cap, 1e6, Ls, q, seed=8, mix=mix)
    srv.reset_stats()
    t0 = time.perf_counter()
    srv.run(burst, realtime=False)
    cap = n_cap / (time.perf_counter() - t0)
    log(f"capacity {cap:.1f} requests/s ({n_cap}-request burst)")
    del burst
    rates = {"light": 0.3 * cap, "knee": 0.8 * cap, "saturating": 1.3 * cap}
    results = {}
    for k, (name, rate) in enumerate(rates.items()):
        reqs = serve.poisson_requests(args.serve_requests, rate, Ls, q, seed=100 + k, mix=mix)
        srv.reset_stats()
        t0 = time.perf_counter()
        srv.run(reqs, realtime=True,
                progress=lambda d, n: log(f"{name}: {d} of {n} requests done"))
        wall = time.perf_counter() - t0
        sm = serve.summarize(reqs)
        st = srv.stats
        n_req = len(reqs)
        sm.update({"offered_per_s": rate, "wall_s": wall,
                   "peak_admitted_GiB": st.peak_bytes / 2**30,
                   "graph_launches": dict(st.launches), "eager_launches": dict(st.eager),
                   "request_launches": dict(st.batched),
                   "launches_per_request": (sum(st.launches.values()) +
                                            sum(st.eager.values())) / n_req})
        results[name] = sm
        log(f"{name}: offered {rate:.1f}/s served {sm['requests_per_s']:.1f}/s; " + "; ".join(
            f"{kd} p50 {sm[kd]['p50_ms']:.1f} p99 {sm[kd]['p99_ms']:.1f} ms"
            for kd in serve.KINDS if kd in sm) +
            f"; {sm['launches_per_request']:.2f} launches per request")
        del reqs
    sat = results["saturating"]
    out = {
        "metric": METRIC, "value": sat["requests_per_s"], "unit": "requests/s", "n_gpus": 1,
        "steps": args.serve_requests, "warmup": 48, "ms_per_step": 1e3 / sat["requests_per_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (planted models as stand-ins for trained ones; uniform random "
                "sequences and wild types)",
        "config": {"workload": "serving: 8 resident models L 64..512, q=21; Poisson arrivals; "
                               "energy 1k-100k sequences, full single-mutant scans, sampling "
                               "100-10000 chains x 50 sweeps (mix 0.4/0.4/0.2)",
                   "budget_GiB": args.serve_budget_gib, "lanes": args.lanes,
                   "chunk_sweeps": args.serve_chunk, "sample_cus": args.serve_cus,
                   "requests_per_rate": args.serve_requests},
        "roofline": None,
        "extras": {"capacity_per_s": cap, "arena_GiB": srv.stats.arena_bytes / 2**30,
                   "rates": results},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
