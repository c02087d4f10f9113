"""Request loop over resident trained models (scoring, mutant scans, sampling).

Uses of a trained Potts model from Sec. 4 of the paper (energies of a sequence
set, Sec. 4.3; the single-mutant library, Sec. 4.4; sampling, Sec. 4.1)
served to a stream of requests:

  - models stay resident in HBM (h, J as float32);
  - every (kind, model) pair owns an engine: fixed device arenas (inputs,
    outputs, workspace, a device work table) sized once from the HBM budget,
    and ONE captured HIP graph of the library's serving call over the whole
    arena (bmdca_energy_batch, bmdca_mutant_scan_batch, bmdca_sample_tick).
    The live item count, and for sampling each chain's random stream, are
    device data the host writes before a replay, so the same graph serves
    every batch: one graph launch per batch;
  - admission by HBM footprint: a request is admitted into its engine's
    arena, in arrival order among that engine's requests, once its items fit
    beside the ones in flight (a full arena holds back only its own
    requests); a request larger than its arena is refused at once;
  - continuous batching (iteration-level): each engine has at most one
    replay in flight; when it is free, every admitted request of that engine
    that fits goes into the next replay.  Sampling runs in ticks of
    `chunk_sweeps` sweeps over all live chains of the model: requests join at
    the next tick, leave when their sweeps are done (their chains are copied
    out and the arena compacted), and each chain draws with its own request's
    key, chain index and sweep offset from the work table;
  - engines run on `lanes` streams (default priority), sampling and scoring
    on disjoint ones, and overlap on the GPU; completion is seen by polling
    events, results come back through pinned host buffers on the engine's
    stream.

A request's result does not depend on what else is in flight: energies of a
sequence are independent of the batch (pair order fixed by L), mutant scans
are per wild type, and the gather-form sampler's draws depend only on the
chain's stream record (its field sums follow lanes per chain fixed by q and
the draw, or narrow lanes that give the same bits), so
every result equals the plain library call made alone, bit for bit.  Every
computation runs in the HIP library; this module moves data and decides
what to launch when.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as B
from . import api

KINDS = ("energy", "mutant", "sample")
# default arena capacities (items): two of the largest energy batches, a
# batch of mutant scans, and the chains of several sampling requests
DEFAULT_CAPS = {"energy": 200000, "mutant": 64, "sample": 65536}


@dataclass
class Request:
    rid: int
    kind: str           # "energy" | "mutant" | "sample"
    model: int          # index of the resident model
    arrival: float      # seconds after the start of the run
    seqs: np.ndarray | None = None   # energy: int8 [B, L]
    wt: np.ndarray | None = None     # mutant: int8 [L]
    n_chains: int = 0                # sample
    sweeps: int = 0                  # sample
    seed: int = 0                    # sample
    # filled by the server
    result: np.ndarray | None = None
    t_admit: float = math.nan
    t_done: float = math.nan
    footprint: int = 0
    refused: str | None = None

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival

    @property
    def items(self) -> int:
        if self.kind == "energy":
            return int(self.seqs.shape[0])
        return 1 if self.kind == "mutant" else int(self.n_chains)


@dataclass
class _Live:
    """An admitted request: its pinned input and output, and its arena slot."""
    req: Request
    host_in: torch.Tensor | None = None
    host_out: torch.Tensor | None = None
    off: int = -1          # first arena item (sampling: while in the arena)
    done_sweeps: int = 0
    base: int = 0          # sampling: stream-record sweep offset (mod 2^64)


@dataclass
class Stats:
    peak_bytes: int = 0
    arena_bytes: int = 0
    launches: dict = field(default_factory=lambda: {k: 0 for k in KINDS})  # graph replays
    batched: dict = field(default_factory=lambda: {k: 0 for k in KINDS})   # request-launches
    eager: dict = field(default_factory=lambda: {k: 0 for k in KINDS})     # launches outside graphs


class _Engine:
    """Arena, work table and captured graph of one (kind, model)."""

    def __init__(self, kind, h, J, cap, stream, chunk, cus, device):
        self.kind, self.h, self.J, self.cap, self.stream = kind, h, J, int(cap), stream
        L, q = api._model(h, J)
        self.L, self.q, self.chunk = L, q, chunk
        dev = device
        self.n_live = torch.zeros(1, dtype=torch.int64, device=dev)
        self.n_host = torch.zeros(1, dtype=torch.int64, pin_memory=True)
        self.pending: list[_Live] = []   # admitted, waiting for the next replay
        self.flight: list[_Live] = []    # in the replay in flight (sampling: the live set)
        self.event = None
        self.busy = False
        if kind == "energy":
            self.inp = torch.zeros((cap, L), dtype=torch.int8, device=dev)
            self.out = torch.zeros(cap, dtype=torch.float32, device=dev)
            self.ws = api.workspace(B.WS_ENERGY, cap, L, q, 0, dev)
            call = lambda: api.energy_batch(h, J, self.inp, self.n_live, self.out, self.ws)
        elif kind == "mutant":
            self.inp = torch.zeros((cap, L), dtype=torch.int8, device=dev)
            self.out = torch.zeros((cap, L * q), dtype=torch.float32, device=dev)
            self.ws = api.workspace(B.WS_MUTANT, cap, L, q, 0, dev)
            call = lambda: api.mutant_scan_batch(h, J, self.inp, self.n_live, self.out, self.ws)
        else:
            self.inp = torch.zeros((cap, L), dtype=torch.int8, device=dev)
            self.scratch = torch.zeros((cap, L), dtype=torch.int8, device=dev)
            self.table = torch.zeros(24 * cap, dtype=torch.uint8, device=dev)
            self.rec_host = np.zeros(cap, dtype=[("seed", "<u8"), ("sweep_offset", "<u8"),
                                                 ("chain", "<u4"), ("reserved", "<u4")])
            self.table_host = torch.zeros(24 * cap, dtype=torch.uint8, pin_memory=True)
            self.tick = torch.zeros(1, dtype=torch.int64, device=dev)
            self.ticks = 0  # host mirror of the device tick
            self.ws = api.workspace(B.WS_GIBBS, cap, L, q, B.SAMPLER_GATHER, dev)
            self.dirty = 0  # first table record that changed since the last upload
            with torch.cuda.stream(stream):
                # lay the couplings out once; the graphs then only sweep
                api.gibbs(h, J, self.inp[:1], 0, 0, H_ws=self.ws, sampler="gather")
            # one graph per capacity bucket (powers of two up to cap): a tick
            # replays the smallest bucket that holds the live chains, so the
            # launch shape (chains per workgroup) follows the live count
            self.buckets = []
            b = min(256, cap)
            while True:  # ratio sqrt(2): at most ~1.4x the live chains per launch
                self.buckets.append(b)
                if b >= cap:
                    break
                b = min(max(b + 1, int(b * 1.4142)), cap)
            self.graphs = {}
            for b in self.buckets:
                call = (lambda b=b: api.sample_tick(
                    h, J, self.inp[:b], self.n_live, chunk, self.table[:24 * b], self.tick,
                    self.ws, keep_layout=True, cus=cus))
                self.graphs[b] = self._capture(call, stream)
            self.tick.zero_()
            torch.cuda.synchronize()
            return
        self.graph = self._capture(call, stream)

    @staticmethod
    def _capture(call, stream):
        """One eager call (kernel loading, attributes), then the capture."""
        stream.synchronize()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            call()
        stream.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream, capture_error_mode="thread_local"):
            call()
        torch.cuda.synchronize()
        return g

    def sample_graph(self, n: int):
        """The graph of the smallest capacity bucket that holds n live chains."""
        for b in self.buckets:
            if n <= b:
                return self.graphs[b]
        raise ValueError(f"{n} live chains exceed the arena of {self.cap}")

    def item_bytes(self) -> int:
        """Device bytes per arena item (the footprint unit of admission)."""
        L, q = self.L, self.q
        if self.kind == "energy":
            return L + 4 + api.workspace_bytes(B.WS_ENERGY, 64, L, q, 0) // 64
        if self.kind == "mutant":
            return L + 8 * L * q
        return 2 * L + 24

    def arena_bytes(self) -> int:
        tot = self.inp.numel() + self.ws.numel() * self.ws.element_size() + 16
        if self.kind in ("energy", "mutant"):
            tot += self.out.numel() * 4
        else:
            tot += self.scratch.numel() + self.table.numel()
        return tot

    def used(self) -> int:
        """Arena items held by admitted requests; finished sampling requests
        leave at the next tick's compaction, before any joiner is placed."""
        return sum(lv.req.items for lv in self.pending + self.flight
                   if lv.req.kind != "sample" or lv.done_sweeps < lv.req.sweeps)


class Server:
    def reset_stats(self) -> None:
        """Fresh counters for a new run on the same engines."""
        arena = self.stats.arena_bytes
        self.stats = Stats()
        self.stats.arena_bytes = arena

    def __init__(self, models, budget_bytes: int, lanes: int = 4, chunk_sweeps: int = 1,
                 sample_cus: int = 0, caps=None, device="cuda"):
        """models: list of (h float32 [L, q], J float32 [Lq, Lq]) device tensors.
        Arenas of `caps` items per kind and model (scaled down to fit
        `budget_bytes` in total); sample_cus: compute units a sampling tick
        is sized for (0: all)."""
        self.models = []
        for h, J in models:
            L, q = api._model(h, J)
            self.models.append((h, J, L, q))
        self.budget = int(budget_bytes)
        self.chunk = int(chunk_sweeps)
        self.device = device
        self.lanes = [torch.cuda.Stream(device=device) for _ in range(lanes)]
        self.stats = Stats()
        caps = dict(DEFAULT_CAPS, **(caps or {}))
        # arena capacities: the requested ones, scaled down until every
        # arena (inputs, outputs, workspace, work table) fits the budget
        scale = 1.0
        while True:
            plan = {(k, m): self._cap(k, caps[k] * scale) for m in range(len(self.models))
                    for k in KINDS}
            total = sum(self._arena_bytes(k, m, c) for (k, m), c in plan.items())
            if total <= self.budget or scale < 1e-4:
                break
            scale *= 0.9
        self.engines = {}
        for (k, m), cap in plan.items():
            h, J = self.models[m][:2]
            s = self.lanes[self.lane_of(k, m)]
            self.engines[(k, m)] = _Engine(k, h, J, cap, s, self.chunk, sample_cus, device)
        self.stats.arena_bytes = sum(e.arena_bytes() for e in self.engines.values())

    def lane_of(self, kind: str, model: int) -> int:
        """Sampling engines and scoring engines use disjoint lanes (with two or
        more), so a scoring batch never queues behind a sampling tick in
        stream order."""
        n = len(self.lanes)
        if n == 1:
            return 0
        ns = n // 2  # lanes for sampling ticks
        if kind == "sample":
            return model % ns
        return ns + (model + (n - ns) // 2 * (kind == "mutant")) % (n - ns)

    @staticmethod
    def _cap(kind: str, c: float) -> int:
        c = max(1, int(c))
        return max(64, c // 64 * 64) if kind == "energy" else c

    def _arena_bytes(self, kind: str, m: int, cap: int) -> int:
        """Device bytes of one engine's arena (as _Engine allocates it)."""
        L, q = self.models[m][2:]
        if kind == "energy":
            return cap * L + 4 * cap + api.workspace_bytes(B.WS_ENERGY, cap, L, q, 0) + 16
        if kind == "mutant":
            return cap * L + 4 * cap * L * q + api.workspace_bytes(B.WS_MUTANT, cap, L, q, 0) + 16
        return (2 * cap * L + 24 * cap + 16 +
                api.workspace_bytes(B.WS_GIBBS, cap, L, q, B.SAMPLER_GATHER))

    # ------------------------------------------------------------ footprints
    def footprint(self, r: Request) -> int:
        return r.items * self.engines[(r.kind, r.model)].item_bytes()

    def fits_ever(self, r: Request) -> bool:
        return r.items <= self.engines[(r.kind, r.model)].cap

    # ------------------------------------------------------------ launches
    def _launch_scores(self, e: _Engine) -> None:
        """Energies or mutant scans: the admitted requests that fit, in
        arrival order, packed into the arena, one graph replay."""
        batch, n = [], 0
        while e.pending and n + e.pending[0].req.items <= e.cap:
            lv = e.pending.pop(0)
            lv.off = n
            n += lv.req.items
            batch.append(lv)
        if not batch:
            return
        with torch.cuda.stream(e.stream):
            for lv in batch:
                k = lv.req.items
                e.inp[lv.off:lv.off + k].copy_(lv.host_in.view(k, e.L), non_blocking=True)
            e.n_host[0] = n
            e.n_live.copy_(e.n_host, non_blocking=True)
            e.graph.replay()
            for lv in batch:
                k = lv.req.items
                shape = (k,) if e.kind == "energy" else (e.L * e.q,)
                lv.host_out = torch.empty(shape, dtype=torch.float32, pin_memory=True)
                src = e.out[lv.off:lv.off + k]
                lv.host_out.copy_(src if e.kind == "energy" else src[0], non_blocking=True)
            e.event = torch.cuda.Event()
            e.event.record(e.stream)
        e.flight = batch
        e.busy = True
        self.stats.launches[e.kind] += 1
        self.stats.batched[e.kind] += len(batch)

    def _launch_tick(self, e: _Engine) -> None:
        """One sampling tick over every live chain of the model: compaction of
        the requests that left, new requests joined at the end, the work
        table's changed records and the live count uploaded, one replay."""
        L, q, chunk = e.L, e.q, self.chunk
        with torch.cuda.stream(e.stream):
            # compaction: requests that finished in the previous tick left holes
            live = [lv for lv in e.flight if lv.done_sweeps < lv.req.sweeps]
            n = 0
            moved = None
            for lv in live:
                k = lv.req.items
                if lv.off != n:
                    e.scratch[n:n + k].copy_(e.inp[lv.off:lv.off + k], non_blocking=True)
                    moved = n if moved is None else moved
                    lv.off = n
                    self._records(e, lv)
                elif moved is not None:
                    e.scratch[n:n + k].copy_(e.inp[n:n + k], non_blocking=True)
                n += k
            if moved is not None:
                e.inp[moved:n].copy_(e.scratch[moved:n], non_blocking=True)
                e.dirty = min(e.dirty, moved)
            # new requests join at this tick: their first sweep is sweep 0
            while e.pending and n + e.pending[0].req.items <= e.cap:
                lv = e.pending.pop(0)
                k = lv.req.items
                lv.off = n
                lv.base = (-e.ticks * chunk) % (1 << 64)
                api.init_chains(k, L, q, lv.req.seed, out=e.inp[n:n + k])
                self.stats.eager["sample"] += 1
                self._records(e, lv)
                e.dirty = min(e.dirty, n)
                live.append(lv)
                n += k
            if not live:
                e.flight = []
                return
            if e.dirty < n:
                a, b = 24 * e.dirty, 24 * n
                e.table_host.numpy()[a:b] = e.rec_host[e.dirty:n].view(np.uint8)
                e.table[a:b].copy_(e.table_host[a:b], non_blocking=True)
            e.dirty = e.cap
            e.n_host[0] = n
            e.n_live.copy_(e.n_host, non_blocking=True)
            e.sample_graph(n).replay()
            e.ticks += 1
            for lv in live:
                lv.done_sweeps += chunk
                if lv.done_sweeps == lv.req.sweeps:
                    k = lv.req.items
                    lv.host_out = torch.empty((k, L), dtype=torch.int8, pin_memory=True)
                    lv.host_out.copy_(e.inp[lv.off:lv.off + k], non_blocking=True)
            e.event = torch.cuda.Event()
            e.event.record(e.stream)
        e.flight = live
        e.busy = True
        self.stats.launches["sample"] += 1
        self.stats.batched["sample"] += len(live)

    @staticmethod
    def _records(e: _Engine, lv: _Live) -> None:
        k, o = lv.req.items, lv.off
        rec = e.rec_host[o:o + k]
        rec["seed"] = lv.req.seed
        rec["sweep_offset"] = lv.base
        rec["chain"] = np.arange(k, dtype=np.uint32)
        rec["reserved"] = 0

    # ------------------------------------------------------------ main loop
    def run(self, requests, realtime: bool = True, idle_sleep: float = 20e-6, progress=None,
            every: float = 15.0):
        """Serves `requests` (sorted by arrival).  With realtime=False every
        request counts as arrived at once (throughput mode).  progress(done,
        total), if given, is called every `every` seconds."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in reqs:
            if r.kind == "sample" and r.sweeps % self.chunk:
                raise ValueError(f"request {r.rid}: sweeps {r.sweeps} not a multiple of the "
                                 f"tick's {self.chunk}")
        waiting: list[Request] = []
        in_use = 0
        nxt = 0
        live_count = 0
        t0 = time.perf_counter()

        def clock():
            return time.perf_counter() - t0

        t_report = every
        while nxt < len(reqs) or waiting or live_count:
            now = clock()
            if progress is not None and now >= t_report:
                progress(sum(r.t_done == r.t_done for r in reqs), len(reqs))
                t_report = now + every
            while nxt < len(reqs) and (not realtime or reqs[nxt].arrival <= now):
                r = reqs[nxt]
                nxt += 1
                if not realtime:
                    r.arrival = now
                r.footprint = self.footprint(r)
                if not self.fits_ever(r):
                    e = self.engines[(r.kind, r.model)]
                    r.refused = (f"{r.items} items, the {r.kind} arena of model {r.model} "
                                 f"holds {e.cap}")
                    r.t_done = now
                    continue
                waiting.append(r)
            # admission in arrival order per engine: a request waits only for
            # room in its own arena (no head-of-line blocking across engines)
            full = set()
            still = []
            for r in waiting:
                key = (r.kind, r.model)
                e = self.engines[key]
                if key in full or e.used() + r.items > e.cap:
                    full.add(key)
                    still.append(r)
                    continue
                lv = _Live(r)
                if r.kind != "sample":
                    x = r.seqs if r.kind == "energy" else r.wt[None]
                    lv.host_in = torch.from_numpy(
                        np.ascontiguousarray(x, dtype=np.int8).reshape(-1)).pin_memory()
                r.t_admit = now
                e.pending.append(lv)
                live_count += 1
                in_use += r.footprint
                self.stats.peak_bytes = max(self.stats.peak_bytes, in_use)
            waiting = still
            # one replay per free engine with work
            for e in self.engines.values():
                if e.busy:
                    continue
                if e.kind == "sample":
                    if e.pending or e.flight:
                        self._launch_tick(e)
                elif e.pending:
                    self._launch_scores(e)
            # completions
            progressed = False
            for e in self.engines.values():
                if not e.busy or not e.event.query():
                    continue
                progressed = True
                e.busy = False
                t = clock()
                for lv in e.flight:
                    r = lv.req
                    if r.kind == "sample" and lv.done_sweeps < r.sweeps:
                        continue  # next tick
                    r.result = lv.host_out.numpy()
                    r.t_done = t
                    lv.host_in = None
                    live_count -= 1
                    in_use -= r.footprint
                if e.kind != "sample":
                    e.flight = []
            if not progressed and idle_sleep > 0:
                time.sleep(idle_sleep)
        return reqs


# ---------------------------------------------------------------- workloads
def resident_models(Ls=(64, 128, 200, 256, 320, 400, 450, 512), q: int = 21, seed: int = 5000,
                    device="cuda"):
    """Stand-ins for trained models: planted Potts parameters of each size."""
    from . import synth
    out = []
    for k, L in enumerate(Ls):
        h, J = synth.planted_dense(L, q, seed=seed + k, sigma_J=0.05)
        out.append((torch.from_numpy(h).to(device), torch.from_numpy(J).to(device)))
    return out


def poisson_requests(n: int, rate: float, Ls, q: int, seed: int, mix=(0.4, 0.4, 0.2),
                     energy_range=(1000, 100000), chain_range=(100, 10000), sweeps: int = 50):
    """n requests with exponential inter-arrival times (mean 1/rate seconds),
    kinds drawn with probabilities `mix`, the model uniformly, energy batch
    sizes and chain counts log-uniform over their ranges, uniform random
    sequences and wild types."""
    g = np.random.default_rng(seed)
    t = np.cumsum(g.exponential(1.0 / rate, size=n))
    out = []
    for k in range(n):
        kind = KINDS[int(g.choice(3, p=np.asarray(mix) / np.sum(mix)))]
        m = int(g.integers(len(Ls)))
        L = Ls[m]
        r = Request(k, kind, m, float(t[k]))
        if kind == "energy":
            b = int(round(math.exp(g.uniform(math.log(energy_range[0]), math.log(energy_range[1])))))
            r.seqs = g.integers(0, q, size=(b, L), dtype=np.int8)
        elif kind == "mutant":
            r.wt = g.integers(0, q, size=L, dtype=np.int8)
        else:
            r.n_chains = int(round(math.exp(g.uniform(math.log(chain_range[0]),
                                                      math.log(chain_range[1])))))
            r.sweeps = sweeps
            r.seed = int(g.integers(1, 2**62))
        out.append(r)
    return out


def summarize(reqs):
    """p50/p99 latency (ms) per kind over served requests, and the request rate."""
    res = {}
    served = [r for r in reqs if r.refused is None]
    for kind in KINDS:
        lat = np.array([r.latency for r in served if r.kind == kind]) * 1e3
        if lat.size:
            res[kind] = {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50)),
                         "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean())}
    if served:
        span = max(r.t_done for r in served) - min(r.arrival for r in served)
        res["requests_per_s"] = len(served) / span if span > 0 else float("inf")
    res["refused"] = sum(r.refused is not None for r in reqs)
    return res
