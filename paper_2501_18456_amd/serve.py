"""Request loop over resident trained models (scoring, mutant scans, sampling).

Uses of a trained Potts model from Sec. 4 of the paper (energies of a sequence
set, the single-mutant library, sampling) served to a stream of requests:

  - models stay resident in HBM (h, J as float32);
  - admission by HBM footprint: a request is admitted, in arrival order, once
    the memory its inputs, outputs and workspace need fits the budget beside
    everything in flight; a request that can never fit is refused at once;
  - continuous batching (iteration-level): each (kind, model) pair has at most
    one launch in flight; when it is free, everything of that pair that is
    ready goes out as one launch -- the admitted energy requests of the model
    as one bmdca_energy call, its mutant scans as one
    bmdca_single_mutant_scan call, and its sampling requests as one
    bmdca_gibbs_streams call over all their chains for the next
    `chunk_sweeps` sweeps (each chain keeps its own request's key, chain
    index and sweep count).  Requests that arrive while a launch runs join
    the next one, at the next chunk boundary for sampling;
  - launches go to `lanes` streams (default priority) and overlap on the GPU;
    every (kind, model) pair has a fixed lane, so a batch never waits on
    another lane's work; completion is seen by polling events, results are
    copied back on the lane that made them.

A request's result does not depend on what else is in flight: energies of a
sequence are independent of the batch (fixed pair order per L), mutant scans
are per wild type, and chunked sampling uses the counter-based draws of the
whole request.  Every computation runs in the HIP library; this module only
moves data and decides what to launch when.
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


@dataclass
class _Live:
    """An admitted request and its device buffers."""
    req: Request
    lane: int
    inp: torch.Tensor | None = None       # device input (sequences, wild type, chains)
    host_in: torch.Tensor | None = None   # pinned input, alive until uploaded
    host_out: torch.Tensor | None = None  # pinned result
    dev_out: torch.Tensor | None = None   # device result, alive until copied
    done_sweeps: int = 0
    busy: bool = False


@dataclass
class _Launch:
    event: torch.cuda.Event
    lives: list
    kind: str
    model: int


@dataclass
class Stats:
    peak_bytes: int = 0
    launches: dict = field(default_factory=lambda: {k: 0 for k in KINDS})
    batched: dict = field(default_factory=lambda: {k: 0 for k in KINDS})


class Server:
    def __init__(self, models, budget_bytes: int, lanes: int = 4, chunk_sweeps: int = 5,
                 sample_cus: int = 0, device="cuda"):
        """models: list of (h float32 [L, q], J float32 [Lq, Lq]) device tensors.
        sample_cus: compute units a sampling launch is sized for (0: all)."""
        self.models = []
        for h, J in models:
            L, q = api._model(h, J)
            self.models.append((h, J, L, q))
        self.budget = int(budget_bytes)
        self.chunk = int(chunk_sweeps)
        self.sample_cus = int(sample_cus)
        self.device = device
        self.lanes = [torch.cuda.Stream(device=device) for _ in range(lanes)]
        self.stats = Stats()

    # ------------------------------------------------------------ footprints
    def footprint(self, r: Request) -> int:
        h, J, L, q = self.models[r.model]
        if r.kind == "energy":
            n = r.seqs.shape[0]
            return n * L + 4 * n + api.workspace_bytes(B.WS_ENERGY, n, L, q, 0)
        if r.kind == "mutant":
            return L + 4 * L * q + api.workspace_bytes(B.WS_MUTANT, 1, L, q, 0)
        if r.kind == "sample":
            return r.n_chains * L + api.workspace_bytes(B.WS_GIBBS, r.n_chains, L, q,
                                                       B.SAMPLER_GATHER if L <= 512 else 0)
        raise ValueError(f"unknown request kind {r.kind}")

    # ------------------------------------------------------------ admission
    def lane_of(self, kind: str, model: int) -> int:
        return (len(KINDS) * model + KINDS.index(kind)) % len(self.lanes)

    def _admit(self, r: Request, now: float) -> _Live:
        h, J, L, q = self.models[r.model]
        lane = self.lane_of(r.kind, r.model)
        lv = _Live(r, lane)
        s = self.lanes[lane]
        with torch.cuda.stream(s):
            if r.kind in ("energy", "mutant"):
                x = r.seqs if r.kind == "energy" else r.wt[None]
                lv.host_in = torch.from_numpy(np.ascontiguousarray(x, dtype=np.int8)).pin_memory()
                lv.inp = lv.host_in.to(self.device, non_blocking=True)
            else:
                lv.inp = api.init_chains(r.n_chains, L, q, r.seed, device=self.device)
        r.t_admit = now
        return lv

    # ------------------------------------------------------------ launches
    def _launch_group(self, kind: str, model: int, lives: list) -> _Launch:
        """One batched launch for several admitted requests of one model."""
        h, J, L, q = self.models[model]
        s = self.lanes[lives[0].lane]  # the lane of (kind, model): inputs were uploaded there
        with torch.cuda.stream(s):
            if kind == "energy":
                seqs = lives[0].inp if len(lives) == 1 else torch.cat([lv.inp for lv in lives])
                n = seqs.shape[0]
                ws = api.workspace(B.WS_ENERGY, n, L, q, 0, self.device)
                out = api.energy(h, J, seqs, ws=ws)
                o = 0
                for lv in lives:
                    k = lv.inp.shape[0]
                    lv.host_out = torch.empty(k, dtype=torch.float32, pin_memory=True)
                    lv.host_out.copy_(out[o:o + k], non_blocking=True)
                    o += k
            else:
                wts = lives[0].inp if len(lives) == 1 else torch.cat([lv.inp for lv in lives])
                out = api.single_mutant_scan(h, J, wts)
                for k, lv in enumerate(lives):
                    lv.host_out = torch.empty((L * q,), dtype=torch.float32, pin_memory=True)
                    lv.host_out.copy_(out[k], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        for lv in lives:
            lv.busy = True
            lv.dev_out = out
        self.stats.launches[kind] += 1
        self.stats.batched[kind] += len(lives)
        return _Launch(ev, lives, kind, model)

    def _launch_samples(self, model: int, lives: list) -> _Launch:
        """The next chunk of every listed sampling request of one model, as one
        launch over all their chains."""
        h, J, L, q = self.models[model]
        s = self.lanes[lives[0].lane]  # the lane of (sample, model)
        n = min(self.chunk, min(lv.req.sweeps - lv.done_sweeps for lv in lives))
        counts = [lv.req.n_chains for lv in lives]
        seeds = np.concatenate([np.full(k, lv.req.seed, dtype=np.uint64)
                                for k, lv in zip(counts, lives)])
        offs = np.concatenate([np.full(k, lv.done_sweeps, dtype=np.uint64)
                               for k, lv in zip(counts, lives)])
        ids = np.concatenate([np.arange(k, dtype=np.uint32) for k in counts])
        sampler = "gather" if L <= 512 else "fields"
        with torch.cuda.stream(s):
            chains = lives[0].inp if len(lives) == 1 else torch.cat([lv.inp for lv in lives])
            table = api.chain_streams(seeds, offs, ids, self.device)
            api.gibbs_streams(h, J, chains, n, table, sampler=sampler, cus=self.sample_cus)
            o = 0
            for k, lv in zip(counts, lives):
                if len(lives) > 1:
                    lv.inp.copy_(chains[o:o + k])
                o += k
                lv.done_sweeps += n
                if lv.done_sweeps == lv.req.sweeps:
                    lv.host_out = torch.empty(tuple(lv.inp.shape), dtype=torch.int8,
                                              pin_memory=True)
                    lv.host_out.copy_(lv.inp, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        for lv in lives:
            lv.busy = True
        self.stats.launches["sample"] += 1
        self.stats.batched["sample"] += len(lives)
        return _Launch(ev, lives, "sample", model)

    # ------------------------------------------------------------ main loop
    def run(self, requests, realtime: bool = True, idle_sleep: float = 20e-6):
        """Serves `requests` (sorted by arrival).  With realtime=False every
        request counts as arrived at once (throughput mode)."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        waiting: list[Request] = []
        ready: list[_Live] = []      # admitted, not in flight
        inflight: list[_Launch] = []
        in_use = 0
        nxt = 0
        t0 = time.perf_counter()

        def clock():
            return time.perf_counter() - t0

        while nxt < len(reqs) or waiting or ready or inflight:
            now = clock()
            while nxt < len(reqs) and (not realtime or reqs[nxt].arrival <= now):
                r = reqs[nxt]
                nxt += 1
                if not realtime:
                    r.arrival = now
                r.footprint = self.footprint(r)
                if r.footprint > self.budget:
                    r.refused = f"needs {r.footprint} bytes, budget {self.budget}"
                    r.t_done = now
                    continue
                waiting.append(r)
            # admission in arrival order while the head fits
            while waiting and in_use + waiting[0].footprint <= self.budget:
                r = waiting.pop(0)
                ready.append(self._admit(r, now))
                in_use += r.footprint
                self.stats.peak_bytes = max(self.stats.peak_bytes, in_use)
            # batched launches of everything ready
            groups: dict = {}
            busy_keys = {(ln.kind, ln.model) for ln in inflight}
            for lv in ready:
                key = (lv.req.kind, lv.req.model)
                if not lv.busy and key not in busy_keys:
                    groups.setdefault(key, []).append(lv)
            for (kind, model), lives in groups.items():
                if kind == "sample":
                    inflight.append(self._launch_samples(model, lives))
                else:
                    inflight.append(self._launch_group(kind, model, lives))
            # completions
            progressed = False
            still = []
            for ln in inflight:
                if not ln.event.query():
                    still.append(ln)
                    continue
                progressed = True
                t = clock()
                for lv in ln.lives:
                    lv.busy = False
                    r = lv.req
                    if ln.kind == "sample" and lv.done_sweeps < r.sweeps:
                        continue  # next chunk at the next tick
                    r.result = lv.host_out.numpy()
                    r.t_done = t
                    lv.dev_out = lv.host_in = None
                    ready.remove(lv)
                    in_use -= r.footprint
            inflight = still
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
