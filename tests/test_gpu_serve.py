"""Serving loop: every request's result is bit-identical to the same call made
alone (energies, mutant scans, sampling in ticks), batching really merges
requests into one replay of each engine's captured graph, and admission
respects the arenas sized from the HBM budget."""
import numpy as np
import pytest
import torch

from paper_2501_18456_amd import api, serve

pytestmark = pytest.mark.gpu

LS, Q = (40, 77, 130), 21


@pytest.fixture(scope="module")
def models():
    ms = serve.resident_models(LS, Q, seed=6000)
    torch.cuda.synchronize()
    return ms


def alone(models, r):
    h, J = models[r.model]
    q = h.shape[1]
    if r.kind == "energy":
        out = api.energy(h, J, torch.from_numpy(r.seqs).cuda())
    elif r.kind == "mutant":
        out = api.single_mutant_scan(h, J, torch.from_numpy(r.wt[None]).cuda())[0]
    else:
        L = h.shape[0]
        ch = api.init_chains(r.n_chains, L, q, r.seed)
        out = api.gibbs(h, J, ch, r.sweeps, r.seed, sampler="gather")
    torch.cuda.synchronize()
    return out.cpu().numpy()


def requests(n, seed, rate=5000.0, Ls=LS, q=Q):
    return serve.poisson_requests(n, rate, Ls, q, seed, energy_range=(50, 3000),
                                  chain_range=(10, 300), sweeps=12)


@pytest.mark.parametrize("realtime", [False, True])
def test_results_same_alone_and_in_mix(models, realtime):
    srv = serve.Server(models, budget_bytes=8 << 30, lanes=3, chunk_sweeps=4,
                       caps={"energy": 20000, "sample": 4096})
    reqs = srv.run(requests(36, 61 + realtime), realtime=realtime)
    assert all(r.refused is None and r.result is not None for r in reqs)
    for r in reqs:
        ref = alone(models, r)
        assert r.result.shape == ref.shape
        assert np.array_equal(r.result, ref), f"request {r.rid} ({r.kind}) differs from alone"
    # sampling in ticks of 4 sweeps: 12 sweeps -> 3 ticks a request
    n_sample = sum(r.kind == "sample" for r in reqs)
    assert srv.stats.batched["sample"] == 3 * n_sample
    assert srv.stats.eager["sample"] == n_sample  # one chain initialisation each
    if not realtime:  # all arrived at once: requests of one model share replays
        for kind in serve.KINDS:
            assert srv.stats.batched[kind] > srv.stats.launches[kind], kind
    s = serve.summarize(reqs)
    assert s["refused"] == 0 and all(s[k]["p99_ms"] >= s[k]["p50_ms"] for k in serve.KINDS)


def test_rna_like_model_in_mix():
    """q = 5 (16 states fewer than a protein alphabet): merged sampling ticks,
    energies and scans equal their alone calls."""
    ms = serve.resident_models((61, 100), 5, seed=6100)
    srv = serve.Server(ms, budget_bytes=4 << 30, lanes=2, chunk_sweeps=3,
                       caps={"energy": 8192, "sample": 8192})
    reqs = serve.poisson_requests(18, 1e6, (61, 100), 5, 63, energy_range=(50, 2000),
                                  chain_range=(500, 3000), sweeps=9)
    out = srv.run(reqs, realtime=False)
    assert all(r.result is not None for r in out)
    for r in out:
        assert np.array_equal(r.result, alone(ms, r)), f"request {r.rid} ({r.kind})"


def test_admission_follows_the_arenas(models):
    """Arenas sized from the budget; a request larger than its arena is
    refused at once, the others wait for room and are all served correctly."""
    caps = {"energy": 4096, "mutant": 2, "sample": 1024}
    srv = serve.Server(models, budget_bytes=8 << 30, lanes=2, chunk_sweeps=4, caps=caps)
    assert srv.stats.arena_bytes <= 8 << 30
    assert srv.engines[("energy", 2)].cap == 4096
    reqs = requests(24, 71, rate=1e6)
    big_e = serve.Request(998, "energy", 2, 0.0, seqs=np.zeros((5000, LS[2]), dtype=np.int8))
    big_s = serve.Request(999, "sample", 1, 0.0, n_chains=1500, sweeps=12, seed=5)
    out = srv.run(reqs + [big_e, big_s], realtime=False)
    assert big_e.refused is not None and big_e.result is None
    assert big_s.refused is not None and big_s.result is None
    served = [r for r in out if r.rid < 998]
    assert all(r.refused is None and r.result is not None for r in served)
    for e in srv.engines.values():
        assert e.used() == 0
    for r in served[:8]:
        assert np.array_equal(r.result, alone(models, r))


def test_tiny_budget_scales_the_arenas(models):
    """A budget below the default arenas scales every arena down to fit."""
    srv = serve.Server(models, budget_bytes=100 << 20, lanes=1, chunk_sweeps=4)
    assert srv.stats.arena_bytes <= 100 << 20
    assert srv.engines[("energy", 0)].cap < serve.DEFAULT_CAPS["energy"]
