"""Serving loop: every request's result is bit-identical to the same call made
alone (energies, mutant scans, chunked sampling), batching really merges
requests, and admission never exceeds the HBM budget."""
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
    if r.kind == "energy":
        out = api.energy(h, J, torch.from_numpy(r.seqs).cuda())
    elif r.kind == "mutant":
        out = api.single_mutant_scan(h, J, torch.from_numpy(r.wt[None]).cuda())[0]
    else:
        L = h.shape[0]
        ch = api.init_chains(r.n_chains, L, Q, r.seed)
        out = api.gibbs(h, J, ch, r.sweeps, r.seed, sampler="gather")
    torch.cuda.synchronize()
    return out.cpu().numpy()


def requests(n, seed, rate=5000.0):
    return serve.poisson_requests(n, rate, LS, Q, seed, energy_range=(50, 3000),
                                  chain_range=(10, 300), sweeps=12)


@pytest.mark.parametrize("realtime", [False, True])
def test_results_same_alone_and_in_mix(models, realtime):
    srv = serve.Server(models, budget_bytes=8 << 30, lanes=3, chunk_sweeps=5)
    reqs = srv.run(requests(36, 61 + realtime), realtime=realtime)
    assert all(r.refused is None and r.result is not None for r in reqs)
    for r in reqs:
        ref = alone(models, r)
        assert r.result.shape == ref.shape
        assert np.array_equal(r.result, ref), f"request {r.rid} ({r.kind}) differs from alone"
    # chunked sampling: 12 sweeps in chunks of at most 5 -> at least 3 chunks a request
    n_sample = sum(r.kind == "sample" for r in reqs)
    assert srv.stats.batched["sample"] >= 3 * n_sample
    if not realtime:  # all arrived at once: launches of one model were merged
        for kind in serve.KINDS:
            assert srv.stats.batched[kind] > srv.stats.launches[kind], kind
        assert srv.stats.batched["sample"] == 3 * n_sample
    s = serve.summarize(reqs)
    assert s["refused"] == 0 and all(s[k]["p99_ms"] >= s[k]["p50_ms"] for k in serve.KINDS)


def test_admission_respects_budget(models):
    reqs = requests(20, 71, rate=1e6)
    sizes = sorted(serve.Server(models, 1 << 40).footprint(r) for r in reqs)
    budget = sizes[-1] + sizes[-2] // 2  # the largest fits, never two of the largest
    srv = serve.Server(models, budget_bytes=budget, lanes=2, chunk_sweeps=5)
    big = serve.Request(999, "energy", 2, 0.0,
                        seqs=np.zeros((200000, LS[2]), dtype=np.int8))
    out = srv.run(reqs + [big], realtime=False)
    assert srv.stats.peak_bytes <= budget
    assert big.refused is not None and big.result is None
    served = [r for r in out if r is not big]
    assert all(r.refused is None and r.result is not None for r in served)
    for r in served[:6]:
        assert np.array_equal(r.result, alone(models, r))
