"""Grouped training: several models of uneven L, q and N in one enqueued (or
graph-replayed) epoch give, model by model, the same bits as their own
bmdca_train_step calls; the device control record advances the epoch, stops a
model at its Pearson target, and an inactive model is left untouched."""
import numpy as np
import pytest
import torch

from paper_2501_18456_amd import api, synth

pytestmark = pytest.mark.gpu

# (L, q, N, prec, sampler): both samplers, both count products, ragged tiles
SHAPES = [(12, 21, 300, "bf16x2", "auto"), (30, 5, 500, "bf16x2", "auto"),
          (9, 21, 128, "fp32", "fields"), (50, 21, 700, "bf16x2", "gather"),
          (7, 3, 200, "fp32", "auto"), (140, 21, 256, "bf16x2", "auto")]
LR, SWEEPS, EPOCHS = 0.05, 4, 3


def problem(k):
    L, q, N, prec, sampler = SHAPES[k]
    h, J = synth.planted_dense(L, q, seed=700 + k, sigma_J=0.1)
    hg, Jg = torch.from_numpy(h).cuda(), torch.from_numpy(J).cuda()
    msa = api.init_chains(400, L, q, seed=800 + k)
    api.gibbs(hg, Jg, msa, 20, 800 + k)
    f1, f2, _ = api.stats(msa, q, None, -1.0, "fp32")
    h0 = torch.log(f1).float().reshape(L, q).contiguous()
    J0 = torch.zeros((L * q, L * q), dtype=torch.float32, device="cuda")
    ch = api.init_chains(N, L, q, seed=900 + k)
    return dict(h=h0, J=J0, chains=ch, f1=f1, f2=f2, seed=900 + k, prec=prec, sampler=sampler)


@pytest.fixture(scope="module")
def problems():
    ps = [problem(k) for k in range(len(SHAPES))]
    torch.cuda.synchronize()
    return ps


def clone(p):
    return {k: (v.clone() if isinstance(v, torch.Tensor) else v) for k, v in p.items()}


def solo_run(p, epochs):
    p = clone(p)
    rs = []
    for e in range(epochs):
        r = api.train_step(p["h"], p["J"], p["chains"], p["f1"], p["f2"], LR, SWEEPS, p["seed"], e,
                           p["prec"], sampler=p["sampler"])
        rs.append(r.clone())
    torch.cuda.synchronize()
    return p, [float(r.item()) for r in rs]


def models_of(ps, targets=None):
    out = []
    for k, p in enumerate(ps):
        p = clone(p)
        out.append(api.TrainModel(p["h"], p["J"], p["chains"], p["f1"], p["f2"], LR, SWEEPS,
                                  p["seed"], p["prec"], p["sampler"],
                                  target_pearson=(targets[k] if targets else 0.0)))
    return out


def same(m, p):
    return (torch.equal(m.h, p["h"]) and torch.equal(m.J, p["J"])
            and torch.equal(m.chains, p["chains"]))


@pytest.fixture(scope="module")
def solo(problems):
    return [solo_run(p, EPOCHS) for p in problems]


@pytest.mark.parametrize("lanes", [1, 4])
def test_group_step_equals_solo(problems, solo, lanes):
    ms = models_of(problems)
    rs = [[] for _ in ms]
    for e in range(EPOCHS):
        api.train_group_step(ms, lanes=lanes)
        for k, m in enumerate(ms):
            rs[k].append(m.pearson.clone())
    torch.cuda.synchronize()
    for k, m in enumerate(ms):
        ps, rsolo = solo[k]
        assert same(m, ps), f"model {k} {SHAPES[k]} differs from its solo run"
        assert [float(r.item()) for r in rs[k]] == rsolo
        c = api.read_ctl(m.ctl)
        assert c["epoch"] == EPOCHS and c["active"] and c["converged_at"] == -1


def test_group_graph_replay_equals_solo(problems, solo):
    ms = models_of(problems)
    g = api.TrainGroupGraph(ms, lanes=4)
    torch.cuda.synchronize()
    rs = [[] for _ in ms]
    for e in range(EPOCHS):
        g.launch()
        torch.cuda.synchronize()  # eager host work between replays
        for k, m in enumerate(ms):
            rs[k].append(float(m.pearson.item()))
    g.close()
    for k, m in enumerate(ms):
        ps, rsolo = solo[k]
        assert same(m, ps), f"model {k} {SHAPES[k]} differs after graph replays"
        assert rs[k] == rsolo
        assert api.read_ctl(m.ctl)["epoch"] == EPOCHS


def test_inactive_model_is_untouched(problems, solo):
    ms = models_of(problems)
    api.train_group_step(ms, lanes=4)
    torch.cuda.synchronize()
    frozen = dict(h=ms[1].h.clone(), J=ms[1].J.clone(), chains=ms[1].chains.clone())
    ms[1].ctl.copy_(api.train_ctl("cuda", epoch=1, active=False))
    for _ in range(EPOCHS - 1):
        api.train_group_step(ms, lanes=4)
    torch.cuda.synchronize()
    assert torch.equal(ms[1].h, frozen["h"]) and torch.equal(ms[1].J, frozen["J"])
    assert torch.equal(ms[1].chains, frozen["chains"])
    assert api.read_ctl(ms[1].ctl)["epoch"] == 1
    ps, _ = solo[0]
    assert same(ms[0], ps)  # the others ran all epochs as before


def test_pearson_target_stops_a_model(problems, solo):
    # target = the Pearson value model 2 reaches after its first epoch
    r1 = solo[2][1][0]
    targets = [0.0] * len(problems)
    targets[2] = r1
    ms = models_of(problems, targets)
    g = api.TrainGroupGraph(ms, lanes=2)
    after1 = None
    for e in range(EPOCHS):
        g.launch()
        torch.cuda.synchronize()
        if e == 0:
            after1 = (ms[2].h.clone(), ms[2].J.clone(), ms[2].chains.clone())
    g.close()
    c = api.read_ctl(ms[2].ctl)
    assert c["active"] is False and c["converged_at"] == 1 and c["epoch"] == 1
    assert torch.equal(ms[2].h, after1[0]) and torch.equal(ms[2].J, after1[1])
    assert torch.equal(ms[2].chains, after1[2])
    ps, _ = solo[3]
    assert same(ms[3], ps)
