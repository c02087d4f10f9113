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


def test_group_q5_many_chains_equal_solo():
    """RNA-like models (q = 5) with 4096 chains on 8 lanes (a 32-CU share each):
    the share plan takes the lanes per chain of the solo plan (fixed by q and
    the draw), so the grouped epochs equal solo bmdca_train_step calls."""
    ps = []
    for k, L in enumerate((100, 61)):
        h, J = synth.planted_dense(L, 5, seed=720 + k, sigma_J=0.3)
        hg, Jg = torch.from_numpy(h).cuda(), torch.from_numpy(J).cuda()
        msa = api.init_chains(600, L, 5, seed=820 + k)
        api.gibbs(hg, Jg, msa, 20, 820 + k)
        f1, f2, _ = api.stats(msa, 5, None, -1.0, "fp32")
        ps.append(dict(h=torch.log(f1).float().reshape(L, 5).contiguous(),
                       J=torch.zeros((L * 5, L * 5), dtype=torch.float32, device="cuda"),
                       chains=api.init_chains(4096, L, 5, seed=920 + k), f1=f1, f2=f2,
                       seed=920 + k, prec="bf16x2", sampler="auto"))
    torch.cuda.synchronize()
    solo = [solo_run(p, EPOCHS) for p in ps]
    ms = models_of(ps)
    for e in range(EPOCHS):
        api.train_group_step(ms, lanes=8)
    torch.cuda.synchronize()
    for k, m in enumerate(ms):
        assert same(m, solo[k][0]), f"q=5 model {k} differs from its solo run"


def test_group_epochs_follow_the_oracle(problems):
    """Two models of the group (gather form and field form, BF16 and FP32
    counts) against the oracle's train_step, epoch by epoch: chains follow the
    oracle's trajectories (boundary events excused by replay, then both sides
    continue from the oracle's state); h, J bit-exact and Pearson within 1e-12
    after every epoch without a boundary event."""
    from oracle import oracle as O
    from tests.trajectory_check import check_chains

    picks = [0, 2]  # (12, 21, 300, bf16x2, auto -> gather), (9, 21, 128, fp32, fields)
    ms = models_of([problems[k] for k in picks])
    state = []
    for m in ms:
        state.append([m.h.cpu().numpy().copy(), m.J.cpu().numpy().copy(),
                      m.chains.cpu().numpy().copy()])
    f = [(problems[k]["f1"].cpu().numpy(), problems[k]["f2"].cpu().numpy()) for k in picks]
    events = 0
    for e in range(EPOCHS):
        api.train_group_step(ms, lanes=2)
        torch.cuda.synchronize()
        for i, m in enumerate(ms):
            L, q = SHAPES[picks[i]][:2]
            h, J, ch = state[i]
            h2, J2, ch2, r, _, _ = O.train_step(h, J, ch, f[i][0], f[i][1], q, LR, SWEEPS,
                                                problems[picks[i]]["seed"], e)
            g = m.chains.cpu().numpy()
            bad = check_chains(h, J, ch, g, ch2, q, SWEEPS, problems[picks[i]]["seed"],
                               sweep_offset=e * SWEEPS)
            if len(bad):
                events += len(bad)
                m.h.copy_(torch.from_numpy(h2.reshape(m.h.shape)))
                m.J.copy_(torch.from_numpy(J2))
                m.chains.copy_(torch.from_numpy(ch2))
            else:
                assert np.array_equal(m.h.cpu().numpy().reshape(-1), h2.reshape(-1))
                assert np.array_equal(m.J.cpu().numpy(), J2)
                assert abs(float(m.pearson.item()) - r) <= 1e-12
            state[i] = [h2, J2, ch2]
    assert events <= 3
