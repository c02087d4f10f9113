"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same
seeded inputs. Sizes span several 128-wide tiles and ragged tails; every
tolerance is stated where it is used.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2501_18456_amd import api, synth
from paper_2501_18456_amd import _lib as B
from tests.trajectory_check import BOUNDARY, check_chains

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def err_flag():
    return torch.zeros(1, dtype=torch.int32, device="cuda")


def onehot(X, q):
    M, L = X.shape
    Y = np.zeros((M, L * q))
    Y[np.arange(M)[:, None], np.arange(L)[None, :] * q + X] = 1.0
    return Y


def check_trajectory(gpu_ch, orc_ch, margins, sweep_index=0):
    """Chains that differ must have differed first at a visit whose oracle
    margin is below BOUNDARY (single-sweep calls). Returns the excused chains."""
    bad = np.nonzero((gpu_ch != orc_ch).any(axis=1))[0]
    for c in bad:
        i = int(np.nonzero(gpu_ch[c] != orc_ch[c])[0][0])
        m = margins[c, sweep_index, i]
        assert m < BOUNDARY, f"chain {c} site {i}: margin {m:.3e} is not a boundary event"
    return bad


# ----------------------------------------------------------------- chains / fields
@pytest.mark.parametrize("N,L,q", [(1000, 37, 21), (333, 64, 5), (7, 3, 2)])
def test_init_chains_bitexact(N, L, q):
    g = api.init_chains(N, L, q, seed=1234 + q)
    assert np.array_equal(host(g), O.init_chains(N, L, q, 1234 + q))


@pytest.mark.parametrize("L,q,N", [(20, 21, 64), (37, 5, 50)])
def test_local_fields_match_oracle(L, q, N):
    h, J = synth.planted_dense(L, q, seed=40 + L, sigma_J=0.3)
    ch = O.init_chains(N, L, q, seed=41)
    H = torch.empty(api.workspace_bytes(B.WS_GIBBS, N, L, q, B.SAMPLER_FIELDS) // 4,
                    dtype=torch.float32, device="cuda")
    api.gibbs(dev(h), dev(J), dev(ch), sweeps=0, seed=0, H_ws=H, sampler="fields")
    Hg = host(H)[: N * L * q].reshape(N, L * q)
    for c in range(N):
        Ho = O.local_fields(h, J, ch[c], q)
        assert np.all(np.abs(Hg[c] - Ho) <= 1e-5 * (1 + np.abs(Ho)))


# ----------------------------------------------------------------- Gibbs trajectories
@pytest.mark.parametrize("sampler", ["fields", "gather"])
@pytest.mark.parametrize("L,q,N,sJ", [(20, 21, 500, 0.1), (33, 5, 300, 0.5), (70, 21, 130, 0.2)])
def test_gibbs_trajectory_single_sweeps(L, q, N, sJ, sampler):
    """Shared Philox counters: identical states after every sweep except at
    boundary events, after which the chain is resynchronised to the oracle."""
    h, J = synth.planted_dense(L, q, seed=50 + L, sigma_J=sJ)
    seed = 77
    ch = O.init_chains(N, L, q, seed=51)
    hg, Jg, chg = dev(h), dev(J), dev(ch)
    excused = 0
    for s in range(12):
        api.gibbs(hg, Jg, chg, sweeps=1, seed=seed, sweep_offset=s, sampler=sampler)
        orc, mg, _ = O.gibbs(h, J, ch, q, sweeps=1, seed=seed, sweep_offset=s, want_margins=True)
        g = host(chg)
        bad = check_trajectory(g, orc, mg)
        excused += len(bad)
        ch = orc
        if len(bad):
            chg.copy_(dev(orc))
    assert excused <= max(2, N * 12 // 1000)


def test_gibbs_multi_sweep_drift_and_states():
    """Ten sweeps in one call: the incrementally updated local fields stay within
    1e-5 (1 + |H|) of fields rebuilt from scratch, and every chain whose final
    state differs from the oracle's went through a boundary event."""
    L, q, N = 20, 21, 400
    h, J = synth.planted_dense(L, q, seed=60, sigma_J=0.1)
    ch = O.init_chains(N, L, q, seed=61)
    H = torch.empty(api.workspace_bytes(B.WS_GIBBS, N, L, q, B.SAMPLER_FIELDS) // 4,
                    dtype=torch.float32, device="cuda")
    flips = torch.zeros(1, dtype=torch.int64, device="cuda")
    chg = dev(ch)
    api.gibbs(dev(h), dev(J), chg, sweeps=10, seed=62, sweep_offset=5, H_ws=H, flips=flips,
              sampler="fields")
    g = host(chg)
    orc, _, oflips = O.gibbs(h, J, ch, q, sweeps=10, seed=62, sweep_offset=5)
    bad = check_chains(h, J, ch, g, orc, q, 10, 62, sweep_offset=5)
    good = np.setdiff1d(np.arange(N), bad)
    Hg = host(H)[: N * L * q].reshape(N, L * q)
    for c in good[:100]:
        Ho = O.local_fields(h, J, g[c], q)
        assert np.all(np.abs(Hg[c] - Ho) <= 1e-5 * (1 + np.abs(Ho)))
    if len(bad) == 0:
        assert int(host(flips)[0]) == oflips


@pytest.mark.parametrize("L,q,N", [(20, 21, 400), (150, 21, 64), (37, 4, 200)])
def test_gibbs_gather_multi_sweep_states(L, q, N):
    """Gather form, ten sweeps in one call: every chain that ends in a state
    different from the oracle's went through a boundary event; flips agree
    when none did."""
    h, J = synth.planted_dense(L, q, seed=63 + L, sigma_J=0.1)
    ch = O.init_chains(N, L, q, seed=64)
    flips = torch.zeros(1, dtype=torch.int64, device="cuda")
    chg = dev(ch)
    api.gibbs(dev(h), dev(J), chg, sweeps=10, seed=65, sweep_offset=3, flips=flips,
              sampler="gather")
    g = host(chg)
    orc, _, oflips = O.gibbs(h, J, ch, q, sweeps=10, seed=65, sweep_offset=3)
    bad = check_chains(h, J, ch, g, orc, q, 10, 65, sweep_offset=3)
    assert len(bad) <= max(2, N // 50)
    if len(bad) == 0:
        assert int(host(flips)[0]) == oflips


@pytest.mark.parametrize("L,q,N", [
    # a chain's 8 lanes as 8, 4, 2 and 1 site groups (q <= 4, <= 8, <= 16, > 16)
    (30, 2, 2600), (61, 3, 300), (45, 7, 2100), (130, 13, 700),
    # several waves per workgroup, one chunk per site, many chunks, largest L and q
    (77, 21, 2300), (24, 9, 3000), (200, 17, 120), (300, 32, 16), (512, 21, 10),
    # q <= 16 with more than 8 waves (the 16-wave instantiation), and q <= 8
    # where 8 lanes per chain replace 16 (the 8-wave instantiation)
    (40, 5, 20000), (30, 13, 20000), (60, 8, 10000),
    # narrow chains (one lane per quad: 5, 6, 7 lanes) in the 12-wave
    # instantiation, and 6-lane chains with 13 waves (the 16-wave one)
    (40, 17, 22000), (60, 21, 19000), (50, 25, 19000), (20, 21, 32768)])
def test_gibbs_gather_lane_splits(L, q, N):
    """Gather form over the lane layouts and workgroup shapes it picks from
    (L, q, N): after three sweeps in one call every chain that differs from
    the oracle went through a boundary event."""
    h, J = synth.planted_dense(L, q, seed=163 + L, sigma_J=0.1)
    ch = O.init_chains(N, L, q, seed=164)
    flips = torch.zeros(1, dtype=torch.int64, device="cuda")
    chg = dev(ch)
    api.gibbs(dev(h), dev(J), chg, sweeps=3, seed=165, sweep_offset=7, flips=flips,
              sampler="gather")
    g = host(chg)
    orc, _, oflips = O.gibbs(h, J, ch, q, sweeps=3, seed=165, sweep_offset=7)
    bad = check_chains(h, J, ch, g, orc, q, 3, 165, sweep_offset=7)
    assert len(bad) <= max(2, N // 50)
    if len(bad) == 0:
        assert int(host(flips)[0]) == oflips


@pytest.mark.parametrize("L,q", [(256, 21), (200, 12), (100, 5)])
def test_gibbs_gather_schedules_agree(L, q):
    """A chain's trajectory does not depend on the launch it runs in: 100
    chains alone (few chains per workgroup: one barrier per chunk-step, three
    chunks in flight, 8-lane chains) and the same 100 at the head of 20 000
    (paired chunk-steps; narrow chains at q = 21) end in the same states, bit
    for bit, after 4 sweeps."""
    h, J = synth.planted_dense(L, q, seed=171 + q, sigma_J=0.1)
    hg, Jg = dev(h), dev(J)
    big = api.init_chains(20000, L, q, 172)
    small = big[:100].clone()
    api.gibbs(hg, Jg, big, sweeps=4, seed=173, sweep_offset=11, sampler="gather")
    api.gibbs(hg, Jg, small, sweeps=4, seed=173, sweep_offset=11, sampler="gather")
    assert torch.equal(big[:100], small)


@pytest.mark.parametrize("L,q", [(256, 21), (100, 21), (200, 12)])
def test_metropolis_gather_schedules_agree(L, q):
    """The same for Metropolis sweeps: 100 chains alone (one barrier per
    chunk-step) and at the head of 20 000 (paired chunk-steps) end in the
    same states after 4 sweeps; at these shapes both launches take the same
    chunk length, which the Metropolis summation order also follows."""
    h, J = synth.planted_dense(L, q, seed=181 + q, sigma_J=0.1)
    hg, Jg = dev(h), dev(J)
    big = api.init_chains(20000, L, q, 182)
    small = big[:100].clone()
    api.gibbs(hg, Jg, big, sweeps=4, seed=183, sweep_offset=5, sampler="metropolis-gather")
    api.gibbs(hg, Jg, small, sweeps=4, seed=183, sweep_offset=5, sampler="metropolis-gather")
    assert torch.equal(big[:100], small)


def _sidak_z(n_tests, alpha=0.01):
    from scipy.stats import norm
    a1 = 1 - (1 - alpha) ** (1.0 / n_tests)
    return norm.ppf(1 - a1 / 2)


@pytest.mark.parametrize("sampler", ["fields", "gather"])
def test_gibbs_stationary_tiny_model(sampler):
    """L=4, q=3: 10^5 chains x 50 sweeps; every p_i and p_ij within the
    Sidak-corrected 3-sigma-equivalent band of exact enumeration."""
    L, q, N = 4, 3, 100000
    h, J = synth.planted_dense(L, q, seed=70, sigma_J=1.0)
    p1, p2, _ = O.enumerate_exact(h, J, L, q)
    chg = api.init_chains(N, L, q, seed=71)
    api.gibbs(dev(h), dev(J), chg, sweeps=50, seed=72, sampler=sampler)
    Y = onehot(host(chg).astype(np.int64), q)
    s1, s2 = Y.mean(0), Y.T @ Y / N
    z1 = np.abs(s1 - p1) / np.sqrt(np.maximum(p1 * (1 - p1), 1e-12) / N)
    z2 = np.abs(s2 - p2) / np.sqrt(np.maximum(p2 * (1 - p2), 1e-12) / N)
    assert max(z1.max(), z2.max()) < _sidak_z(len(p1) + p2.size)


@pytest.mark.parametrize("sampler", ["fields", "gather"])
def test_gibbs_beta_zero_is_uniform_and_two_state(sampler):
    N = 200000
    h = np.array([[0.3, -0.9]], dtype=np.float32)
    J = np.zeros((2, 2), dtype=np.float32)
    chg = torch.zeros((N, 1), dtype=torch.int8, device="cuda")
    api.gibbs(dev(h), dev(J), chg, sweeps=1, seed=5, sampler=sampler)
    p = np.exp(-0.9) / (np.exp(0.3) + np.exp(-0.9))
    f = host(chg).mean()
    assert abs(f - p) < 5 * np.sqrt(p * (1 - p) / N)
    api.gibbs(dev(h), dev(J), chg, sweeps=1, seed=6, beta=0.0, sampler=sampler)
    assert abs(host(chg).mean() - 0.5) < 5 * np.sqrt(0.25 / N)


# ----------------------------------------------------------------- statistics
@pytest.mark.parametrize("prec", ["bf16x2", "fp32"])
@pytest.mark.parametrize("L,q,M", [(20, 21, 700), (37, 5, 300), (7, 2, 129), (11, 21, 50),
                                   (11, 21, 100), (6, 4, 257)])
def test_stats_unit_weights_bitexact(prec, L, q, M):
    X = synth.clustered_msa(M, L, q, seed=80 + L)
    f1g, f2g, mg = api.stats(dev(X), q, None, -1.0, prec)
    f1o, f2o, mo = O.stats(X, q, None, -1.0)
    assert host(mg)[0] == mo
    assert np.array_equal(host(f1g), f1o)
    assert np.array_equal(host(f2g), f2o)


@pytest.mark.parametrize("prec,tol", [("bf16x2", 1e-5), ("fp32", 1e-6)])
@pytest.mark.parametrize("L,q,M", [(20, 21, 1500), (37, 5, 700), (9, 2, 500), (13, 3, 400),
                                   (15, 21, 40), (15, 21, 170), (8, 5, 1090)])
def test_stats_weighted(L, q, M, prec, tol):
    X = synth.clustered_msa(M, L, q, seed=90 + q)
    w = synth.weights_open_unit(M, 91)
    f1g, f2g, mg = api.stats(dev(X), q, dev(w), -1.0, prec)
    f1o, f2o, mo = O.stats(X, q, w, -1.0)
    assert abs(host(mg)[0] - mo) <= 1e-12 * mo
    e1 = np.abs(host(f1g) - f1o).max()
    e2 = np.abs(host(f2g) - f2o).max()
    print(f"stats {prec}: max|df1|={e1:.3e} max|df2|={e2:.3e}")
    assert e1 <= tol and e2 <= tol
    f2 = host(f2g)
    assert np.array_equal(f2, f2.T)


def test_stats_token_error_flag():
    X = synth.random_sequences(100, 10, 21, 3)
    X[5, 3] = 25
    e = err_flag()
    api.stats(dev(X), 21, None, -1.0, "bf16x2", dev_err=e)
    assert int(host(e)[0]) & B.DEVERR_TOKEN


@pytest.mark.parametrize("L,q", [(20, 21), (37, 5), (1, 2)])
def test_profile_fields(L, q):
    """bmdca_profile_fields against the oracle: float32 of the FP64 log; a
    zero frequency raises the non-finite flag."""
    X = synth.clustered_msa(400, L, q, seed=95 + L)
    f1, _, _ = O.stats(X, q, None, -1.0)
    e = err_flag()
    h = api.profile_fields(dev(f1), L, q, dev_err=e)
    ho = O.profile_fields(f1, L, q)
    hg = host(h)
    # FP64 log on the GPU and in libm may differ in the last bit; rounded to
    # float32 they agree unless the FP64 value lies within 1 ulp of a float32
    # rounding boundary
    diff = hg != ho
    assert diff.sum() <= max(1, hg.size // 1000)
    assert np.all(np.abs(hg[diff] - ho[diff]) <= np.spacing(np.abs(ho[diff])))
    assert int(host(e)[0]) == 0
    f0 = f1.copy()
    f0[0] = 0.0
    api.profile_fields(dev(f0), L, q, dev_err=e)
    assert int(host(e)[0]) & B.DEVERR_NONFINITE


# ----------------------------------------------------------------- reweighting
@pytest.mark.parametrize("L,M,theta", [(40, 1500, 0.8), (100, 700, 0.8), (256, 300, 0.5),
                                       (35, 400, 0.8)])
def test_reweight_bitexact(L, M, theta):
    q = 21
    X = synth.clustered_msa(M, L, q, seed=100 + L, mut_rate=0.12)
    n, w, meff = api.reweight(dev(X), q, theta)
    no, wo, mo = O.reweight(X, theta)
    assert np.array_equal(host(n), no)
    assert np.array_equal(host(w), wo)
    assert abs(host(meff)[0] - mo) <= 1e-12 * mo
    assert no.max() > 1


# ----------------------------------------------------------------- scoring
def term_scale(h, J, S, q):
    """sum_i |h_i(s_i)| + sum_{i<j} |J_ij(s_i,s_j)| per sequence (tolerance scale)."""
    L = S.shape[1]
    out = []
    for s in S:
        idx = np.arange(L) * q + s
        a = np.abs(h.reshape(-1)[idx].astype(np.float64)).sum()
        sub = np.abs(J[np.ix_(idx, idx)].astype(np.float64))
        out.append(a + np.triu(sub, 1).sum())
    return np.array(out)


# several sequence blocks (2048 per workgroup for q > 8, 1024 otherwise) with
# a ragged tail; L below, at and across the 16-site column chunks; q across
# the template range and every LDS row pad (0: q = 2, 3; 4: q = 16, 32;
# 8: q = 5, 8, 21; 12: q = 12, 20)
@pytest.mark.parametrize("L,q,Bn", [(30, 21, 1000), (130, 21, 64), (9, 5, 257), (1, 21, 5),
                                    (2, 2, 3000), (16, 3, 100), (17, 32, 2100), (100, 21, 2500),
                                    (40, 12, 4500), (33, 8, 2100), (25, 20, 2049), (18, 16, 700)])
def test_energy(L, q, Bn):
    h, J = synth.planted_dense(L, q, seed=110 + L, sigma_J=0.3)
    S = synth.random_sequences(Bn, L, q, 111)
    Eg = host(api.energy(dev(h), dev(J), dev(S)))
    Eo = O.energy(h, J, S, q)
    assert np.all(np.abs(Eg - Eo) <= 1e-4 * term_scale(h, J, S, q))


def test_energy_independent_of_batch():
    """A sequence scores the same bits alone, in a small batch and in a large one."""
    L, q = 77, 21
    h, J = synth.planted_dense(L, q, seed=112, sigma_J=0.3)
    S = synth.random_sequences(3000, L, q, 113)
    big = host(api.energy(dev(h), dev(J), dev(S)))
    for lo, hi in [(0, 1), (1500, 1501), (2047, 2300), (5, 1029)]:
        part = host(api.energy(dev(h), dev(J), dev(S[lo:hi])))
        assert np.array_equal(part, big[lo:hi])


def test_single_mutant_scan():
    L, q = 30, 21
    h, J = synth.planted_dense(L, q, seed=120, sigma_J=0.3)
    WT = synth.random_sequences(4, L, q, 121)
    dE = host(api.single_mutant_scan(dev(h), dev(J), dev(WT)))
    scale = term_scale(h, J, WT, q)
    for b in range(4):
        ref = O.mutant_scan(h, J, WT[b], q)
        assert np.all(np.abs(dE[b] - ref) <= 1e-4 * scale[b])
        assert np.all(dE[b].reshape(L, q)[np.arange(L), WT[b]] == 0)


@pytest.mark.parametrize("L,q,gap", [(45, 21, 0), (45, 21, -1), (2, 21, 0), (3, 7, -1),
                                     (33, 2, 1), (64, 13, 12), (77, 32, 0), (50, 5, 2)])
def test_apc_frobenius(L, q, gap):
    """Blocks per wave 64 // q from 2 (q = 32) to 32 (q = 2), rows paired as
    (i, L - 1 - i) with an odd L's middle row alone; no gap, the first,
    an inner and the last state as the gap."""
    if L == 45:
        _, J = synth.planted_sparse(L, q, seed=130, sigma_J=0.5)
    else:  # every block nonzero
        _, J = synth.planted_dense(L, q, seed=130 + L + q, sigma_J=0.3)
    F, Fa = api.apc_frobenius(dev(J), L, q, gap)
    Fo, Fao = O.apc_frobenius(J, L, q, gap)
    sc = np.abs(Fo).max()
    assert np.abs(host(F) - Fo).max() <= 1e-5 * sc
    assert np.abs(host(Fa) - Fao).max() <= 1e-5 * sc


# ----------------------------------------------------------------- one epoch
def c1_problem(L=20, q=21, M=500, N=500):
    """Plain bmDCA at CPU-seconds size: planted dense model, alignment of M
    sequences drawn by 200 sweeps of the oracle sampler, 80% identity weights."""
    h, J = synth.planted_dense(L, q, seed=1001, sigma_J=0.1)
    msa0 = O.init_chains(M, L, q, seed=2001)
    msa, _, _ = O.gibbs(h, J, msa0, q, sweeps=200, seed=2001)
    n, w, meff = O.reweight(msa, 0.8)
    f1, f2, _ = O.stats(msa, q, w, -1.0)
    chains = O.init_chains(N, L, q, seed=3001)
    return h, J, msa, w, f1, f2, chains


@pytest.mark.parametrize("sampler", ["fields", "gather"])
def test_train_step_c1_epochs(sampler):
    """20 epochs, lr 0.05, 10 sweeps, N = 500, both sides fed the same data
    frequencies: chains, h and J bit-exact after every epoch without boundary
    events; Pearson within 1e-12. After a boundary event both sides restart
    the next epoch from the oracle's state."""
    L, q = 20, 21
    _, _, _, _, f1, f2, chains = c1_problem()
    h = np.zeros((L, q), np.float32)
    J = np.zeros((L * q, L * q), np.float32)
    hg, Jg, cg = dev(h), dev(J), dev(chains)
    f1g, f2g = dev(f1), dev(f2)
    ws = api.workspace(B.WS_TRAIN_STEP, 500, L, q, B.PREC_BF16X2 | B.SAMPLER[sampler])
    e = err_flag()
    events = 0
    for ep in range(20):
        pr = api.train_step(hg, Jg, cg, f1g, f2g, 0.05, 10, seed=4001, epoch=ep, prec="bf16x2",
                            ws=ws, dev_err=e, sampler=sampler)
        h2, J2, ch2, r, _, _ = O.train_step(h, J, chains, f1, f2, q, 0.05, 10, 4001, ep)
        gch = host(cg)
        bad = check_chains(h, J, chains, gch, ch2, q, 10, 4001, sweep_offset=ep * 10)
        if len(bad):
            events += len(bad)
            hg.copy_(dev(h2)); Jg.copy_(dev(J2)); cg.copy_(dev(ch2))
        else:
            assert np.array_equal(host(hg), h2)
            assert np.array_equal(host(Jg), J2)
            assert abs(host(pr)[0] - r) <= 1e-12
        h, J, chains = h2, J2, ch2
    assert int(host(e)[0]) == 0
    assert events <= 5
    Jn = host(Jg).reshape(L, q, L, q)
    for i in range(L):
        assert np.all(Jn[i, :, i, :] == 0)
    assert np.array_equal(host(Jg), host(Jg).T)


def test_train_step_fp32_counts_match_bf16():
    L, q, N = 20, 21, 500
    _, _, _, _, f1, f2, chains = c1_problem()
    outs = []
    for prec in ["bf16x2", "fp32"]:
        hg = torch.zeros((L, q), dtype=torch.float32, device="cuda")
        Jg = torch.zeros((L * q, L * q), dtype=torch.float32, device="cuda")
        cg = dev(chains)
        pr = api.train_step(hg, Jg, cg, dev(f1), dev(f2), 0.05, 10, 4001, 0, prec=prec)
        outs.append((host(hg), host(Jg), host(pr)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2][0] == outs[1][2][0]


@pytest.mark.parametrize("L,q,N", [(20, 21, 500), (37, 5, 1000), (9, 32, 130), (2, 2, 1),
                                   (130, 7, 300), (64, 21, 4099)])
def test_train_step_direct_counts_equal_products(L, q, N):
    """Chain counts counted directly (the default) and from the one-hot
    product in both precisions are the same integers, so h, J, chains and the
    Pearson value agree bit for bit; the shapes take ragged site groups
    (L % 4 != 0), q = 32, a single chain and chain counts off the 64-row pad.
    With one chain the model correlations are all zero, so the Pearson value
    is 0/0 and raises the non-finite flag in every form alike."""
    rng = np.random.default_rng(L * 1000 + q)
    chains = rng.integers(0, q, size=(N, L), dtype=np.int8)
    h = (0.3 * rng.standard_normal((L, q))).astype(np.float32)
    J = (0.1 * rng.standard_normal((L * q, L * q))).astype(np.float32)
    J = (J + J.T) / 2
    Jv = J.reshape(L, q, L, q)
    for i in range(L):
        Jv[i, :, i, :] = 0
    f1 = rng.random(L * q)
    f2 = rng.random((L * q) ** 2)
    outs = []
    for prec in (B.PREC_FP32, B.PREC_FP32 | B.COUNTS_PRODUCT, B.PREC_BF16X2 | B.COUNTS_PRODUCT):
        hg, Jg, cg = dev(h), dev(J), dev(chains)
        e = err_flag()
        pr = api.train_step(hg, Jg, cg, dev(f1), dev(f2), 0.05, 1, 77, 0, prec=prec, dev_err=e)
        assert int(host(e)[0]) == (B.DEVERR_NONFINITE if N == 1 else 0)
        outs.append((host(hg), host(Jg), host(cg), host(pr)[0]))
    for o in outs[1:]:
        assert np.array_equal(outs[0][0], o[0]) and np.array_equal(outs[0][1], o[1])
        assert np.array_equal(outs[0][2], o[2])
        assert outs[0][3] == o[3] or (N == 1 and np.isnan(outs[0][3]) and np.isnan(o[3]))


def test_train_step_nonfinite_flag():
    """A huge learning rate overflows the float32 parameters: the device flag is
    raised; nothing faults."""
    L, q = 20, 21
    _, _, _, _, f1, f2, chains = c1_problem()
    hg = torch.zeros((L, q), dtype=torch.float32, device="cuda")
    Jg = torch.zeros((L * q, L * q), dtype=torch.float32, device="cuda")
    e = err_flag()
    api.train_step(hg, Jg, dev(chains), dev(f1), dev(f2), 1e300, 1, 1, 0, dev_err=e)
    assert int(host(e)[0]) & B.DEVERR_NONFINITE


@pytest.mark.parametrize("sampler", ["gather", "fields", "metropolis-gather", "metropolis-fields"])
@pytest.mark.parametrize("cus", [0, 8])
def test_gibbs_streams_equal_separate_calls(sampler, cus):
    """Chains of two callers swept in one launch through a stream table make
    the same draws as in their own calls (keys, chain indices, sweep offsets)."""
    L, q = 45, 21
    h, J = synth.planted_dense(L, q, seed=130, sigma_J=0.3)
    hg, Jg = dev(h), dev(J)
    a0, b0 = api.init_chains(300, L, q, seed=131), api.init_chains(77, L, q, seed=132)
    a, b = a0.clone(), b0.clone()
    api.gibbs(hg, Jg, a, 6, seed=1111, sweep_offset=0, sampler=sampler)
    api.gibbs(hg, Jg, b, 6, seed=2222, sweep_offset=35, sampler=sampler)
    both = torch.cat([a0, b0])
    seeds = np.array([1111] * 300 + [2222] * 77, dtype=np.uint64)
    offs = np.array([0] * 300 + [35] * 77, dtype=np.uint64)
    ids = np.concatenate([np.arange(300), np.arange(77)]).astype(np.uint32)
    st = api.chain_streams(seeds, offs, ids)
    api.gibbs_streams(hg, Jg, both, 6, st, sampler=sampler, cus=cus)
    assert torch.equal(both[:300], a) and torch.equal(both[300:], b)


# ----------------------------------------------------------------- Metropolis
MH_FORMS = ["metropolis-fields", "metropolis-gather"]


@pytest.mark.parametrize("sampler", MH_FORMS)
def test_metropolis_trajectories_match_oracle(sampler):
    L, q, N = 30, 21, 300
    h, J = synth.planted_dense(L, q, seed=140, sigma_J=0.3)
    ch0 = O.init_chains(N, L, q, seed=141)
    cg = dev(ch0)
    api.gibbs(dev(h), dev(J), cg, 1, seed=142, sampler=sampler)
    ref, mg, _ = O.metropolis(h, J, ch0, q, 1, 142, want_margins=True)
    check_trajectory(host(cg), ref, mg)
    # several sweeps, continued by offset: chains that differ met a boundary event
    cg = dev(ch0)
    api.gibbs(dev(h), dev(J), cg, 2, seed=143, sampler=sampler)
    api.gibbs(dev(h), dev(J), cg, 2, seed=143, sweep_offset=2, sampler=sampler)
    ref, _, _ = O.metropolis(h, J, ch0, q, 4, 143)
    bad = check_chains(h, J, ch0, host(cg), ref, q, 4, 143, metropolis=True)
    assert len(bad) <= N // 50


@pytest.mark.parametrize("L,q,N", [
    # the lane layouts of the gather form (8 lanes as 8, 4, 2, 1 site groups),
    # several waves per workgroup, many chunks, largest L and q
    (30, 2, 2600), (61, 3, 300), (45, 7, 2100), (130, 13, 700),
    (77, 21, 2300), (200, 17, 120), (300, 32, 16), (512, 21, 10)])
def test_metropolis_gather_lane_splits(L, q, N):
    """Gather-form Metropolis over the lane layouts and workgroup shapes:
    after three sweeps in one call every chain that differs from the oracle
    went through a boundary event, and with none the flip counts agree."""
    h, J = synth.planted_dense(L, q, seed=263 + L, sigma_J=0.1)
    ch = O.init_chains(N, L, q, seed=264)
    flips = torch.zeros(1, dtype=torch.int64, device="cuda")
    chg = dev(ch)
    api.gibbs(dev(h), dev(J), chg, sweeps=3, seed=265, sweep_offset=5, flips=flips,
              sampler="metropolis-gather")
    g = host(chg)
    orc, _, oflips = O.metropolis(h, J, ch, q, 3, 265, sweep_offset=5)
    bad = check_chains(h, J, ch, g, orc, q, 3, 265, sweep_offset=5, metropolis=True)
    assert len(bad) <= max(2, N // 50)
    if len(bad) == 0:
        assert int(host(flips)[0]) == oflips


@pytest.mark.parametrize("sampler", MH_FORMS)
@pytest.mark.parametrize("beta", [0.5, 1.7])
def test_metropolis_at_other_temperatures(sampler, beta):
    """beta != 1 (the sampling temperature of the sampling routine): both
    forms follow the oracle's trajectories, boundary events excused."""
    L, q, N = 40, 21, 400
    h, J = synth.planted_dense(L, q, seed=151, sigma_J=0.3)
    ch0 = O.init_chains(N, L, q, seed=152)
    cg = dev(ch0)
    api.gibbs(dev(h), dev(J), cg, 3, seed=153, sweep_offset=2, beta=beta, sampler=sampler)
    ref, _, _ = O.metropolis(h, J, ch0, q, 3, 153, sweep_offset=2, beta=beta)
    bad = check_chains(h, J, ch0, host(cg), ref, q, 3, 153, sweep_offset=2, beta=beta,
                       metropolis=True)
    assert len(bad) <= N // 50


@pytest.mark.parametrize("sampler", MH_FORMS)
def test_metropolis_stationary_marginals_vs_enumeration(sampler):
    L, q, N = 4, 3, 100000
    h, J = synth.planted_dense(L, q, seed=144, sigma_J=1.0)
    p1, p2, _ = O.enumerate_exact(h, J, L, q)
    cg = api.init_chains(N, L, q, seed=145)
    api.gibbs(dev(h), dev(J), cg, 80, seed=146, sampler=sampler)
    Y = onehot(host(cg).astype(np.int64), q)
    s1, s2 = Y.mean(0), Y.T @ Y / N
    z = max((np.abs(s1 - p1) / np.sqrt(np.maximum(p1 * (1 - p1), 1e-12) / N)).max(),
            (np.abs(s2 - p2) / np.sqrt(np.maximum(p2 * (1 - p2), 1e-12) / N)).max())
    assert z < 4.5, z


@pytest.mark.parametrize("sampler", MH_FORMS)
def test_train_step_with_metropolis_sweeps(sampler):
    """train_step's sampler leg with the Metropolis flag is bmdca_gibbs with it."""
    L, q, N = 20, 21, 500
    h, J = synth.planted_dense(L, q, seed=147, sigma_J=0.1)
    X = synth.clustered_msa(400, L, q, seed=148)
    f1, f2, _ = api.stats(dev(X), q, None, -1.0, "fp32")
    ch0 = O.init_chains(N, L, q, seed=149)
    hg, Jg, cg = dev(h), dev(J), dev(ch0)
    api.train_step(hg, Jg, cg, f1, f2, 0.05, 5, 150, 3, "bf16x2", sampler=sampler)
    c2 = dev(ch0)
    api.gibbs(dev(h), dev(J), c2, 5, 150, sweep_offset=15, sampler=sampler)
    assert torch.equal(cg, c2)
    # both forms at once is not a sampler: rejected (no workspace size, and the call)
    bad = B.SAMPLER_METROPOLIS | B.SAMPLER_GATHER | B.SAMPLER_FIELDS
    assert B.lib().bmdca_workspace_bytes(B.WS_GIBBS, N, L, q, bad) == 0
    ws = api.workspace(B.WS_GIBBS, N, L, q, B.SAMPLER_METROPOLIS)
    with pytest.raises(B.BmdcaError):
        api.gibbs(dev(h), dev(J), dev(ch0), 1, 1, H_ws=ws, sampler=bad)


# ----------------------------------------------------------------- serving forms
def test_serving_forms_equal_plain_calls():
    """bmdca_energy_batch, bmdca_mutant_scan_batch and bmdca_sample_tick over
    arenas larger than the live count: live items equal the plain calls bit
    for bit, items past the count are untouched, and a request joining the
    sampling arena at a later tick draws as its own bmdca_gibbs call."""
    L, q = 57, 21
    h, J = synth.planted_dense(L, q, seed=160, sigma_J=0.3)
    hg, Jg = dev(h), dev(J)
    S = dev(synth.random_sequences(3000, L, q, 161))
    n = torch.tensor([1234], dtype=torch.int64, device="cuda")
    E = torch.full((3000,), float("nan"), dtype=torch.float32, device="cuda")
    ws = api.workspace(B.WS_ENERGY, 3000, L, q, 0)
    api.energy_batch(hg, Jg, S, n, E, ws)
    assert torch.equal(E[:1234], api.energy(hg, Jg, S[:1234]))
    assert bool(torch.isnan(E[1234:]).all())
    W = dev(synth.random_sequences(5, L, q, 162))
    dE = torch.full((5, L * q), float("nan"), dtype=torch.float32, device="cuda")
    n3 = torch.tensor([3], dtype=torch.int64, device="cuda")
    api.mutant_scan_batch(hg, Jg, W, n3, dE, api.workspace(B.WS_MUTANT, 5, L, q, 0))
    assert torch.equal(dE[:3], api.single_mutant_scan(hg, Jg, W[:3]))
    assert bool(torch.isnan(dE[3:]).all())
    # sampling arena of 500 chains: request A (300 chains) from tick 0,
    # request B (150 chains) joins at tick 2; 2 sweeps a tick, 5 ticks
    cap, sw = 500, 2
    arena = torch.zeros((cap, L), dtype=torch.int8, device="cuda")
    api.init_chains(300, L, q, 11, out=arena[:300])
    tick = torch.zeros(1, dtype=torch.int64, device="cuda")
    live = torch.tensor([300], dtype=torch.int64, device="cuda")
    seeds = np.array([11] * 300 + [22] * 150 + [0] * 50, dtype=np.uint64)
    offs = np.array([0] * 300 + [(-2 * sw) % (1 << 64)] * 150 + [0] * 50, dtype=np.uint64)
    ids = np.concatenate([np.arange(300), np.arange(150), np.zeros(50)]).astype(np.uint32)
    table = api.chain_streams(seeds, offs, ids)
    wsg = api.workspace(B.WS_GIBBS, cap, L, q, B.SAMPLER_GATHER)
    api.gibbs(hg, Jg, arena[:1].clone(), 0, 0, H_ws=wsg, sampler="gather")  # lays J out
    tail = arena[450:].clone()
    for t in range(5):
        if t == 2:
            api.init_chains(150, L, q, 22, out=arena[300:450])
            live.fill_(450)
        api.sample_tick(hg, Jg, arena, live, sw, table, tick, wsg, keep_layout=True)
    assert int(tick.item()) == 5
    a = api.gibbs(hg, Jg, api.init_chains(300, L, q, 11), 10, 11, sampler="gather")
    b = api.gibbs(hg, Jg, api.init_chains(150, L, q, 22), 6, 22, sampler="gather")
    assert torch.equal(arena[:300], a) and torch.equal(arena[300:450], b)
    assert torch.equal(arena[450:], tail)
