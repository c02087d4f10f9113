"""Parity at the full sizes of the benchmark configurations, in the launch
configuration the benchmark uses: sampled outputs the oracle computes one by
one, plus invariants that hold at any size.  Edge cases at the end.

Workloads (synthetic, seeded):
  protein scale   L=100, q=21, N=10 000 chains, M=20 000 rows
  precision form  L=256, q=21, N=20 000 chains, M=100 000 weighted rows
  RNA-like        L=400, q=5,  N=4096 chains
  largest served  L=512, q=21 (energies, mutant scan, contact scores)
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2501_18456_amd import api, synth
from paper_2501_18456_amd import _lib as B
from tests.trajectory_check import check_chains

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


_cache = {}


def protein_problem():
    if "protein" not in _cache:
        L, q, M = 100, 21, 20000
        h, J = synth.planted_sparse(L, q, seed=1002, sigma_J=0.5, gap_mass=0.15)
        X = synth.clustered_msa(M, L, q, seed=2002, n_families=40, mut_rate=0.25)
        _cache["protein"] = (h, J, X)
    return _cache["protein"]


def precision_msa():
    if "precision" not in _cache:
        L, q, M = 256, 21, 100000
        X = synth.clustered_msa(M, L, q, seed=2003, n_families=200, mut_rate=0.3)
        w = synth.weights_open_unit(M, 4003)
        _cache["precision"] = (X, w)
    return _cache["precision"]


def sample_pairs(Lq, n, seed):
    g = np.random.default_rng(seed)
    r1 = g.integers(0, Lq, n)
    r2 = g.integers(0, Lq, n)
    return r1, r2


# ---------------------------------------------------------------- protein scale
def test_protein_reweight_sampled_rows():
    _, _, X = protein_problem()
    n, w, meff = api.reweight(dev(X), 21, 0.8)
    n, w = host(n), host(w)
    rows = np.random.default_rng(5).choice(len(X), 60, replace=False)
    ref = O.reweight_rows(X, rows, 0.8)
    assert np.array_equal(n[rows], ref)
    assert np.array_equal(w[rows], 1.0 / ref)
    assert n.max() > 1  # the alignment is redundant at 80% identity
    assert abs(host(meff)[0] - w.sum()) <= 1e-10 * w.sum()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("bf16x2", 1e-5)])
def test_protein_stats_sampled_entries(prec, tol):
    _, _, X = protein_problem()
    L, q = 100, 21
    w = synth.weights_open_unit(len(X), 6)
    f1, f2, meff = api.stats(dev(X), q, dev(w), -1.0, prec)
    f1, f2 = host(f1), host(f2)
    r1, r2 = sample_pairs(L * q, 3000, 7)
    ref = O.stats_entries(X, q, r1, r2, w, -1.0)
    assert np.abs(f2[r1, r2] - ref).max() <= tol
    d = np.arange(L * q)
    assert np.abs(f1 - O.stats_entries(X, q, d, d, w, -1.0)).max() <= tol
    assert np.array_equal(f2, f2.T)
    F2 = f2.reshape(L, q, L, q)
    marg = F2.sum(axis=3)  # sum over b of f_ij(a, b) = f_i(a) for j != i
    off = ~np.eye(L, dtype=bool)
    assert np.abs(marg.transpose(0, 2, 1)[off] - f1.reshape(L, q)[:, None, :].repeat(L, 1)[off]).max() <= q * tol


@pytest.mark.parametrize("sampler", ["gather", "fields"])
def test_protein_epoch(sampler):
    """One epoch at full size: sampled chains follow the oracle's trajectories
    (boundary events excused by replay); h and J equal the oracle's update
    (Eq. 5) on the chain frequencies of the GPU's own chains, bit for bit, and
    the Pearson value matches the oracle's on those chains."""
    h_true, J_true, X = protein_problem()
    L, q, N, lr = 100, 21, 10000, 0.05
    _, w, _ = O.reweight(X[:2000], 0.8)  # weights of a block; any weights will do here
    ww = np.ones(len(X))
    ww[:2000] = w
    f1, f2, _ = O.stats(X, q, ww, -1.0)
    h0 = np.log(f1).astype(np.float32).reshape(L, q)
    J0 = J_true * 0.5  # a non-trivial starting model
    ch0 = O.init_chains(N, L, q, seed=3002)
    hg, Jg, cg = dev(h0), dev(J0), dev(ch0)
    pr = api.train_step(hg, Jg, cg, dev(f1), dev(f2), lr, 10, seed=3002, epoch=3, prec="fp32",
                        sampler=sampler)
    g = host(cg)
    # sampled slices of chains against the oracle
    for c0 in (0, 4321, N - 37):
        sl = slice(c0, c0 + 37)
        ref, _, _ = O.gibbs_range(h0, J0, ch0[sl], c0, q, 10, 3002, sweep_offset=30)
        bad = check_chains(h0, J0, ch0[sl], g[sl], ref, q, 10, 3002, sweep_offset=30, c0=c0)
        assert len(bad) <= 2
    # the update of Eq. (5) on the GPU's own chains: bit for bit
    P1, P2 = O.chain_freqs(g, q)
    h1o, J1o = O.update(h0, J0, f1, f2, P1, P2, L, q, lr)
    assert np.array_equal(host(hg).reshape(-1), h1o.reshape(-1))
    assert np.array_equal(host(Jg), J1o)
    assert abs(host(pr)[0] - O.pearson(f1, f2, P1, P2, L, q)) < 1e-10


def test_protein_metropolis_gather_sampled_chains():
    """Gather-form Metropolis at full size (10 sweeps of 10 000 chains):
    sampled slices follow the oracle's trajectories, boundary events excused."""
    h_true, J_true, _ = protein_problem()
    L, q, N = 100, 21, 10000
    ch0 = O.init_chains(N, L, q, seed=3012)
    cg = dev(ch0)
    api.gibbs(dev(h_true), dev(J_true), cg, 10, seed=3013, sweep_offset=4,
              sampler="metropolis-gather")
    g = host(cg)
    for c0 in (0, 5000, N - 37):
        sl = slice(c0, c0 + 37)
        ref, _, _ = O.metropolis(h_true, J_true, ch0[sl], q, 10, 3013, sweep_offset=4, c0=c0)
        bad = check_chains(h_true, J_true, ch0[sl], g[sl], ref, q, 10, 3013, sweep_offset=4,
                           metropolis=True, c0=c0)
        assert len(bad) <= 2


def _tied(sc, r1, r2, pairs, thr):
    for a, b in pairs:
        lo, hi = min(a, b), max(a, b)
        s = sc[(r1 == lo) & (r2 == hi)][0]
        assert abs(s - thr) <= 1e-12 * max(abs(thr), 1e-300), (a, b, s, thr)


def test_protein_graph_updates():
    """One edDCA and one eaDCA graph update over the 2.18e6 elements of the
    protein-scale model, from 10 000 chains: masks equal to the oracle's
    except elements tied with the threshold to ~1 ulp (exp and log on the
    GPU vs libm), same active counts when equal."""
    h_true, J_true, X = protein_problem()
    L, q, N = 100, 21, 10000
    Lq = L * q
    ch = O.init_chains(N, L, q, seed=3022)
    ch = host(api.gibbs(dev(h_true), dev(J_true), dev(ch), 3, seed=3023))
    full = np.ones((Lq, Lq), np.uint8)
    for i in range(L):
        full[i * q:(i + 1) * q, i * q:(i + 1) * q] = 0
    Y = np.zeros((N, Lq), np.float32)
    Y[np.arange(N)[:, None], np.arange(L)[None, :] * q + ch] = 1.0
    Cg = torch.from_numpy(Y).cuda()
    p2 = ((Cg.T @ Cg).double() / N).cpu().numpy()  # exact counts / N
    r1, r2 = np.triu_indices(Lq, 1)
    keep = r1 // q != r2 // q
    r1, r2 = r1[keep], r2[keep]
    # decimation of 1% of the full graph
    J0 = (J_true * full).astype(np.float32)
    Jg, mg = dev(J0), dev(full)
    n = api.decimate(Jg, mg, dev(ch), q, 0.01, 0.0)
    Jn, mn, no = O.decimate(J0, full, ch, q, 0.01, 0.0)
    diff = np.argwhere(host(mg) != mn)
    if diff.size:
        sc = np.array([O.skl_element(J0[a, b], p2[a, b]) for a, b in zip(r1, r2)])
        _tied(sc, r1, r2, diff, np.sort(sc)[len(sc) - no - 1])
    else:
        assert int(host(n)[0]) == no and np.array_equal(host(Jg), Jn)
    # activation of 0.1% of the empty graph's inactive count
    f2 = O.stats(X, q, None, -1.0)[1]
    empty = np.zeros((Lq, Lq), np.uint8)
    mg = dev(empty)
    n = api.activate(mg, dev(ch), dev(f2), q, 0.001)
    mo, no = O.activate(empty, ch, f2, q, 0.001)
    diff = np.argwhere(host(mg) != mo)
    if diff.size:
        sc = np.array([O.bernoulli_kl(f2[a, b], p2[a, b]) for a, b in zip(r1, r2)])
        _tied(sc, r1, r2, diff, np.sort(sc)[::-1][no - 1])
    else:
        assert int(host(n)[0]) == no


def test_protein_seqid_sums():
    """SeqID of 10 000 chain pairs at L = 100: exact integer sums."""
    L, q, N = 100, 21, 10000
    A = O.init_chains(N, L, q, seed=3031)
    Bm = np.where(np.random.default_rng(3032).random((N, L)) < 0.3, A,
                  O.init_chains(N, L, q, seed=3033)).astype(np.int8)
    perm = np.random.default_rng(3034).permutation(N).astype(np.int32)
    for pm in (None, perm):
        got = host(api.seqid(dev(A), dev(Bm), None if pm is None else dev(pm)))
        m, sd = O.seqid(A, Bm, pm)
        assert got[0] == m and abs(got[1] - sd) <= 1e-15 * max(1.0, sd)


# ---------------------------------------------------------------- precision form
@pytest.mark.parametrize("prec,tol", [("bf16x2", 1e-5), ("fp32", 1e-6)])
def test_precision_stats_sampled_entries(prec, tol):
    X, w = precision_msa()
    L, q = 256, 21
    f1, f2, meff = api.stats(dev(X), q, dev(w), -1.0, prec)
    r1, r2 = sample_pairs(L * q, 800, 8)
    sel = torch.from_numpy(r1 * (L * q) + r2).cuda()
    got = host(f2.reshape(-1)[sel])
    ref = O.stats_entries(X, q, r1, r2, w, -1.0)
    err = np.abs(got - ref).max()
    print(f"precision-form stats {prec}: max |f2 - oracle| over 800 entries = {err:.3e}")
    assert err <= tol
    d = np.arange(0, L * q, 7)
    assert np.abs(host(f1)[d] - O.stats_entries(X, q, d, d, w, -1.0)).max() <= tol
    assert bool((f2 == f2.T).all())
    assert abs(host(meff)[0] - w.sum()) <= 1e-10 * w.sum()


def test_precision_gibbs_sampled_chains():
    L, q, N = 256, 21, 20000
    h, J = synth.planted_dense(L, q, seed=1003, sigma_J=0.05)
    ch0 = O.init_chains(N, L, q, seed=3003)
    cg = dev(ch0)
    api.gibbs(dev(h), dev(J), cg, 2, seed=3003, sweep_offset=7)
    g = host(cg)
    for c0 in (0, 12345, N - 20):
        sl = slice(c0, c0 + 20)
        ref, _, _ = O.gibbs_range(h, J, ch0[sl], c0, q, 2, 3003, sweep_offset=7)
        bad = check_chains(h, J, ch0[sl], g[sl], ref, q, 2, 3003, sweep_offset=7, c0=c0)
        assert len(bad) <= 1


# ---------------------------------------------------------------- RNA-like
def test_rna_gibbs_and_counts():
    L, q, N = 400, 5, 4096
    h, J = synth.planted_dense(L, q, seed=1004, sigma_J=0.05)
    ch0 = O.init_chains(N, L, q, seed=3004)
    cg = dev(ch0)
    api.gibbs(dev(h), dev(J), cg, 1, seed=3004)
    g = host(cg)
    for c0 in (0, 2000):
        sl = slice(c0, c0 + 16)
        ref, _, _ = O.gibbs_range(h, J, ch0[sl], c0, q, 1, 3004)
        check_chains(h, J, ch0[sl], g[sl], ref, q, 1, 3004, c0=c0)
    # unit-weight statistics of these chains: bit-exact sampled entries
    f1, f2, _ = api.stats(cg, q, None, 0.0, "bf16x2")
    r1, r2 = sample_pairs(L * q, 500, 9)
    assert np.array_equal(host(f2)[r1, r2], O.stats_entries(g, q, r1, r2, None, 0.0))


@pytest.mark.parametrize("L,q,N", [(256, 21, 20000), (512, 21, 4096), (400, 5, 10000)])
def test_direct_chain_counts_full_size(L, q, N):
    """The epoch's chain counts at full sizes (the precision-form shape, the
    largest model, the RNA shape): with h = J = 0, zero data frequencies and
    no sweeps, the update writes J'[r1][r2] = float32(lr (0 - C/N)) for sites
    i != j, so sampled entries pin C against the oracle's counts of the same
    chains; the whole h and J equal those of the one-hot product path bit for
    bit. (The Pearson value is 0/0 here, so no device flag is read.)"""
    Lq, lr = L * q, 0.05
    ch0 = O.init_chains(N, L, q, seed=5100 + L)
    f1 = torch.zeros(Lq, dtype=torch.float64, device="cuda")
    f2 = torch.zeros(Lq * Lq, dtype=torch.float64, device="cuda")
    outs = []
    for prec in (B.PREC_FP32, B.PREC_BF16X2 | B.COUNTS_PRODUCT):
        hg = torch.zeros((L, q), dtype=torch.float32, device="cuda")
        Jg = torch.zeros((Lq, Lq), dtype=torch.float32, device="cuda")
        api.train_step(hg, Jg, dev(ch0), f1, f2, lr, 0, 1, 0, prec=prec)
        outs.append((hg, Jg))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    r1, r2 = sample_pairs(Lq, 600, L)
    keep = (r1 // q) != (r2 // q)
    r1, r2 = r1[keep], r2[keep]
    p = O.stats_entries(ch0, q, r1, r2, None, 0.0)
    want = (lr * (0.0 - p)).astype(np.float32)
    got = host(outs[0][1])[r1, r2]
    assert np.array_equal(got, want)
    del outs
    torch.cuda.empty_cache()


# ---------------------------------------------------------------- launches split in chunks
def test_local_fields_past_one_launch():
    """More (chain, column block) workgroups than one launch takes (2^22):
    4 197 304 chains of an L = 20, q = 2 model (one column block each) are
    built in two launches; chains at both ends of each launch match the
    oracle's fields."""
    L, q = 20, 2
    N = (1 << 22) + 3000
    h, J = synth.planted_dense(L, q, seed=1201, sigma_J=0.3)
    ch = api.init_chains(N, L, q, 1202)
    H = torch.empty(api.workspace_bytes(B.WS_GIBBS, N, L, q, B.SAMPLER_FIELDS) // 4,
                    dtype=torch.float32, device="cuda")
    api.gibbs(dev(h), dev(J), ch, sweeps=0, seed=0, H_ws=H, sampler="fields")
    g = np.random.default_rng(1203)
    picks = [0, 1, (1 << 22) - 1, 1 << 22, (1 << 22) + 1, N - 1] + list(g.integers(0, N, 20))
    for c in picks:
        Hg = host(H[c * L * q:(c + 1) * L * q])
        Ho = O.local_fields(h, J, host(ch[c]), q)
        assert np.all(np.abs(Hg - Ho) <= 1e-5 * (1 + np.abs(Ho))), c


# ---------------------------------------------------------------- batches past 2^31 bytes
def test_energy_batch_beyond_2gib_of_tokens():
    """40 million sequences at L = 64: the transposed tokens (L x B bytes)
    pass 2^31, so every 32-bit offset over the whole array would overflow;
    sampled energies, the last sequences among them, follow the oracle."""
    L, q, Bn = 64, 21, 40_000_000
    h, J = synth.planted_dense(L, q, seed=1011, sigma_J=0.05)
    gen = torch.Generator(device="cuda").manual_seed(12)
    S = torch.randint(0, q, (Bn, L), generator=gen, dtype=torch.int64, device="cuda").to(torch.int8)
    E = api.energy(dev(h), dev(J), S)
    idx = np.concatenate([[0, 1, Bn // 2, Bn - 2, Bn - 1],
                          np.random.default_rng(13).integers(0, Bn, 40)])
    sel = torch.from_numpy(idx).cuda()
    Eg = host(E[sel])
    Ss = host(S[sel])
    del S, E
    torch.cuda.empty_cache()
    Eo = O.energy(h, J, Ss, q)
    assert np.all(np.abs(Eg - Eo) <= 1e-4 * np.abs(Eo).max())


# ---------------------------------------------------------------- largest served model
def test_largest_model_scores():
    L, q = 512, 21
    h, J = synth.planted_dense(L, q, seed=1005, sigma_J=0.02)
    S = synth.random_sequences(1500, L, q, 10)
    E = host(api.energy(dev(h), dev(J), dev(S)))
    Eo = O.energy(h, J, S, q)
    assert np.abs(E - Eo).max() <= 1e-4 * np.abs(Eo).max()
    wt = S[:2]
    dE = host(api.single_mutant_scan(dev(h), dev(J), dev(wt))).reshape(2, L, q)
    g = np.random.default_rng(11)
    for b in range(2):
        e0 = O.energy(h, J, wt[b:b + 1], q)[0]
        for _ in range(40):
            i, a = int(g.integers(L)), int(g.integers(q))
            t = wt[b].copy()
            t[i] = a
            ref = O.energy(h, J, t[None], q)[0] - e0
            assert abs(dE[b, i, a] - ref) <= 1e-4 * (1 + abs(e0))
    F, Fa = api.apc_frobenius(dev(J), L, q, 0)
    Fo, Fao = O.apc_frobenius(J, L, q, 0)
    assert np.abs(host(Fa) - Fao).max() <= 1e-5 * np.abs(Fo).max()


def test_served_sampling_shape_streams():
    """The largest served model's sampling shape: 10 000 chains of three
    requests (own keys, chain indices and sweep offsets) at L = 512, q = 21 in
    one bmdca_gibbs_streams launch sized for a 32-CU share, 2 sweeps; sampled
    chains of every request follow the oracle's trajectories."""
    L, q = 512, 21
    h, J = synth.planted_dense(L, q, seed=1006, sigma_J=0.02)
    sizes, seeds, offs = [6000, 3000, 1000], [5001, 5002, 5003], [0, 17, 40]
    ch0 = O.init_chains(sum(sizes), L, q, seed=3040)
    sd = np.repeat(seeds, sizes).astype(np.uint64)
    of = np.repeat(offs, sizes).astype(np.uint64)
    ids = np.concatenate([np.arange(n) for n in sizes]).astype(np.uint32)
    cg = dev(ch0)
    api.gibbs_streams(dev(h), dev(J), cg, 2, api.chain_streams(sd, of, ids), cus=32)
    g = host(cg)
    pick = np.concatenate([np.arange(0, 8), np.arange(5995, 6005), np.arange(7490, 7498),
                           np.arange(9992, 10000)])
    ref = np.stack([O.gibbs_range(h, J, ch0[k:k + 1], int(ids[k]), q, 2, int(sd[k]),
                                  sweep_offset=int(of[k]))[0][0] for k in pick])
    bad = check_chains(h, J, ch0[pick], g[pick], ref, q, 2, 0, ids=ids[pick], seeds=sd[pick],
                       offsets=of[pick])
    assert len(bad) <= 2


# ---------------------------------------------------------------- edge cases
def test_edge_single_chain_two_sites():
    L, q = 2, 2
    h, J = synth.planted_dense(L, q, seed=12, sigma_J=0.5)
    ch0 = O.init_chains(1, L, q, seed=13)
    for sampler in ("gather", "fields"):
        cg = dev(ch0)
        api.gibbs(dev(h), dev(J), cg, 5, seed=14, sampler=sampler)
        ref, _, _ = O.gibbs(h, J, ch0, q, 5, 14)
        check_chains(h, J, ch0, host(cg), ref, q, 5, 14)
    X = ch0
    f1, f2, _ = api.stats(dev(X), q, None, -1.0)
    o1, o2, _ = O.stats(X, q, None, -1.0)
    assert np.array_equal(host(f1), o1) and np.array_equal(host(f2), o2)
    n, w, meff = api.reweight(dev(X), q, 0.8)
    assert host(n)[0] == 1 and host(meff)[0] == 1.0
    hg, Jg = dev(h), dev(J)
    f1d, f2d = dev(o1), dev(o2)
    e = torch.zeros(1, dtype=torch.int32, device="cuda")
    pr = api.train_step(hg, Jg, dev(ch0), f1d, f2d, 0.05, 2, 15, 0, dev_err=e)
    # one chain has no connected correlations: the Pearson coefficient is 0/0
    # on both sides (flagged), the parameters stay finite
    _, _, _, r, _, _ = O.train_step(h, J, ch0, o1, o2, q, 0.05, 2, 15, 0)
    assert np.isnan(r) and np.isnan(host(pr)[0])
    assert int(host(e)[0]) == B.DEVERR_NONFINITE
    assert np.isfinite(host(hg)).all() and np.isfinite(host(Jg)).all()


def test_edge_empty_batch_and_zero_sweeps():
    L, q = 30, 21
    h, J = synth.planted_dense(L, q, seed=16, sigma_J=0.1)
    out = api.energy(dev(h), dev(J), torch.empty((0, L), dtype=torch.int8, device="cuda"))
    assert out.numel() == 0
    ch0 = O.init_chains(70, L, q, seed=17)
    for sampler in ("gather", "fields"):
        cg = dev(ch0)
        api.gibbs(dev(h), dev(J), cg, 0, seed=18, sampler=sampler)
        assert np.array_equal(host(cg), ch0)


def test_edge_ragged_tiles_and_tail_rows():
    """Lq not a multiple of the 128-wide tiles, M not a multiple of the 64-row
    stage, single-row alignment."""
    for (L, q, M) in [(13, 11, 1), (13, 11, 65), (29, 7, 1000)]:
        X = synth.clustered_msa(M, L, q, seed=19 + M)
        w = synth.weights_open_unit(M, 20)
        for prec in ("fp32", "bf16x2"):
            f1, f2, _ = api.stats(dev(X), q, None, -1.0, prec)
            o1, o2, _ = O.stats(X, q, None, -1.0)
            assert np.array_equal(host(f2), o2)
            g1, g2, _ = api.stats(dev(X), q, dev(w), 0.3, prec)
            p1, p2, _ = O.stats(X, q, w, 0.3)
            assert np.abs(host(g2) - p2).max() <= 1e-5
