"""Seeded synthetic inputs for tests and benchmarks.

This module only draws random numbers and arranges them into the shapes of the
method's inputs (Potts parameters, aligned sequences, weights). It contains none
of the method's arithmetic: no energies, no sampling, no statistics. Both the
HIP path and the CPU oracle are fed from here.

Shapes follow the model of Sec. 2.1 (Eq. 1): tokens are int8 in 0..q-1 with
token 0 the alignment gap (Table 1 lists the gap first); fields h are float32
[L, q]; couplings J are float32 [L*q, L*q], stored full-symmetric
(J[(i,a),(j,b)] == J[(j,b),(i,a)]) with zero diagonal blocks J_ii (Sec. 2.1).
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(int(seed))


def symmetric_couplings(blocks: dict, L: int, q: int) -> np.ndarray:
    """Assemble full-symmetric J from upper-triangle blocks {(i, j): q x q}, i < j."""
    J = np.zeros((L, q, L, q), dtype=np.float32)
    for (i, j), B in blocks.items():
        assert i < j
        J[i, :, j, :] = B
        J[j, :, i, :] = B.T
    return J.reshape(L * q, L * q)


def planted_dense(L: int, q: int, seed: int, sigma_h: float = 1.0,
                  sigma_J: float = 0.1):
    """h ~ N(0, sigma_h), every pair i<j has a q x q block ~ N(0, sigma_J).

    The second argument of N(., .) is read as a standard deviation.
    """
    g = _rng(seed)
    h = g.normal(0.0, sigma_h, size=(L, q)).astype(np.float32)
    iu = np.triu_indices(L, 1)
    B = g.normal(0.0, sigma_J, size=(len(iu[0]), q, q)).astype(np.float32)
    J = np.zeros((L, q, L, q), dtype=np.float32)
    J[iu[0], :, iu[1], :] = B
    J[iu[1], :, iu[0], :] = np.transpose(B, (0, 2, 1))
    return h, J.reshape(L * q, L * q)


def planted_sparse(L: int, q: int, seed: int, n_pairs: int | None = None,
                   sigma_J: float = 0.5, gap_mass: float = 0.15):
    """Sparse-contact model: n_pairs (default 3L) random pairs i<j carry
    q x q blocks ~ N(0, sigma_J); all other blocks are zero.

    Fields: h_i(a) ~ N(0, 1) for a != 0, and the gap field is set so that the
    independent-site (J = 0) profile gives the gap exactly `gap_mass`:
    exp(h_i(0)) / sum_a exp(h_i(a)) == gap_mass.
    """
    g = _rng(seed)
    n_pairs = 3 * L if n_pairs is None else int(n_pairs)
    allpairs = np.array(np.triu_indices(L, 1)).T
    pick = g.choice(len(allpairs), size=min(n_pairs, len(allpairs)), replace=False)
    h = g.normal(0.0, 1.0, size=(L, q))
    rest = np.log(np.exp(h[:, 1:]).sum(axis=1))
    h[:, 0] = np.log(gap_mass / (1.0 - gap_mass)) + rest
    blocks = {}
    for k in sorted(pick.tolist()):
        i, j = (int(x) for x in allpairs[k])
        blocks[(i, j)] = g.normal(0.0, sigma_J, size=(q, q)).astype(np.float32)
    return h.astype(np.float32), symmetric_couplings(blocks, L, q)


def random_sequences(B: int, L: int, q: int, seed: int) -> np.ndarray:
    """B sequences of L tokens, each token uniform on 0..q-1 (int8 [B, L])."""
    return _rng(seed).integers(0, q, size=(B, L), dtype=np.int8)


def clustered_msa(M: int, L: int, q: int, seed: int, n_families: int = 8,
                  mut_rate: float = 0.15, gap_frac: float = 0.15) -> np.ndarray:
    """An alignment with phylogeny-like redundancy.

    A few random ancestors are drawn; every sequence copies one ancestor (and
    sometimes a previous sequence of the same family) and resamples each
    position with probability `mut_rate`, a resampled position being a gap with
    probability `gap_frac`. Near-duplicates make identity-based weights
    non-trivial.
    """
    g = _rng(seed)
    anc = g.integers(1, q, size=(n_families, L), dtype=np.int8)
    X = np.empty((M, L), dtype=np.int8)
    fam = g.integers(0, n_families, size=M)
    for m in range(M):
        base = anc[fam[m]]
        if m > 0 and g.random() < 0.5:
            prev = np.nonzero(fam[:m] == fam[m])[0]
            if len(prev):
                base = X[g.choice(prev)]
        s = base.copy()
        mut = g.random(L) < mut_rate
        k = int(mut.sum())
        if k:
            new = g.integers(1, q, size=k, dtype=np.int8)
            gaps = g.random(k) < gap_frac
            new[gaps] = 0
            s[mut] = new
        X[m] = s
    return X


def weights_open_unit(M: int, seed: int) -> np.ndarray:
    """Non-uniform float weights in (0, 1]: w = 1 - U[0, 1) (float64 [M])."""
    return 1.0 - _rng(seed).random(M)


def mutate(seqs: np.ndarray, q: int, n_mut: int, seed: int) -> np.ndarray:
    """Copies of `seqs` with n_mut random positions per row set to random tokens."""
    g = _rng(seed)
    out = seqs.copy()
    B, L = out.shape
    for b in range(B):
        pos = g.choice(L, size=min(n_mut, L), replace=False)
        out[b, pos] = g.integers(0, q, size=len(pos), dtype=np.int8)
    return out
