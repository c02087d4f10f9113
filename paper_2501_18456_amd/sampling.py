"""Sampling from a trained model in equilibrium (Sec. 4.1 of the paper).

The routine first measures the mixing time t_mix of the model: `nmeasure`
chains start from data sequences drawn according to their weights; after
t = 1, 2, 4, 8, ... sweeps it records

  SeqID(t)       mean and standard deviation of SeqID(a_k(t), a_sigma(k)(t)),
                 the chains against a permutation sigma of themselves,
  SeqID(t, t/2)  the same for SeqID(a_k(t), a_k(t/2)), the chains against
                 their state at the previous checkpoint (t/2; the data start
                 for t = 1),

with SeqID(a, b) = (1/L) sum_i [a_i == b_i], and stops at the first t where
the two means are within the sum of their errors of the mean (std / sqrt(n)):
the curves have merged, the chains have forgotten their start.  Then `ngen`
chains start uniformly at random and run nmix * t_mix sweeps.

Every step runs in the HIP library (weighted row draw, row gather, Gibbs
sweeps, SeqID sums); this module only sequences the calls and reads back two
doubles per checkpoint.  Random streams: the row draw and the measuring
chains use key `seed`; the generated chains use key `seed + 1`.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import api


def default_permutation(n: int, seed: int) -> np.ndarray:
    """The permutation sigma of SeqID(t): uniformly random, seeded."""
    return np.random.default_rng(seed).permutation(n).astype(np.int32)


def mixing_time(h, J, msa, w, nmeasure: int, seed: int, perm=None, max_sweeps: int = 10000,
                beta: float = 1.0, sampler: str = "auto"):
    """Returns (t_mix or None if not reached within max_sweeps, records
    [(t, SeqID(t) mean, std, SeqID(t, t/2) mean, std)], chains at the end)."""
    L, q = api._model(h, J)
    n = int(min(nmeasure, msa.shape[0]))
    dev = msa.device
    if perm is None:
        perm = default_permutation(n, seed)
    perm_d = torch.from_numpy(np.ascontiguousarray(perm, dtype=np.int32)).to(dev)
    rows = api.draw_rows(w, n, seed)
    A = api.gather_rows(msa, rows)
    prev = A.clone()
    out = torch.empty(4, dtype=torch.float64, device=dev)

    def overlaps(ref):
        api.seqid(A, A, perm_d, out=out[0:2])
        api.seqid(A, ref, None, out=out[2:4])
        return out.cpu().tolist()

    m1, s1, _, _ = overlaps(A)
    records = [(0, m1, s1, 1.0, 0.0)]
    t_prev, t = 0, 1
    H = api.workspace(api.B.WS_GIBBS, n, L, q, api._sampler(sampler), dev)
    while t <= max_sweeps:
        api.gibbs(h, J, A, t - t_prev, seed, sweep_offset=t_prev, beta=beta, H_ws=H,
                  sampler=sampler)
        m1, s1, m2, s2 = overlaps(prev)
        records.append((t, m1, s1, m2, s2))
        if abs(m2 - m1) <= (s1 + s2) / math.sqrt(n):
            return t, records, A
        prev.copy_(A)
        t_prev, t = t, 2 * t
    return None, records, A


def sample_equilibrium(h, J, msa, w, nmeasure: int, ngen: int, seed: int, nmix: int = 2,
                       max_sweeps: int = 10000, beta: float = 1.0, sampler: str = "auto",
                       perm=None):
    """Measures t_mix, then returns (ngen chains after nmix * t_mix sweeps
    from a uniform start, t_mix, records).  If the curves did not merge
    within max_sweeps, the chains run nmix * max_sweeps sweeps and t_mix is
    returned as None."""
    L, q = api._model(h, J)
    t_mix, records, _ = mixing_time(h, J, msa, w, nmeasure, seed, perm, max_sweeps, beta, sampler)
    t_eq = (t_mix if t_mix is not None else max_sweeps) * nmix
    chains = api.init_chains(ngen, L, q, seed + 1, device=msa.device)
    api.gibbs(h, J, chains, t_eq, seed + 1, beta=beta, sampler=sampler)
    return chains, t_mix, records
