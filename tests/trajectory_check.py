"""Trajectory parity under shared Philox counters.

The GPU samplers form the local fields in FP32 and the oracle in FP64, so a
visit whose uniform lies within BOUNDARY of a threshold (a CDF step of the
Gibbs draw, or min(1, p) of the Metropolis test) may be resolved either way.
A chain whose end state differs from the oracle's is excused only when the
oracle, replayed on that chain with the other outcome taken at some of its
near-threshold visits (at most `depth` of them), ends exactly where the GPU
chain ended.  Any other difference is an error.
"""
import numpy as np

from oracle import oracle as O

BOUNDARY = 1e-5  # a uniform this close to a threshold may fall either way (FP32 vs FP64)


def reproduces(h, J, s0, target, c, q, sweeps, seed, sweep_offset=0, beta=1.0,
               metropolis=False, depth=3):
    """True if some choice of other outcomes at <= depth near-threshold visits
    of chain c (global index), replayed by the oracle from s0, ends in target."""
    L = len(s0)
    nv = sweeps * L
    target = np.asarray(target, dtype=np.int8)

    def search(force, start, d):
        end, drawn, lo, hi = O.chain_forced(h, J, s0, c, q, sweeps, seed, sweep_offset, beta,
                                            metropolis, BOUNDARY, force)
        if np.array_equal(end, target):
            return True
        if d == 0:
            return False
        close = np.nonzero((lo != drawn) | (hi != drawn))[0]
        for v in close[close >= start]:
            for a in range(int(lo[v]), int(hi[v]) + 1):
                if a == drawn[v]:
                    continue
                f = force.copy()
                f[v] = a
                if search(f, v + 1, d - 1):
                    return True
        return False

    return search(np.full(nv, -1, dtype=np.int8), 0, depth)


def check_chains(h, J, ch0, gpu, orc, q, sweeps, seed, sweep_offset=0, beta=1.0,
                 metropolis=False, c0=0, ids=None, seeds=None, offsets=None, depth=3):
    """Every chain k whose GPU end state gpu[k] differs from the oracle's orc[k]
    must be reproduced by a boundary replay from ch0[k] (chain index ids[k] or
    c0 + k, key seeds[k] or seed, first sweep offsets[k] or sweep_offset).
    Returns the indices of the excused chains."""
    gpu = np.asarray(gpu)
    bad = np.nonzero((gpu != orc).any(axis=1))[0]
    for k in bad:
        c = int(ids[k]) if ids is not None else c0 + int(k)
        sd = int(seeds[k]) if seeds is not None else seed
        off = int(offsets[k]) if offsets is not None else sweep_offset
        assert reproduces(h, J, ch0[k], gpu[k], c, q, sweeps, sd, off, beta, metropolis, depth), (
            f"chain {k} (index {c}) left the oracle's trajectory where no boundary event "
            f"explains it")
    return bad
