"""Python view of the FP64 CPU oracle (bmdca_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product path. It shares no
code with the HIP library; it implements the same written definitions of the
method (adabmDCA 2.0, arXiv:2501.18456) independently, in double precision.

Every function takes and returns numpy arrays. Parameters follow the storage
conventions of the library: h float32 [L, q] (or flat L*q), J float32
[L*q, L*q] full-symmetric with zero diagonal blocks, tokens int8 0..q-1.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bmdca_oracle.c")
_LIB = os.path.join(_HERE, "libbmdca_oracle.so")
_LIB_OMP = os.path.join(_HERE, "libbmdca_oracle_omp.so")


def _compile(out: str, extra, force: bool) -> str:
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               *extra, "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, contraction off) into oracle/: the
    single-threaded library the tests use, and an OpenMP build (chains spread
    over threads, same results) used only to time the oracle on all host
    cores."""
    _compile(_LIB_OMP, ["-fopenmp"], force)
    return _compile(_LIB, [], force)


_lib = None
_lib_omp = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _declare(_lib)
    return _lib


def lib_threads():
    """The OpenMP build (OMP_NUM_THREADS threads): the CPU-baseline timing leg."""
    global _lib_omp
    if _lib_omp is None:
        build()
        _lib_omp = C.CDLL(_LIB_OMP)
        _declare(_lib_omp)
    return _lib_omp


_p = C.c_void_p
_i32, _i64, _u64, _f64 = C.c_int32, C.c_int64, C.c_uint64, C.c_double


def _declare(L):
    sig = {
        "orc_philox4x32_10": (None, [_p, _p, _p]),
        "orc_gibbs_uniform": (_f64, [_u64, _u64, _u64, _i32]),
        "orc_init_chains": (None, [_p, _i64, _i32, _i32, _u64]),
        "orc_identity_threshold": (_i32, [_f64, _i32]),
        "orc_reweight": (None, [_p, _i64, _i32, _f64, _p, _p, _p]),
        "orc_stats": (None, [_p, _p, _i64, _i32, _i32, _f64, _p, _p, _p]),
        "orc_energy_one": (_f64, [_p, _p, _p, _i32, _i32]),
        "orc_energy": (None, [_p, _p, _p, _i64, _i32, _i32, _p]),
        "orc_local_field": (None, [_p, _p, _p, _i32, _i32, _i32, _p]),
        "orc_local_fields_all": (None, [_p, _p, _p, _i32, _i32, _p]),
        "orc_gibbs": (None, [_p, _p, _p, _i64, _i32, _i32, _i32, _u64, _u64, _f64, _p, _p]),
        "orc_gibbs_range": (None, [_p, _p, _p, _i64, _i64, _i32, _i32, _i32, _u64, _u64, _f64, _p,
                                   _p]),
        "orc_chain_freqs": (None, [_p, _i64, _i32, _i32, _p, _p]),
        "orc_pearson": (_f64, [_p, _p, _p, _p, _i32, _i32]),
        "orc_update": (None, [_p, _p, _p, _p, _p, _p, _i32, _i32, _f64]),
        "orc_train_step": (_f64, [_p, _p, _p, _i64, _i32, _i32, _p, _p, _f64, _i32, _u64,
                                  _u64, _p, _p]),
        "orc_mutant_scan": (None, [_p, _p, _p, _i32, _i32, _p]),
        "orc_apc_frobenius": (None, [_p, _i32, _i32, _i32, _p, _p]),
        "orc_enumerate": (C.c_int, [_p, _p, _i32, _i32, _f64, _p, _p, _p]),
        "orc_reweight_rows": (None, [_p, _i64, _i32, _f64, _p, _i64, _p]),
        "orc_stats_entries": (None, [_p, _p, _i64, _i32, _i32, _f64, _p, _p, _i64, _p]),
        "orc_draw_rows": (None, [_p, _i64, _i64, _u64, _p, _p]),
        "orc_metropolis_range": (None, [_p, _p, _p, _i64, _i64, _i32, _i32, _i32, _u64, _u64,
                                        _f64, _p, _p]),
        "orc_seqid": (None, [_p, _p, _p, _i64, _i32, _p]),
        "orc_skl_element": (_f64, [_f64, _f64]),
        "orc_decimate": (_i64, [_p, _p, _p, _i64, _i32, _i32, _f64, _f64]),
        "orc_bernoulli_kl": (_f64, [_f64, _f64]),
        "orc_activate": (_i64, [_p, _p, _i64, _i32, _i32, _p, _f64]),
        "orc_chain_forced": (None, [_p, _p, _p, _u64, _i32, _i32, _i32, _u64, _u64, _f64, _i32,
                                    _f64, _p, _p, _p, _p]),
        "orc_profile_fields": (None, [_p, _i32, _i32, _p]),
        "orc_mask_apply": (_i64, [_p, _p, _i32, _i32]),
        "orc_train_step_masked": (_f64, [_p, _p, _p, _p, _i64, _i32, _i32, _p, _p, _f64, _i32,
                                         _u64, _u64, _p, _p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i8(a):
    return np.ascontiguousarray(a, dtype=np.int8)


# --------------------------------------------------------------------------
# Philox4x32-10 (Salmon et al., SC'11)
# --------------------------------------------------------------------------
def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def gibbs_uniform(seed: int, c: int, sg: int, i: int) -> float:
    return lib().orc_gibbs_uniform(seed, c, sg, i)


def init_chains(N: int, L: int, q: int, seed: int) -> np.ndarray:
    ch = np.zeros((N, L), dtype=np.int8)
    lib().orc_init_chains(_ptr(ch), N, L, q, seed)
    return ch


# --------------------------------------------------------------------------
# Pre-processing (Sec. 2.3)
# --------------------------------------------------------------------------
def identity_threshold(theta: float, L: int) -> int:
    return lib().orc_identity_threshold(theta, L)


def reweight(msa, theta: float = 0.8):
    msa = _i8(msa)
    M, L = msa.shape
    n = np.zeros(M, dtype=np.int32)
    w = np.zeros(M, dtype=np.float64)
    meff = np.zeros(1, dtype=np.float64)
    lib().orc_reweight(_ptr(msa), M, L, theta, _ptr(n), _ptr(w), _ptr(meff))
    return n, w, float(meff[0])


def stats(X, q: int, w=None, pseudocount: float = -1.0):
    """Returns (f1 [L*q], f2 [Lq, Lq], meff)."""
    X = _i8(X)
    M, L = X.shape
    Lq = L * q
    f1 = np.zeros(Lq, dtype=np.float64)
    f2 = np.zeros((Lq, Lq), dtype=np.float64)
    meff = np.zeros(1, dtype=np.float64)
    wv = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    lib().orc_stats(_ptr(X), _ptr(wv), M, L, q, pseudocount, _ptr(f1), _ptr(f2), _ptr(meff))
    return f1, f2, float(meff[0])


def reweight_rows(msa, rows, theta: float = 0.8):
    """N^(m) of Eq. (7) for the listed rows only."""
    msa = _i8(msa)
    M, L = msa.shape
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.zeros(len(rows), dtype=np.int32)
    lib().orc_reweight_rows(_ptr(msa), M, L, theta, _ptr(rows), len(rows), _ptr(out))
    return out


def stats_entries(X, q: int, r1, r2, w=None, pseudocount: float = -1.0):
    """Entries f2'[r1[k], r2[k]] of the pseudocounted two-site table."""
    X = _i8(X)
    M, L = X.shape
    r1 = np.ascontiguousarray(r1, dtype=np.int64)
    r2 = np.ascontiguousarray(r2, dtype=np.int64)
    out = np.zeros(len(r1), dtype=np.float64)
    wv = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    lib().orc_stats_entries(_ptr(X), _ptr(wv), M, L, q, pseudocount, _ptr(r1), _ptr(r2),
                            len(r1), _ptr(out))
    return out


# --------------------------------------------------------------------------
# Energies and fields (Eq. 1)
# --------------------------------------------------------------------------
def energy(h, J, seqs, q: int):
    h, J, seqs = _f32(h), _f32(J), _i8(seqs)
    B, L = seqs.shape
    E = np.zeros(B, dtype=np.float64)
    lib().orc_energy(_ptr(h), _ptr(J), _ptr(seqs), B, L, q, _ptr(E))
    return E


def local_fields(h, J, s, q: int):
    h, J, s = _f32(h), _f32(J), _i8(s)
    L = s.shape[0]
    H = np.zeros(L * q, dtype=np.float64)
    lib().orc_local_fields_all(_ptr(h), _ptr(J), _ptr(s), L, q, _ptr(H))
    return H


# --------------------------------------------------------------------------
# Sampling and learning (Sec. 2.1)
# --------------------------------------------------------------------------
def gibbs(h, J, chains, q: int, sweeps: int, seed: int, sweep_offset: int = 0,
          beta: float = 1.0, want_margins: bool = False):
    """Returns (new chains, margins [N, sweeps, L] or None, flips)."""
    h, J = _f32(h), _f32(J)
    ch = _i8(chains).copy()
    N, L = ch.shape
    mg = np.zeros((N, sweeps, L), dtype=np.float64) if want_margins else None
    flips = np.zeros(1, dtype=np.int64)
    lib().orc_gibbs(_ptr(h), _ptr(J), _ptr(ch), N, L, q, sweeps, seed, sweep_offset,
                    float(beta), _ptr(mg), _ptr(flips))
    return ch, mg, int(flips[0])


def gibbs_range(h, J, chains, c0: int, q: int, sweeps: int, seed: int, sweep_offset: int = 0,
                beta: float = 1.0, want_margins: bool = False):
    """As gibbs(), for chains whose global indices are c0, c0+1, ..."""
    h, J = _f32(h), _f32(J)
    ch = _i8(chains).copy()
    N, L = ch.shape
    mg = np.zeros((N, sweeps, L), dtype=np.float64) if want_margins else None
    flips = np.zeros(1, dtype=np.int64)
    lib().orc_gibbs_range(_ptr(h), _ptr(J), _ptr(ch), N, c0, L, q, sweeps, seed, sweep_offset,
                          float(beta), _ptr(mg), _ptr(flips))
    return ch, mg, int(flips[0])


def metropolis(h, J, chains, q: int, sweeps: int, seed: int, sweep_offset: int = 0,
               beta: float = 1.0, want_margins: bool = False, c0: int = 0):
    """Single-site Metropolis sweeps. Returns (new chains, margins or None, flips)."""
    h, J = _f32(h), _f32(J)
    ch = _i8(chains).copy()
    N, L = ch.shape
    mg = np.zeros((N, sweeps, L), dtype=np.float64) if want_margins else None
    flips = np.zeros(1, dtype=np.int64)
    lib().orc_metropolis_range(_ptr(h), _ptr(J), _ptr(ch), N, c0, L, q, sweeps, seed,
                               sweep_offset, float(beta), _ptr(mg), _ptr(flips))
    return ch, mg, int(flips[0])


def chain_forced(h, J, s0, c: int, q: int, sweeps: int, seed: int, sweep_offset: int = 0,
                 beta: float = 1.0, metropolis: bool = False, tol: float = 0.0, force=None):
    """One chain (global index c) replayed with forced outcomes: force[v] >= 0
    replaces the drawn state at visit v = sweep*L + site.  Returns (end state,
    drawn [sweeps*L], alt_lo, alt_hi): the states each visit could take had
    every comparison within tol of its threshold gone the other way."""
    h, J = _f32(h), _f32(J)
    s = _i8(s0).copy()
    L = s.shape[0]
    nv = sweeps * L
    drawn = np.zeros(nv, dtype=np.int8)
    lo = np.zeros(nv, dtype=np.int8)
    hi = np.zeros(nv, dtype=np.int8)
    fv = None if force is None else np.ascontiguousarray(force, dtype=np.int8)
    lib().orc_chain_forced(_ptr(h), _ptr(J), _ptr(s), c, L, q, sweeps, seed, sweep_offset,
                           float(beta), int(bool(metropolis)), float(tol), _ptr(fv), _ptr(drawn),
                           _ptr(lo), _ptr(hi))
    return s, drawn, lo, hi


def chain_freqs(chains, q: int):
    ch = _i8(chains)
    N, L = ch.shape
    p1 = np.zeros(L * q, dtype=np.float64)
    p2 = np.zeros((L * q, L * q), dtype=np.float64)
    lib().orc_chain_freqs(_ptr(ch), N, L, q, _ptr(p1), _ptr(p2))
    return p1, p2


def pearson(f1, f2, p1, p2, L: int, q: int) -> float:
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (f1, f2, p1, p2)]
    return lib().orc_pearson(*[_ptr(x) for x in a], L, q)


def update(h, J, f1, f2, p1, p2, L: int, q: int, lr: float):
    """Eq. (5) update; returns new (h, J) as float32 copies."""
    h = _f32(h).copy()
    J = _f32(J).copy()
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (f1, f2, p1, p2)]
    lib().orc_update(_ptr(h), _ptr(J), *[_ptr(x) for x in a], L, q, lr)
    return h, J


def train_step(h, J, chains, f1, f2, q: int, lr: float, sweeps: int, seed: int,
               epoch: int, want_margins: bool = False, threads: bool = False):
    """One epoch. Returns (h', J', chains', pearson, margins, flips).
    threads=True runs the OpenMP build (the same results)."""
    h = _f32(h).copy()
    J = _f32(J).copy()
    ch = _i8(chains).copy()
    N, L = ch.shape
    f1 = np.ascontiguousarray(f1, dtype=np.float64)
    f2 = np.ascontiguousarray(f2, dtype=np.float64)
    mg = np.zeros((N, sweeps, L), dtype=np.float64) if want_margins else None
    flips = np.zeros(1, dtype=np.int64)
    lb = lib_threads() if threads else lib()
    r = lb.orc_train_step(_ptr(h), _ptr(J), _ptr(ch), N, L, q, _ptr(f1), _ptr(f2), lr,
                          sweeps, seed, epoch, _ptr(mg), _ptr(flips))
    return h, J, ch, r, mg, int(flips[0])


# --------------------------------------------------------------------------
# Applications (Sec. 4)
# --------------------------------------------------------------------------
def mutant_scan(h, J, wt, q: int):
    h, J, wt = _f32(h), _f32(J), _i8(wt)
    L = wt.shape[0]
    dE = np.zeros(L * q, dtype=np.float64)
    lib().orc_mutant_scan(_ptr(h), _ptr(J), _ptr(wt), L, q, _ptr(dE))
    return dE


def apc_frobenius(J, L: int, q: int, gap: int = 0):
    J = _f32(J)
    F = np.zeros((L, L), dtype=np.float64)
    Fa = np.zeros((L, L), dtype=np.float64)
    lib().orc_apc_frobenius(_ptr(J), L, q, gap, _ptr(F), _ptr(Fa))
    return F, Fa


def enumerate_exact(h, J, L: int, q: int, beta: float = 1.0):
    """Exact marginals by enumeration of all q^L states: (p1, p2, logZ)."""
    h, J = _f32(h), _f32(J)
    p1 = np.zeros(L * q, dtype=np.float64)
    p2 = np.zeros((L * q, L * q), dtype=np.float64)
    lz = np.zeros(1, dtype=np.float64)
    rc = lib().orc_enumerate(_ptr(h), _ptr(J), L, q, beta, _ptr(p1), _ptr(p2), _ptr(lz))
    if rc != 0:
        raise ValueError("q^L too large for enumeration")
    return p1, p2, float(lz[0])


# --------------------------------------------------------------------------
# Equilibrium sampling and its convergence criterion (Sec. 4.1)
# --------------------------------------------------------------------------
def draw_rows(w, n: int, seed: int, want_margins: bool = False):
    """n row indices drawn with replacement, row m with probability w_m / sum w."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    rows = np.zeros(n, dtype=np.int32)
    mg = np.zeros(n, dtype=np.float64) if want_margins else None
    lib().orc_draw_rows(_ptr(w), w.size, n, seed, _ptr(rows), _ptr(mg))
    return (rows, mg) if want_margins else rows


def seqid(A, B, perm=None):
    """(mean, std) of SeqID(A[k], B[perm[k]]) over the rows k."""
    A, B = _i8(A), _i8(B)
    out = np.zeros(2, dtype=np.float64)
    pr = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
    lib().orc_seqid(_ptr(A), _ptr(B), _ptr(pr), A.shape[0], A.shape[1], _ptr(out))
    return float(out[0]), float(out[1])


def mixing_time(h, J, msa, w, q: int, nmeasure: int, seed: int, perm, max_sweeps: int = 10000,
                beta: float = 1.0):
    """Mixing time of Sec. 4.1: nmeasure chains start from data rows drawn by
    weight; at t = 0, 1, 2, 4, ... sweeps SeqID(t) (chains vs the permuted
    chains) and SeqID(t, t/2) (chains vs the previous checkpoint) are
    recorded; t_mix is the first t where the two means are within the sum of
    their errors of the mean.  Returns (t_mix or None, records [(t, mean1,
    std1, mean2, std2)], chains)."""
    n = int(min(nmeasure, np.shape(msa)[0]))  # min(nmeasure, data size), as the paper's table states
    rows = draw_rows(w, n, seed)
    A = _i8(msa)[rows].copy()
    prev = A.copy()
    m1, s1 = seqid(A, A, perm)
    records = [(0, m1, s1, 1.0, 0.0)]
    t_prev, t = 0, 1
    while t <= max_sweeps:
        A = gibbs(h, J, A, q, t - t_prev, seed, sweep_offset=t_prev, beta=beta)[0]
        m1, s1 = seqid(A, A, perm)
        m2, s2 = seqid(A, prev)
        records.append((t, m1, s1, m2, s2))
        if abs(m2 - m1) <= (s1 + s2) / np.sqrt(n):
            return t, records, A
        prev = A.copy()
        t_prev, t = t, 2 * t
    return None, records, A


# --------------------------------------------------------------------------
# Element decimation (edDCA, Sec. 2.2 and Sec. 3.2)
# --------------------------------------------------------------------------
def skl_element(J: float, p: float) -> float:
    """Symmetric KL between the model and the model without one coupling element."""
    return lib().orc_skl_element(float(J), float(p))


def decimate(J, mask, chains, q: int, drate: float, density: float):
    """One graph update; returns (J, mask, active elements after)."""
    Jc = _f32(J).copy()
    mc = np.ascontiguousarray(mask, dtype=np.uint8).copy()
    ch = _i8(chains)
    N, L = ch.shape
    n = lib().orc_decimate(_ptr(Jc), _ptr(mc), _ptr(ch), N, L, q, float(drate), float(density))
    return Jc, mc, int(n)


def bernoulli_kl(f: float, p: float) -> float:
    """KL divergence of Bernoulli(f) from Bernoulli(p) (element-activation distance)."""
    return lib().orc_bernoulli_kl(float(f), float(p))


def activate(mask, chains, f2, q: int, factivate: float):
    """One element-activation graph update; returns (mask, active elements after)."""
    mc = np.ascontiguousarray(mask, dtype=np.uint8).copy()
    ch = _i8(chains)
    N, L = ch.shape
    f2 = np.ascontiguousarray(f2, dtype=np.float64)
    n = lib().orc_activate(_ptr(mc), _ptr(ch), N, L, q, _ptr(f2), float(factivate))
    return mc, int(n)


def train_step_masked(h, J, mask, chains, f1, f2, q: int, lr: float, sweeps: int, seed: int,
                      epoch: int):
    """Returns (h, J, chains, pearson)."""
    h2, J2 = _f32(h).copy(), _f32(J).copy()
    ch = _i8(chains).copy()
    N, L = ch.shape
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    f1 = np.ascontiguousarray(f1, dtype=np.float64)
    f2 = np.ascontiguousarray(f2, dtype=np.float64)
    r = lib().orc_train_step_masked(_ptr(h2), _ptr(J2), _ptr(m), _ptr(ch), N, L, q, _ptr(f1),
                                    _ptr(f2), float(lr), sweeps, seed, epoch, None, None)
    return h2, J2, ch, r



# --------------------------------------------------------------------------
# Starting point and coupling graphs
# --------------------------------------------------------------------------
def profile_fields(f1, L: int, q: int):
    """h = (float) log f1 of the independent-site model, float32 [L, q]."""
    f1 = np.ascontiguousarray(f1, dtype=np.float64)
    h = np.zeros((L, q), dtype=np.float32)
    lib().orc_profile_fields(_ptr(f1), L, q, _ptr(h))
    return h


def mask_apply(J, mask, q: int):
    """Returns (J with couplings off the graph set to 0, active elements r1 < r2)."""
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    L = m.shape[0] // q
    Jc = None if J is None else _f32(J).copy()
    n = lib().orc_mask_apply(_ptr(Jc), _ptr(m), L, q)
    return Jc, int(n)
