"""Python calls with the names of the C ABI (include/bmdca.h).

Argument marshalling only: tensors are checked for device, dtype and layout,
workspaces are allocated with torch (device memory is plumbing here), and the
C entry point is called on the current stream. Every step of the computation
runs in the HIP library.

Shapes: h float32 [L, q]; J float32 [L*q, L*q]; tokens int8 [rows, L].
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as B
from ._lib import check

PREC = {"fp32": B.PREC_FP32, "bf16x2": B.PREC_BF16X2}


def _ptr(t):
    return None if t is None else t.data_ptr()


def _nbytes(t):
    return t.numel() * t.element_size()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _dev(t: torch.Tensor, dtype, name: str, ndim: int | None = None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dims")
    return t


def _model(h, J):
    _dev(h, torch.float32, "h", 2)
    _dev(J, torch.float32, "J", 2)
    L, q = h.shape
    if J.shape != (L * q, L * q):
        raise ValueError(f"J must be [{L * q}, {L * q}], got {tuple(J.shape)}")
    return L, q


def _prec(prec) -> int:
    return PREC[prec] if isinstance(prec, str) else int(prec)


def _sampler(sampler) -> int:
    return B.SAMPLER[sampler] if isinstance(sampler, str) else int(sampler)


def workspace_bytes(kind: int, MN: int, L: int, q: int, prec=B.PREC_BF16X2) -> int:
    n = B.lib().bmdca_workspace_bytes(kind, MN, L, q, _prec(prec))
    if n == 0:
        raise ValueError(f"no workspace size for kind={kind}, MN={MN}, L={L}, q={q}")
    return n


def workspace(kind: int, MN: int, L: int, q: int, prec=B.PREC_BF16X2, device=None):
    n = workspace_bytes(kind, MN, L, q, prec)
    return torch.empty(n, dtype=torch.uint8, device=device or "cuda")


def identity_threshold(theta: float, L: int) -> int:
    return B.lib().bmdca_identity_threshold(theta, L)


def init_chains(N: int, L: int, q: int, seed: int, out=None, device=None):
    if out is None:
        out = torch.empty((N, L), dtype=torch.int8, device=device or "cuda")
    _dev(out, torch.int8, "chains", 2)
    check(B.lib().bmdca_init_chains(_ptr(out), N, L, q, seed, _stream()))
    return out


def reweight(msa, q: int, theta: float = 0.8, ws=None, dev_err=None):
    """Eq. (7) weights: returns (n_sim int32 [M], w float64 [M], meff float64 [1])."""
    _dev(msa, torch.int8, "msa", 2)
    M, L = msa.shape
    dev = msa.device
    n = torch.empty(M, dtype=torch.int32, device=dev)
    w = torch.empty(M, dtype=torch.float64, device=dev)
    meff = torch.empty(1, dtype=torch.float64, device=dev)
    if ws is None:
        ws = workspace(B.WS_REWEIGHT, M, L, q, 0, dev)
    check(B.lib().bmdca_reweight(_ptr(msa), M, L, q, theta, _ptr(n), _ptr(w), _ptr(meff),
                                 _ptr(ws), _nbytes(ws), _ptr(dev_err), _stream()))
    return n, w, meff


def stats(X, q: int, w=None, pseudocount: float = -1.0, prec="bf16x2", ws=None, dev_err=None,
          out=None):
    """Eqs. (3), (8)-(9): returns (f1 float64 [L*q], f2 float64 [Lq, Lq], meff [1])."""
    _dev(X, torch.int8, "X", 2)
    M, L = X.shape
    dev = X.device
    if w is not None:
        _dev(w, torch.float64, "w", 1)
        if w.numel() != M:
            raise ValueError("w must have one entry per row")
    if out is None:
        f1 = torch.empty(L * q, dtype=torch.float64, device=dev)
        f2 = torch.empty((L * q, L * q), dtype=torch.float64, device=dev)
        meff = torch.empty(1, dtype=torch.float64, device=dev)
    else:
        f1, f2, meff = out
    p = _prec(prec)
    if ws is None:
        ws = workspace(B.WS_STATS, M, L, q, p, dev)
    check(B.lib().bmdca_stats(_ptr(X), _ptr(w), M, L, q, pseudocount, p, _ptr(f1), _ptr(f2),
                              _ptr(meff), _ptr(ws), _nbytes(ws), _ptr(dev_err), _stream()))
    return f1, f2, meff


def gibbs(h, J, chains, sweeps: int, seed: int, sweep_offset: int = 0, beta: float = 1.0,
          H_ws=None, flips=None, keep_fields: bool = False, sampler="auto"):
    """Sweeps the chains in place (Sec. 2.1). Returns the chains tensor.
    sampler: "auto", "fields" (local fields in HBM, incremental) or "gather".
    keep_fields=True (field form) continues from the local fields a previous
    call left in H_ws for the same h, J and chains."""
    L, q = _model(h, J)
    _dev(chains, torch.int8, "chains", 2)
    N = chains.shape[0]
    if chains.shape[1] != L:
        raise ValueError("chains must be [N, L]")
    flags = _sampler(sampler) | (B.GIBBS_KEEP_FIELDS if keep_fields else 0)
    if H_ws is None:
        if keep_fields:
            raise ValueError("keep_fields needs the H_ws of the previous call")
        H_ws = workspace(B.WS_GIBBS, N, L, q, flags, chains.device)
    check(B.lib().bmdca_gibbs(_ptr(h), _ptr(J), _ptr(chains), N, L, q, sweeps, seed, sweep_offset,
                              beta, _ptr(H_ws), _nbytes(H_ws), flags, _ptr(flips), _stream()))
    return chains


def chain_streams(seeds, offsets, chains, device="cuda"):
    """Device table of bmdca_chain_stream records from per-chain numpy arrays."""
    n = len(seeds)
    rec = np.zeros(n, dtype=[("seed", "<u8"), ("sweep_offset", "<u8"), ("chain", "<u4"),
                             ("reserved", "<u4")])
    rec["seed"], rec["sweep_offset"], rec["chain"] = seeds, offsets, chains
    host = torch.frombuffer(bytearray(rec.tobytes()), dtype=torch.uint8).pin_memory()
    return host.to(device, non_blocking=True)


def gibbs_streams(h, J, chains, sweeps: int, streams, beta: float = 1.0, H_ws=None, flips=None,
                  sampler="auto", cus: int = 0):
    """bmdca_gibbs_streams: chain c draws as described by streams[c]."""
    L, q = _model(h, J)
    _dev(chains, torch.int8, "chains", 2)
    _dev(streams, torch.uint8, "streams", 1)
    N = chains.shape[0]
    if streams.numel() != 24 * N:
        raise ValueError("streams must hold one 24-byte record per chain")
    flags = _sampler(sampler)
    if H_ws is None:
        H_ws = workspace(B.WS_GIBBS, N, L, q, flags, chains.device)
    check(B.lib().bmdca_gibbs_streams(_ptr(h), _ptr(J), _ptr(chains), N, L, q, sweeps,
                                      _ptr(streams), beta, _ptr(H_ws), _nbytes(H_ws), flags, cus,
                                      _ptr(flips), _stream()))
    return chains


# ------------------------------------------------------------ serving forms
def energy_batch(h, J, seqs, n_live, E, ws, dev_err=None):
    """bmdca_energy_batch: energies of the first *n_live rows of the arena
    seqs [cap, L] into E [cap] (n_live: device int64 [1])."""
    L, q = _model(h, J)
    _dev(seqs, torch.int8, "seqs", 2)
    _dev(n_live, torch.int64, "n_live")
    check(B.lib().bmdca_energy_batch(_ptr(h), _ptr(J), _ptr(seqs), seqs.shape[0], _ptr(n_live),
                                     L, q, _ptr(E), _ptr(ws), _nbytes(ws), _ptr(dev_err),
                                     _stream()))
    return E


def mutant_scan_batch(h, J, wt, n_live, dE, ws):
    """bmdca_mutant_scan_batch over the first *n_live wild types of wt [cap, L]."""
    L, q = _model(h, J)
    _dev(wt, torch.int8, "wt", 2)
    _dev(n_live, torch.int64, "n_live")
    check(B.lib().bmdca_mutant_scan_batch(_ptr(h), _ptr(J), _ptr(wt), wt.shape[0], _ptr(n_live),
                                          L, q, _ptr(dE), _ptr(ws), _nbytes(ws), _stream()))
    return dE


def sample_tick(h, J, chains, n_live, sweeps: int, streams, tick, ws, beta: float = 1.0,
                keep_layout: bool = True, cus: int = 0):
    """bmdca_sample_tick: `sweeps` sweeps of the first *n_live chains of the
    arena chains [cap, L] with per-chain streams, then tick += 1."""
    L, q = _model(h, J)
    _dev(chains, torch.int8, "chains", 2)
    _dev(n_live, torch.int64, "n_live")
    _dev(streams, torch.uint8, "streams", 1)
    _dev(tick, torch.int64, "tick")
    cap = chains.shape[0]
    if streams.numel() != 24 * cap:
        raise ValueError("streams must hold one 24-byte record per arena chain")
    flags = B.GIBBS_KEEP_LAYOUT if keep_layout else 0
    check(B.lib().bmdca_sample_tick(_ptr(h), _ptr(J), _ptr(chains), cap, _ptr(n_live), L, q,
                                    sweeps, _ptr(streams), _ptr(tick), beta, _ptr(ws),
                                    _nbytes(ws), flags, cus, _stream()))
    return chains


def energy(h, J, seqs, dev_err=None, out=None, ws=None):
    """Eq. (1) energies: float32 [B]."""
    L, q = _model(h, J)
    _dev(seqs, torch.int8, "seqs", 2)
    Bn = seqs.shape[0]
    if out is None:
        out = torch.empty(Bn, dtype=torch.float32, device=seqs.device)
    if ws is None and Bn > 0:
        ws = workspace(B.WS_ENERGY, Bn, L, q, 0, seqs.device)
    check(B.lib().bmdca_energy(_ptr(h), _ptr(J), _ptr(seqs), Bn, L, q, _ptr(out), _ptr(ws),
                               0 if ws is None else _nbytes(ws), _ptr(dev_err), _stream()))
    return out


def train_step(h, J, chains, f1, f2, lr: float, sweeps: int, seed: int, epoch: int,
               prec="bf16x2", ws=None, pearson=None, flips=None, dev_err=None, sampler="auto"):
    """One epoch (Sec. 2.1); h, J and chains are updated in place.
    Returns the device scalar holding the Pearson coefficient."""
    L, q = _model(h, J)
    _dev(chains, torch.int8, "chains", 2)
    _dev(f1, torch.float64, "f1")
    _dev(f2, torch.float64, "f2")
    N = chains.shape[0]
    p = _prec(prec) | _sampler(sampler)
    if ws is None:
        ws = workspace(B.WS_TRAIN_STEP, N, L, q, p, chains.device)
    if pearson is None:
        pearson = torch.empty(1, dtype=torch.float64, device=chains.device)
    check(B.lib().bmdca_train_step(_ptr(h), _ptr(J), _ptr(chains), N, L, q, _ptr(f1), _ptr(f2),
                                   lr, sweeps, seed, epoch, p, _ptr(pearson), _ptr(flips),
                                   _ptr(ws), _nbytes(ws), _ptr(dev_err), _stream()))
    return pearson


# ------------------------------------------------------- equilibrium sampling
def draw_rows(w, n: int, seed: int, dev_err=None, ws=None):
    """n row indices drawn with probability w / sum(w) (int32 device tensor)."""
    _dev(w, torch.float64, "w", 1)
    M = w.numel()
    rows = torch.empty(n, dtype=torch.int32, device=w.device)
    if ws is None:
        ws = workspace(B.WS_DRAW, M, 1, 2, 0, w.device)
    check(B.lib().bmdca_draw_rows(_ptr(w), M, n, seed, _ptr(rows), _ptr(ws), _nbytes(ws),
                                  _ptr(dev_err), _stream()))
    return rows


def gather_rows(X, rows, dev_err=None):
    """X[rows] for an int8 [M, L] tensor and int32 row indices."""
    _dev(X, torch.int8, "X", 2)
    _dev(rows, torch.int32, "rows", 1)
    M, L = X.shape
    out = torch.empty((rows.numel(), L), dtype=torch.int8, device=X.device)
    check(B.lib().bmdca_gather_rows(_ptr(X), M, L, _ptr(rows), rows.numel(), _ptr(out),
                                    _ptr(dev_err), _stream()))
    return out


def seqid(A, Bm, perm=None, dev_err=None, ws=None, out=None):
    """Device double [2]: mean and standard deviation of SeqID(A[k], B[perm[k]])."""
    _dev(A, torch.int8, "A", 2)
    _dev(Bm, torch.int8, "B", 2)
    if A.shape != Bm.shape:
        raise ValueError("A and B must have the same shape")
    if perm is not None:
        _dev(perm, torch.int32, "perm", 1)
        if perm.numel() != A.shape[0]:
            raise ValueError("perm must have one entry per row")
    N, L = A.shape
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=A.device)
    if ws is None:
        ws = workspace(B.WS_SEQID, 0, L, 2, 0, A.device)
    check(B.lib().bmdca_seqid(_ptr(A), _ptr(Bm), _ptr(perm), N, L, _ptr(out), _ptr(ws),
                              _nbytes(ws), _ptr(dev_err), _stream()))
    return out


# ----------------------------------------------------- sparse models (edDCA)
def mask_init(L: int, q: int, full: bool = True, device="cuda", out=None):
    """bmdca_mask_init: the fully connected coupling graph (1 off the diagonal
    blocks) or the empty one, as a uint8 [Lq, Lq] mask."""
    if out is None:
        out = torch.empty((L * q, L * q), dtype=torch.uint8, device=device)
    _dev(out, torch.uint8, "mask", 2)
    check(B.lib().bmdca_mask_init(_ptr(out), L, q, 1 if full else 0, _stream()))
    return out


def full_mask(L: int, q: int, device="cuda"):
    """The fully connected coupling graph: 1 off the diagonal blocks."""
    return mask_init(L, q, True, device)


def mask_apply(J, mask, q: int, n_active=None):
    """bmdca_mask_apply: J = 0 off the graph (J may be None to count only);
    returns the device int64 count of active elements r1 < r2."""
    _dev(mask, torch.uint8, "mask", 2)
    L = mask.shape[0] // q
    if J is not None:
        _dev(J, torch.float32, "J", 2)
    if n_active is None:
        n_active = torch.empty(1, dtype=torch.int64, device=mask.device)
    check(B.lib().bmdca_mask_apply(_ptr(J), _ptr(mask), L, q, _ptr(n_active), _stream()))
    return n_active


def profile_fields(f1, L: int, q: int, dev_err=None, out=None):
    """bmdca_profile_fields: h = (float) log f1, the independent-site model's
    fields, as float32 [L, q]."""
    _dev(f1, torch.float64, "f1")
    if out is None:
        out = torch.empty((L, q), dtype=torch.float32, device=f1.device)
    check(B.lib().bmdca_profile_fields(_ptr(f1), L, q, _ptr(out), _ptr(dev_err), _stream()))
    return out


def train_step_masked(h, J, mask, chains, f1, f2, lr: float, sweeps: int, seed: int, epoch: int,
                      prec="bf16x2", ws=None, pearson=None, flips=None, dev_err=None,
                      sampler="auto"):
    """train_step on the graph `mask`; returns the device Pearson scalar."""
    L, q = _model(h, J)
    _dev(mask, torch.uint8, "mask", 2)
    _dev(chains, torch.int8, "chains", 2)
    N = chains.shape[0]
    p = _prec(prec) | _sampler(sampler)
    if ws is None:
        ws = workspace(B.WS_TRAIN_STEP, N, L, q, p, chains.device)
    if pearson is None:
        pearson = torch.empty(1, dtype=torch.float64, device=chains.device)
    check(B.lib().bmdca_train_step_masked(_ptr(h), _ptr(J), _ptr(mask), _ptr(chains), N, L, q,
                                          _ptr(f1), _ptr(f2), lr, sweeps, seed, epoch, p,
                                          _ptr(pearson), _ptr(flips), _ptr(ws), _nbytes(ws),
                                          _ptr(dev_err), _stream()))
    return pearson


def decimate(J, mask, chains, q: int, drate: float, density: float, ws=None, dev_err=None,
             n_active=None):
    """One element-decimation graph update (in place); returns the device
    int64 count of active elements afterwards."""
    _dev(J, torch.float32, "J", 2)
    _dev(mask, torch.uint8, "mask", 2)
    _dev(chains, torch.int8, "chains", 2)
    N, L = chains.shape
    if ws is None:
        ws = workspace(B.WS_DECIMATE, N, L, q, 0, chains.device)
    if n_active is None:
        n_active = torch.empty(1, dtype=torch.int64, device=chains.device)
    check(B.lib().bmdca_decimate(_ptr(J), _ptr(mask), _ptr(chains), N, L, q, float(drate),
                                 float(density), _ptr(n_active), _ptr(ws), _nbytes(ws),
                                 _ptr(dev_err), _stream()))
    return n_active


def activate(mask, chains, f2, q: int, factivate: float, ws=None, dev_err=None, n_active=None):
    """One element-activation graph update of the mask (in place); returns
    the device int64 count of active elements afterwards."""
    _dev(mask, torch.uint8, "mask", 2)
    _dev(chains, torch.int8, "chains", 2)
    _dev(f2, torch.float64, "f2", 2)
    N, L = chains.shape
    if ws is None:
        ws = workspace(B.WS_DECIMATE, N, L, q, 0, chains.device)
    if n_active is None:
        n_active = torch.empty(1, dtype=torch.int64, device=chains.device)
    check(B.lib().bmdca_activate(_ptr(mask), _ptr(chains), N, L, q, _ptr(f2), float(factivate),
                                 _ptr(n_active), _ptr(ws), _nbytes(ws), _ptr(dev_err), _stream()))
    return n_active


# ------------------------------------------------------------ grouped training
def train_ctl(device, target_pearson: float = 0.0, epoch: int = 0, active: bool = True):
    """A device control record (bmdca_train_ctl) as a uint8 tensor of its 24 bytes."""
    rec = B.TrainCtl(epoch, 1 if active else 0, -1, float(target_pearson))
    host = torch.frombuffer(bytearray(bytes(rec)), dtype=torch.uint8)
    return host.to(device)


def read_ctl(ctl) -> dict:
    """The fields of a device control record (synchronises on the copy)."""
    rec = B.TrainCtl.from_buffer_copy(bytes(ctl.cpu().numpy().tobytes()))
    return {"epoch": rec.epoch, "active": bool(rec.active), "converged_at": rec.converged_at,
            "target_pearson": rec.target_pearson}


class TrainModel:
    """One model of a training group: its tensors and epoch arguments, the
    bmdca_train_problem record that names them, and its control record."""

    def __init__(self, h, J, chains, f1, f2, lr: float, sweeps: int, seed: int,
                 prec="bf16x2", sampler="auto", target_pearson: float = 0.0, ws=None,
                 flips=None, dev_err=None, mask=None):
        L, q = _model(h, J)
        _dev(chains, torch.int8, "chains", 2)
        _dev(f1, torch.float64, "f1")
        _dev(f2, torch.float64, "f2")
        self.h, self.J, self.chains, self.f1, self.f2 = h, J, chains, f1, f2
        self.L, self.q, self.N = L, q, chains.shape[0]
        self.prec = _prec(prec) | _sampler(sampler)
        dev = chains.device
        self.ws = ws if ws is not None else workspace(B.WS_TRAIN_STEP, self.N, L, q, self.prec, dev)
        self.pearson = torch.zeros(1, dtype=torch.float64, device=dev)
        self.flips, self.dev_err = flips, dev_err
        self.ctl = train_ctl(dev, target_pearson)
        if mask is not None:
            _dev(mask, torch.uint8, "mask", 2)
        self.mask = mask
        self.record = B.TrainProblem(
            _ptr(h), _ptr(J), _ptr(chains), _ptr(f1), _ptr(f2), _ptr(self.pearson), _ptr(flips),
            _ptr(dev_err), _ptr(self.ctl), _ptr(self.ws), _nbytes(self.ws), self.N, L, q,
            float(lr), int(seed), int(sweeps), self.prec, _ptr(mask))


def _records(models):
    arr = (B.TrainProblem * len(models))()
    for k, m in enumerate(models):
        arr[k] = m.record
    return arr


def train_group_step(models, lanes: int = 8):
    """One epoch of every active model (bmdca_train_group_step)."""
    arr = _records(models)
    check(B.lib().bmdca_train_group_step(arr, len(models), lanes, _stream()))


class TrainGroupGraph:
    """A captured group epoch (bmdca_train_group_graph); launch() replays it.
    Capture runs on a side stream; the models must stay alive with it."""

    def __init__(self, models, lanes: int = 8):
        self.models = list(models)
        self._stream = torch.cuda.Stream()
        self._stream.wait_stream(torch.cuda.current_stream())
        handle = B._p()
        arr = _records(self.models)
        check(B.lib().bmdca_train_group_graph(arr, len(self.models), lanes,
                                              self._stream.cuda_stream, B.C.byref(handle)))
        self.handle = handle

    def launch(self):
        check(B.lib().bmdca_graph_launch(self.handle, _stream()))

    def close(self):
        if self.handle:
            check(B.lib().bmdca_graph_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def single_mutant_scan(h, J, wt, ws=None, out=None):
    """Sec. 4.4: dE float32 [B, L*q] for wild types wt int8 [B, L]."""
    L, q = _model(h, J)
    _dev(wt, torch.int8, "wt", 2)
    Bn = wt.shape[0]
    if ws is None:
        ws = workspace(B.WS_MUTANT, Bn, L, q, 0, wt.device)
    if out is None:
        out = torch.empty((Bn, L * q), dtype=torch.float32, device=wt.device)
    check(B.lib().bmdca_single_mutant_scan(_ptr(h), _ptr(J), _ptr(wt), Bn, L, q, _ptr(out),
                                           _ptr(ws), _nbytes(ws), _stream()))
    return out


def apc_frobenius(J, L: int, q: int, gap: int = 0, ws=None):
    """Eq. (13): returns (F, F_apc), float32 [L, L]."""
    _dev(J, torch.float32, "J", 2)
    if J.shape != (L * q, L * q):
        raise ValueError("J must be [L*q, L*q]")
    F = torch.empty((L, L), dtype=torch.float32, device=J.device)
    Fa = torch.empty((L, L), dtype=torch.float32, device=J.device)
    if ws is None:
        ws = workspace(B.WS_APC, 0, L, q, 0, J.device)
    check(B.lib().bmdca_apc_frobenius(_ptr(J), L, q, gap, _ptr(F), _ptr(Fa), _ptr(ws), _nbytes(ws),
                                      _stream()))
    return F, Fa
