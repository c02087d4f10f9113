"""ctypes view of libbmdca.so (include/bmdca.h).

The library must have been built in-tree (`python -m paper_2501_18456_amd.build`);
if it is missing, loading fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbmdca.so")

# status codes (bmdca_status)
OK, EINVAL, ETOKEN, EWORKSPACE, EHIP, ENONFINITE = 0, -1, -2, -3, -4, -5
PREC_FP32, PREC_BF16X2 = 0, 1
DEVERR_TOKEN, DEVERR_NONFINITE, DEVERR_INDEX = 1, 2, 4
SAMPLER_FIELDS, SAMPLER_GATHER, GIBBS_KEEP_FIELDS, SAMPLER_METROPOLIS = 0x10, 0x20, 0x40, 0x80
GIBBS_KEEP_LAYOUT = 0x100
COUNTS_PRODUCT = 0x200  # chain counts from the one-hot product (default: counted directly)
SAMPLER = {"auto": 0, "fields": SAMPLER_FIELDS, "gather": SAMPLER_GATHER,
           "metropolis": SAMPLER_METROPOLIS,
           "metropolis-fields": SAMPLER_METROPOLIS | SAMPLER_FIELDS,
           "metropolis-gather": SAMPLER_METROPOLIS | SAMPLER_GATHER}
ENERGY_SCRATCH_BYTES = 64 << 20  # BMDCA_ENERGY_SCRATCH_BYTES
(WS_REWEIGHT, WS_STATS, WS_GIBBS, WS_TRAIN_STEP, WS_APC, WS_MUTANT, WS_ENERGY, WS_DRAW,
 WS_SEQID, WS_DECIMATE) = range(10)

_p, _i32, _i64, _u64, _f64, _f32, _sz = (C.c_void_p, C.c_int32, C.c_int64, C.c_uint64,
                                          C.c_double, C.c_float, C.c_size_t)


class TrainProblem(C.Structure):
    """bmdca_train_problem (include/bmdca.h), field for field."""
    _fields_ = [
        ("h", _p), ("J", _p), ("chains", _p), ("f1", _p), ("f2", _p), ("pearson", _p),
        ("flips_out", _p), ("dev_err", _p), ("ctl", _p), ("ws", _p), ("ws_bytes", _sz),
        ("N", _i64), ("L", _i32), ("q", _i32), ("lr", _f64), ("seed", _u64),
        ("sweeps", _i32), ("prec", _i32), ("mask", _p),
    ]


class ChainStream(C.Structure):
    """bmdca_chain_stream (include/bmdca.h)."""
    _fields_ = [("seed", _u64), ("sweep_offset", _u64), ("chain", C.c_uint32),
                ("reserved", C.c_uint32)]


class TrainCtl(C.Structure):
    """bmdca_train_ctl (include/bmdca.h): the device record's byte layout."""
    _fields_ = [("epoch", _u64), ("active", _i32), ("converged_at", _i32),
                ("target_pearson", _f64)]


SIGNATURES = {
    "bmdca_workspace_bytes": (_sz, [_i32, _i64, _i32, _i32, _i32]),
    "bmdca_last_error": (C.c_char_p, []),
    "bmdca_identity_threshold": (_i32, [_f64, _i32]),
    "bmdca_init_chains": (C.c_int, [_p, _i64, _i32, _i32, _u64, _p]),
    "bmdca_reweight": (C.c_int, [_p, _i64, _i32, _i32, _f64, _p, _p, _p, _p, _sz, _p, _p]),
    "bmdca_stats": (C.c_int, [_p, _p, _i64, _i32, _i32, _f64, _i32, _p, _p, _p, _p, _sz, _p,
                              _p]),
    "bmdca_gibbs": (C.c_int, [_p, _p, _p, _i64, _i32, _i32, _i32, _u64, _u64, _f32, _p, _sz,
                              _i32, _p, _p]),
    "bmdca_gibbs_streams": (C.c_int, [_p, _p, _p, _i64, _i32, _i32, _i32, _p, _f32, _p, _sz,
                                      _i32, _i32, _p, _p]),
    "bmdca_energy": (C.c_int, [_p, _p, _p, _i64, _i32, _i32, _p, _p, _sz, _p, _p]),
    "bmdca_energy_noalloc": (C.c_int, [_p, _p, _p, _i64, _i32, _i32, _p, _p, _p]),
    "bmdca_train_step": (C.c_int, [_p, _p, _p, _i64, _i32, _i32, _p, _p, _f64, _i32, _u64, _u64,
                                   _i32, _p, _p, _p, _sz, _p, _p]),
    "bmdca_single_mutant_scan": (C.c_int, [_p, _p, _p, _i64, _i32, _i32, _p, _p, _sz, _p]),
    "bmdca_apc_frobenius": (C.c_int, [_p, _i32, _i32, _i32, _p, _p, _p, _sz, _p]),
    "bmdca_draw_rows": (C.c_int, [_p, _i64, _i64, _u64, _p, _p, _sz, _p, _p]),
    "bmdca_gather_rows": (C.c_int, [_p, _i64, _i32, _p, _i64, _p, _p, _p]),
    "bmdca_seqid": (C.c_int, [_p, _p, _p, _i64, _i32, _p, _p, _sz, _p, _p]),
    "bmdca_train_step_masked": (C.c_int, [_p, _p, _p, _p, _i64, _i32, _i32, _p, _p, _f64, _i32,
                                          _u64, _u64, _i32, _p, _p, _p, _sz, _p, _p]),
    "bmdca_decimate": (C.c_int, [_p, _p, _p, _i64, _i32, _i32, _f64, _f64, _p, _p, _sz, _p, _p]),
    "bmdca_activate": (C.c_int, [_p, _p, _i64, _i32, _i32, _p, _f64, _p, _p, _sz, _p, _p]),
    "bmdca_profile_fields": (C.c_int, [_p, _i32, _i32, _p, _p, _p]),
    "bmdca_energy_batch": (C.c_int, [_p, _p, _p, _i64, _p, _i32, _i32, _p, _p, _sz, _p, _p]),
    "bmdca_mutant_scan_batch": (C.c_int, [_p, _p, _p, _i64, _p, _i32, _i32, _p, _p, _sz, _p]),
    "bmdca_sample_tick": (C.c_int, [_p, _p, _p, _i64, _p, _i32, _i32, _i32, _p, _p, _f32, _p,
                                    _sz, _i32, _i32, _p]),
    "bmdca_mask_init": (C.c_int, [_p, _i32, _i32, _i32, _p]),
    "bmdca_mask_apply": (C.c_int, [_p, _p, _i32, _i32, _p, _p]),
    "bmdca_train_group_step": (C.c_int, [C.POINTER(TrainProblem), _i32, _i32, _p]),
    "bmdca_train_group_graph": (C.c_int, [C.POINTER(TrainProblem), _i32, _i32, _p,
                                          C.POINTER(_p)]),
    "bmdca_graph_launch": (C.c_int, [_p, _p]),
    "bmdca_graph_destroy": (C.c_int, [_p]),
}


_lib = None


class BmdcaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bmdca status {code}: {msg}")
        self.code = code


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2501_18456_amd.build` "
                "(the HIP library is the only implementation)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != OK:
        raise BmdcaError(rc, lib().bmdca_last_error().decode(errors="replace"))
