"""ctypes binding of libmsc.so (the C ABI declared in include/msc.h).

Argument marshalling only: every step of the simulation runs inside the
library.  Device arrays are torch tensors on the context's GPU; host arrays
are numpy arrays.  The library must have been built in-tree
(``python -m paper_2609_19116_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

import numpy as np

_PKG = Path(__file__).resolve().parent
LIB_PATH = _PKG / "libmsc.so"

MSC_OK = 0
MSC_E_PARSE = -1
MSC_E_INVALID = -2
MSC_E_NONDETERMINISTIC = -3
MSC_E_CAPACITY = -4
MSC_E_DEVICE = -5
MSC_E_OOM = -6
MSC_E_STATE = -7

MSC_FP64 = 0
MSC_FP32 = 1
MSC_BF16X3 = 2

# fixed op costs (flop equivalents) of the order-search cost: MSC_ORDER_COST_*
MSC_ORDER_COST_PSWAP = 7.0e5
MSC_ORDER_COST_MOVE = 1.2e6
MSC_ORDER_COST_TWOSITE = 2.5e6

SHOT_DONE = 1
SHOT_REJECTED = 2
SHOT_CHI_CAP = 4
SHOT_NOCONV = 8
SHOT_MPS_RERUN = 16


class CircuitInfo(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_meas", C.c_int32), ("n_channels", C.c_int32),
                ("n_decided", C.c_int32), ("seed_qubit", C.c_int32), ("target", C.c_int32),
                ("words", C.c_int32), ("calibrated", C.c_int32), ("n_ops", C.c_int64),
                ("n_twosite", C.c_int64), ("n_swaps", C.c_int64),
                ("n_product_swaps", C.c_int64), ("n_moves", C.c_int64)]


class SimOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("chi_max", C.c_int32), ("tau_trunc", C.c_double),
                ("tau_rej", C.c_double), ("tau_fail", C.c_double), ("n_slots", C.c_int32),
                ("lds_width", C.c_int32), ("prefix", C.c_int32), ("large_side", C.c_int32),
                ("use_graphs", C.c_int32), ("wave_chi", C.c_int32),
                ("autotune_cache", C.c_char_p)]


class BatchStats(C.Structure):
    _fields_ = [("n_shots", C.c_int64), ("nnz", C.c_int64), ("n_survivors", C.c_int64),
                ("n_accepted", C.c_int64), ("n2q", C.c_int64), ("sweeps", C.c_int64),
                ("flops", C.c_double), ("chi_peak", C.c_int32), ("status_or", C.c_int32),
                ("ms_sample", C.c_double), ("ms_screen", C.c_double), ("ms_simulate", C.c_double)]


class ShotResult(C.Structure):
    _fields_ = [("p_acc", C.c_double), ("infid", C.c_double), ("disc_weight", C.c_double),
                ("chi_peak", C.c_int32), ("status", C.c_int32), ("rejected_at", C.c_int32),
                ("fail", C.c_int32), ("n2q", C.c_int64), ("flops", C.c_double),
                ("sweeps", C.c_int64)]


SHOT_DTYPE = np.dtype([("p_acc", "<f8"), ("infid", "<f8"), ("disc_weight", "<f8"),
                       ("chi_peak", "<i4"), ("status", "<i4"), ("rejected_at", "<i4"),
                       ("fail", "<i4"), ("n2q", "<i8"), ("flops", "<f8"),
                       ("sweeps", "<i8")])
assert SHOT_DTYPE.itemsize == C.sizeof(ShotResult) == 64


class EngineStats(C.Structure):
    _fields_ = [("rounds", C.c_int64), ("updates", C.c_int64), ("contract_flops", C.c_double),
                ("gram_flops", C.c_double), ("contract_ms", C.c_double), ("gram_ms", C.c_double),
                ("factor_ms", C.c_double), ("shot_ms", C.c_double), ("total_ms", C.c_double),
                ("factor_lds", C.c_int64), ("factor_wide", C.c_int64), ("overlapping", C.c_int64),
                ("sweeps", C.c_int64), ("wave_slots", C.c_int64), ("wave_retries", C.c_int64)]


class TuneEntry(C.Structure):
    _fields_ = [("bucket", C.c_int32), ("side", C.c_int32), ("batch", C.c_int32),
                ("rows", C.c_int32), ("b", C.c_int32), ("gram", C.c_int32),
                ("contract_us", C.c_double), ("gram_us", C.c_double)]


class Estimate(C.Structure):
    _fields_ = [("p_acc", C.c_double), ("p_acc_le", C.c_double), ("p_le", C.c_double),
                ("trunc_bound", C.c_double), ("sem_p_acc", C.c_double),
                ("sem_p_acc_le", C.c_double)]


class Interval(C.Structure):
    _fields_ = [("estimate", C.c_double), ("lo", C.c_double), ("hi", C.c_double),
                ("hi_trunc", C.c_double), ("trunc_bound", C.c_double),
                ("unaccepted", C.c_double), ("unsampled_mass", C.c_double),
                ("n_unsampled", C.c_int32), ("n_bins_used", C.c_int32)]


MSC_STAT_PACC, MSC_STAT_PLE = 0, 1

SEGMENT_DTYPE = np.dtype([("first_meas", "<i4"), ("n_qubits", "<i4"), ("depth", "<i4"),
                          ("noisy", "<i4")])

# every exported symbol of include/msc.h with its signature
_P = C.c_void_p
_SIGS = {
    "msc_last_error": (C.c_char_p, []),
    "msc_version": (C.c_char_p, []),
    "msc_ctx_create": (C.c_int, [C.c_int, _P, C.POINTER(_P)]),
    "msc_ctx_destroy": (None, [_P]),
    "msc_ctx_last_kernel_ms": (C.c_double, [_P, C.c_char_p]),
    "msc_ctx_engine_stats": (C.c_int, [_P, C.POINTER(EngineStats)]),
    "msc_circuit_load": (C.c_int, [C.c_char_p, C.c_size_t, _P, C.POINTER(_P)]),
    "msc_circuit_get_info": (C.c_int, [_P, C.POINTER(CircuitInfo)]),
    "msc_circuit_expected": (C.c_int, [_P, _P]),
    "msc_circuit_calibrate": (C.c_int, [_P, _P]),
    "msc_circuit_noiseless": (C.c_int, [_P, _P]),
    "msc_circuit_segments": (C.c_int, [_P, C.c_int32, _P, C.POINTER(C.c_int32)]),
    "msc_order_search": (C.c_int, [_P, C.c_char_p, C.c_size_t, _P, C.c_uint64, C.c_int32, _P,
                                   _P]),
    "msc_order_cost": (C.c_int, [_P, C.POINTER(C.c_double)]),
    "msc_circuit_free": (None, [_P]),
    "msc_sample_faults": (C.c_int, [_P, C.c_uint64, C.c_uint64, C.c_int64, _P, C.c_double,
                                    _P, _P, _P, C.c_int64, C.POINTER(C.c_int64)]),
    "msc_sample_faults_device": (C.c_int, [_P, _P, C.c_uint64, C.c_uint64, C.c_int64, _P,
                                           C.c_double, _P, _P, _P, C.c_int64,
                                           C.POINTER(C.c_int64)]),
    "msc_prescreen_tables": (C.c_int, [_P, _P, _P]),
    "msc_prescreen": (C.c_int, [_P, _P, C.c_int64, _P, _P, _P, _P, _P, C.POINTER(C.c_int64)]),
    "msc_prescreen_noalloc": (C.c_int, [_P, _P, C.c_int64, _P, _P, _P, _P, _P,
                                        C.POINTER(C.c_int64)]),
    "msc_simulate": (C.c_int, [_P, _P, C.POINTER(SimOpts), C.c_int64, _P, _P, _P, _P,
                               C.c_int64, _P]),
    "msc_run_batch": (C.c_int, [_P, _P, C.POINTER(SimOpts), C.c_uint64, C.c_uint64, C.c_int64,
                                C.c_double, C.c_int32, _P, C.POINTER(BatchStats), _P, _P]),
    "msc_twosite_contract": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, _P, _P, _P, _P]),
    "msc_engine_update": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                    C.c_int32, C.c_int32, C.c_int32, C.c_double, _P, _P, _P, _P,
                                    _P]),
    "msc_autotune": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_char_p, _P]),
    "msc_simulate_camps": (C.c_int, [_P, _P, C.POINTER(SimOpts), C.c_int64, _P, _P, _P, _P,
                                     C.c_int64, _P]),
    "msc_camps_candidates": (C.c_int, [_P, _P, C.POINTER(C.c_int32)]),
    "msc_reweight": (C.c_int, [_P, _P, _P, _P, _P, C.c_int32, C.c_int64, _P, C.c_int32, _P]),
    "msc_profile_loglik": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int64, C.c_double, C.c_int32,
                                     C.c_int32, C.c_double, C.POINTER(C.c_double)]),
    "msc_lr_interval": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int64, C.c_double, C.c_int32,
                                  C.c_int32, C.c_double, C.POINTER(Interval)]),
    "msc_ratio_credible": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int64, C.c_double, C.c_int32,
                                     C.c_double, C.c_double, C.c_double, C.c_double,
                                     C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "msc_loss_factor": (C.c_int, [C.c_int64, C.c_double, C.POINTER(C.c_double)]),
    "msc_expected_volume": (C.c_int, [_P, _P, C.c_int32, _P, C.c_int32, C.c_int64, C.c_double,
                                      _P, _P]),
}

_lib = None


class MscError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"msc error {code}: {msg}")
        self.code = code


def lib() -> C.CDLL:
    """Load libmsc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2609_19116_amd.build`")
        L = C.CDLL(str(LIB_PATH))
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != MSC_OK:
        raise MscError(rc, lib().msc_last_error().decode())


def _ptr(a) -> int:
    """Raw pointer of a numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    assert a.is_contiguous()
    return a.data_ptr()
