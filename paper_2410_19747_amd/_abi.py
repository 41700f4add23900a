"""ctypes mirror of include/ttm.h (structures, codes, prototypes)."""
from __future__ import annotations

import ctypes
import os

TTM_OK = 0
TTM_EINVAL = -1
TTM_ESHAPE = -2
TTM_EWORKSPACE = -3
TTM_ECAPACITY = -4
TTM_ENOCONV = -5
TTM_ENONFINITE = -6
TTM_EHIP = -7
TTM_EFORCED = -8
TTM_EUNSUPPORTED = -9

I32P = ctypes.POINTER(ctypes.c_int32)
I64P = ctypes.POINTER(ctypes.c_int64)
F64P = ctypes.POINTER(ctypes.c_double)


class TtmTT(ctypes.Structure):
    _fields_ = [
        ("n_sites", ctypes.c_int32),
        ("phys", I32P),
        ("bonds", I32P),
        ("offsets", I64P),
        ("data", ctypes.c_void_p),
        ("dtype", ctypes.c_int32),
    ]


class TtmTTOut(ctypes.Structure):
    _fields_ = [
        ("bonds", I32P),
        ("offsets", I64P),
        ("data", ctypes.c_void_p),
        ("capacity", ctypes.c_int64),
    ]


class TtmOptions(ctypes.Structure):
    _fields_ = [
        ("chi_mid", ctypes.c_int32),
        ("final_round", ctypes.c_int32),
        ("max_sweeps", ctypes.c_int32),
        ("svd_max_sweeps", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("forced_ranks", I32P),
        ("n_forced", ctypes.c_int32),
        ("trace_cap", ctypes.c_int32),
        ("rank_trace", I32P),
        ("discard_trace", F64P),
        ("profile", ctypes.c_int32),
        ("contract_precision", ctypes.c_int32),
        ("move_factor", ctypes.c_int32),
        ("gauge", ctypes.c_int32),
        ("svd_mode", ctypes.c_int32),
        ("rsvd_power", ctypes.c_int32),
        ("rsvd_tol", ctypes.c_double),
    ]


class TtmStats(ctypes.Structure):
    _fields_ = [
        ("max_bond", ctypes.c_int32),
        ("n_contract", ctypes.c_int32),
        ("n_swap", ctypes.c_int32),
        ("n_qr", ctypes.c_int32),
        ("n_svd", ctypes.c_int32),
        ("n_trace", ctypes.c_int32),
        ("sweeps", ctypes.c_int32),
        ("jacobi_max_sweeps", ctypes.c_int32),
        ("discarded_sq_sum", ctypes.c_double),
        ("error_bound", ctypes.c_double),
        ("model_flops", ctypes.c_double),
        ("svd_model_flops", ctypes.c_double),
        ("jacobi_solve_flops", ctypes.c_double),
        ("peak_ws_bytes", ctypes.c_size_t),
        ("kernel_ms", ctypes.c_double * 7),
        ("kernel_launches", ctypes.c_int64 * 7),
        ("n_rsvd", ctypes.c_int32),
        ("n_rsvd_fallback", ctypes.c_int32),
    ]


TTM_PREC_F64, TTM_PREC_F32, TTM_PREC_BF16, TTM_PREC_BF16X3 = 0, 1, 2, 3
TTM_MOVE_SECOND, TTM_MOVE_SMALLER = 0, 1
TTM_GAUGE_MOVING, TTM_GAUGE_RIGHT = 0, 1
TTM_SVD_JACOBI, TTM_SVD_RANDOMIZED = 0, 1
SVD_MODES = {"jacobi": TTM_SVD_JACOBI, "randomized": TTM_SVD_RANDOMIZED}
PRECISIONS = {"f64": TTM_PREC_F64, "f32": TTM_PREC_F32, "bf16": TTM_PREC_BF16, "bf16x3": TTM_PREC_BF16X3}

KERNEL_CLASSES = ["gemm", "qr", "jacobi_gram", "jacobi_solve", "jacobi_other", "other", "jacobi_apply"]


# Every symbol include/ttm.h declares, with its prototype.
PROTOTYPES = {
    "ttm_default_options": (None, [ctypes.POINTER(TtmOptions)]),
    "ttm_query": (ctypes.c_int, [ctypes.POINTER(TtmTT), ctypes.POINTER(TtmTT), ctypes.c_int32,
                                 ctypes.POINTER(TtmOptions), ctypes.POINTER(ctypes.c_size_t),
                                 ctypes.POINTER(ctypes.c_int64)]),
    "ttm_multiply": (ctypes.c_int, [ctypes.POINTER(TtmTT), ctypes.POINTER(TtmTT), ctypes.c_int32,
                                    ctypes.c_double, ctypes.POINTER(TtmTTOut), ctypes.c_void_p,
                                    ctypes.c_size_t, ctypes.c_void_p]),
    "ttm_multiply_ex": (ctypes.c_int, [ctypes.POINTER(TtmTT), ctypes.POINTER(TtmTT), ctypes.c_int32,
                                       ctypes.c_double, ctypes.POINTER(TtmTTOut), ctypes.c_void_p,
                                       ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(TtmOptions),
                                       ctypes.POINTER(TtmStats)]),
    "ttm_multiply_batch": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(TtmTT), ctypes.POINTER(TtmTT),
                                          I32P, F64P, ctypes.POINTER(TtmTTOut),
                                          ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_size_t),
                                          ctypes.POINTER(TtmOptions), ctypes.POINTER(TtmStats),
                                          ctypes.c_int32, ctypes.c_void_p, I32P]),
    "ttm_inner_grad_query": (ctypes.c_int, [ctypes.POINTER(TtmTT)] * 3 + [ctypes.POINTER(ctypes.c_size_t)]),
    "ttm_inner_grad": (ctypes.c_int, [ctypes.POINTER(TtmTT)] * 3 + [ctypes.c_int32, F64P, ctypes.c_void_p,
                                                                    ctypes.c_void_p, ctypes.c_void_p,
                                                                    ctypes.c_size_t, ctypes.c_void_p]),
    "ttm_inner_grad_query_ex": (ctypes.c_int, [ctypes.POINTER(TtmTT)] * 3 + [ctypes.c_int32,
                                                                             ctypes.POINTER(ctypes.c_size_t)]),
    "ttm_inner_grad_ex": (ctypes.c_int, [ctypes.POINTER(TtmTT)] * 3 + [ctypes.c_int32, F64P, ctypes.c_void_p,
                                                                       ctypes.c_void_p, ctypes.c_int32,
                                                                       ctypes.c_void_p, ctypes.c_size_t,
                                                                       ctypes.c_void_p]),
    "conventional_query": (ctypes.c_int, [ctypes.POINTER(TtmTT), ctypes.POINTER(TtmTT), ctypes.c_int32,
                                          ctypes.POINTER(TtmOptions), ctypes.POINTER(ctypes.c_size_t),
                                          ctypes.POINTER(ctypes.c_int64)]),
    "conventional_multiply": (ctypes.c_int, [ctypes.POINTER(TtmTT), ctypes.POINTER(TtmTT),
                                             ctypes.c_int32, ctypes.c_double, ctypes.POINTER(TtmTTOut),
                                             ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "conventional_multiply_ex": (ctypes.c_int, [ctypes.POINTER(TtmTT), ctypes.POINTER(TtmTT),
                                                ctypes.c_int32, ctypes.c_double,
                                                ctypes.POINTER(TtmTTOut), ctypes.c_void_p,
                                                ctypes.c_size_t, ctypes.c_void_p,
                                                ctypes.POINTER(TtmOptions), ctypes.POINTER(TtmStats)]),
    "ttm_multiply_static": (ctypes.c_int, [ctypes.POINTER(TtmTT), ctypes.POINTER(TtmTT), ctypes.c_int32,
                                           ctypes.c_double, ctypes.POINTER(TtmTTOut), ctypes.c_void_p,
                                           ctypes.POINTER(TtmOptions), ctypes.POINTER(TtmStats)]),
    "ttm_vjp_query": (ctypes.c_int, [ctypes.POINTER(TtmTT), ctypes.POINTER(TtmTT), ctypes.c_int32,
                                     ctypes.POINTER(TtmOptions), ctypes.POINTER(ctypes.c_size_t),
                                     ctypes.POINTER(ctypes.c_int64)]),
    "ttm_multiply_vjp": (ctypes.c_int, [ctypes.POINTER(TtmTT), ctypes.POINTER(TtmTT), ctypes.c_int32,
                                        ctypes.c_double, ctypes.POINTER(TtmOptions), ctypes.POINTER(TtmTT),
                                        ctypes.POINTER(TtmTTOut), ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                        ctypes.POINTER(TtmStats)]),
    "ttm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "ttm_last_error": (ctypes.c_char_p, []),
    "ttm_version": (ctypes.c_char_p, []),
}


# Kernel-level test hooks declared in include/ttm_testing.h.
_VP = ctypes.c_void_p
_I64 = ctypes.c_int64
TESTING_PROTOTYPES = {
    "ttm_test_gemm": (ctypes.c_int, [ctypes.c_int] * 4 + [_VP, _I64, _I64, _I64, _VP, _I64, _I64, _I64,
                                                          _VP, _I64, ctypes.c_int, ctypes.c_int,
                                                          _I64, _I64, _I64, _I64, _VP]),
    "ttm_test_gemm_prec": (ctypes.c_int, [ctypes.c_int] * 4 + [_VP, _I64, _I64, _VP, _I64, _I64, _VP, _I64, _VP]),
    "ttm_test_qr_scratch": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int]),
    "ttm_test_qr": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, _VP, _VP, _VP]),
    "ttm_test_mfma_f64_rate": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _VP, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double), _VP]),
    "ttm_test_qr_pivoted_scratch": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int]),
    "ttm_test_qr_pivoted": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, _VP, _VP]),
    "ttm_test_svd_ws_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int]),
    "ttm_test_svd": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, _VP, _VP,
                                    ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), _VP,
                                    ctypes.c_size_t, _VP]),
    "ttm_test_svd_ws_bytes_bw": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "ttm_test_svd_bw": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, _VP, _VP,
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                       ctypes.c_int, _VP, ctypes.c_size_t, _VP]),
    "ttm_test_cholqr2_ws_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int]),
    "ttm_test_cholqr2": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _VP,
                                        ctypes.c_size_t, _VP]),
}

TTM_STATIC_WS_BYTES = 32 << 20


def library_path():
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "libttm.so")


def load_library():
    path = library_path()
    if not os.path.exists(path):
        raise ImportError("libttm.so is not built (%s); run __graft_entry__.build() or "
                          "python -m paper_2410_19747_amd.build" % path)
    L = ctypes.CDLL(path)
    for name, (res, args) in list(PROTOTYPES.items()) + list(TESTING_PROTOTYPES.items()):
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L
