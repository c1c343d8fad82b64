"""ctypes declarations of the C ABI in include/cwt.h (libcwt.so).

Argument marshalling only: every step of the transform runs in the HIP
kernels of libcwt.  There is no fallback; if the library is missing the
import fails with an error that says how to build it.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libcwt.so")

CWT_OK = 0
CWT_E_INVALID = -1
CWT_E_UNSUPPORTED = -2
CWT_E_NOMEM = -3
CWT_E_HIP = -4
CWT_E_BUDGET = -5
CWT_E_AGAIN = -6

ERROR_NAMES = {
    CWT_E_INVALID: "CWT_E_INVALID", CWT_E_UNSUPPORTED: "CWT_E_UNSUPPORTED",
    CWT_E_NOMEM: "CWT_E_NOMEM", CWT_E_HIP: "CWT_E_HIP", CWT_E_BUDGET: "CWT_E_BUDGET",
    CWT_E_AGAIN: "CWT_E_AGAIN",
}

WAVELET = {"morlet": 0, "gabor": 1, "gmw": 2}
PAD = {"smooth7": 0, "pow2": 1, "none": 2, "explicit": 3, "linear": 4}
OUT = {"complex64": 0, "power": 1, "bandpower": 2}
PRECISION = {"fp32": 0, "split_f16": 1, "split_bf16": 2}

CWT_MAX_LEN = 20480
#: bytes of the static device scratch cwt_execute_noalloc uses for its workspace
CWT_NOALLOC_SCRATCH_BYTES = 16 << 20


#: cwt_alloc_fn / cwt_free_fn: device memory callbacks (include/cwt.h)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                           ctypes.c_void_p)


class PlanOpts(ctypes.Structure):
    _fields_ = [
        ("wavelet", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("explicit_len", ctypes.c_int64),
        ("out", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("n_bands", ctypes.c_int32),
        ("band_edges", ctypes.POINTER(ctypes.c_double)),
        ("gmw_beta", ctypes.c_double),
        ("gmw_gamma", ctypes.c_double),
        ("max_channels", ctypes.c_int64),
        ("alloc", ALLOC_FN),
        ("free", FREE_FN),
        ("alloc_ctx", ctypes.c_void_p),
    ]


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("L", ctypes.c_int64),
        ("n_freqs", ctypes.c_int64),
        ("n_bands", ctypes.c_int64),
        ("out", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("wavelet", ctypes.c_int32),
        ("threads", ctypes.c_int32),
        ("n_passes", ctypes.c_int32),
        ("radix", ctypes.c_int32 * 16),
        ("out_rows", ctypes.c_int64),
        ("out_elem_bytes", ctypes.c_int64),
        ("spectrum_bins", ctypes.c_int64),
        ("max_band_bins", ctypes.c_int64),
        ("kernel", ctypes.c_int32),
        ("spectrum_complex", ctypes.c_int32),
        ("max_channels", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64),
        ("n_segments", ctypes.c_int64),
        ("segment_len", ctypes.c_int64),
        ("segment_outputs", ctypes.c_int64),
        ("segment_margin", ctypes.c_int64),
        ("band_chunks", ctypes.c_int64),
    ]


class ServerOpts(ctypes.Structure):
    _fields_ = [
        ("max_batch", ctypes.c_int32),
        ("deadline_us", ctypes.c_int32),
        ("max_pending", ctypes.c_int32),
        ("max_session_windows", ctypes.c_int32),
        ("alloc", ALLOC_FN),
        ("free", FREE_FN),
        ("alloc_ctx", ctypes.c_void_p),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "batches", "hops", "results", "rejected", "sessions_open", "hbm_bytes_used",
        "hbm_budget_bytes", "max_batch_hops", "max_batch_ns", "slot_waits")]


class BatchItem(ctypes.Structure):
    _fields_ = [
        ("plan", ctypes.c_void_p),
        ("x", ctypes.c_void_p),
        ("C", ctypes.c_int64),
        ("out", ctypes.c_void_p),
    ]


class TuneResult(ctypes.Structure):
    _fields_ = [
        ("n_candidates", ctypes.c_int32),
        ("kernel", ctypes.c_int32),
        ("variant", ctypes.c_int32),
        ("threads", ctypes.c_int32),
        ("n_passes", ctypes.c_int32),
        ("radix", ctypes.c_int32 * 16),
        ("best_ms", ctypes.c_float),
        ("default_ms", ctypes.c_float),
    ]


class CwtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERROR_NAMES.get(code, "CWT_E?"), code, msg))
        self.code = code


_lib = None

#: Every function declared in include/cwt.h, with (restype, argtypes).
_VP = ctypes.c_void_p
_I32, _I64, _DBL, _SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
_PD = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "cwt_plan_opts_init": (ctypes.c_int, [ctypes.POINTER(PlanOpts)]),
    "cwt_plan_create": (ctypes.c_int, [ctypes.POINTER(_VP), _I64, _DBL, _PD, _I32, _PD, _DBL,
                                       ctypes.POINTER(PlanOpts), _VP]),
    "cwt_plan_info": (ctypes.c_int, [_VP, ctypes.POINTER(PlanDesc)]),
    "cwt_plan_describe": (ctypes.c_int, [ctypes.POINTER(PlanDesc), _I64, _DBL, _PD, _I32, _PD,
                                         _DBL, ctypes.POINTER(PlanOpts)]),
    "cwt_plan_band_of_freq": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32)]),
    "cwt_workspace_size": (_SZ, [_VP, _I64]),
    "cwt_execute": (ctypes.c_int, [_VP, _VP, _I64, _VP, _VP, _SZ, _VP]),
    "cwt_execute_noalloc": (ctypes.c_int, [_VP, _VP, _I64, _VP, _VP]),
    "cwt_forward_spectra": (ctypes.c_int, [_VP, _VP, _I64, _VP, _SZ, _VP]),
    "cwt_transform_spectra": (ctypes.c_int, [_VP, _I64, _VP, _VP, _SZ, _VP]),
    "cwt_plan_copy_tables": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_float),
                                            ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_float), _VP]),
    "cwt_plan_destroy": (ctypes.c_int, [_VP, _VP]),
    "cwt_plan_autotune": (ctypes.c_int, [_VP, _I64, _VP, ctypes.POINTER(TuneResult)]),
    "cwt_plan_timing_start": (ctypes.c_int, [_VP, _I32]),
    "cwt_plan_create_from_wavelets": (ctypes.c_int, [ctypes.POINTER(_VP), _I64, ctypes.c_double,
                                                     ctypes.POINTER(ctypes.c_double), _I32,
                                                     ctypes.POINTER(ctypes.c_float), _I64,
                                                     ctypes.POINTER(PlanOpts), _VP]),
    "cwt_batches_workspace_size": (_SZ, [_VP, _I64]),
    "cwt_execute_batches": (ctypes.c_int, [_VP, _VP, _I64, _I32, _I64, _VP, _I64, _VP, _SZ, _VP]),
    "cwt_plan_timing_stop": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_float), _I32,
                                            ctypes.POINTER(_I32)]),
    "cwt_batch_workspace_size": (_SZ, [ctypes.POINTER(BatchItem), _I32]),
    "cwt_execute_batch": (ctypes.c_int, [ctypes.POINTER(BatchItem), _I32, _VP, _SZ, _VP]),
    "cwt_server_opts_init": (ctypes.c_int, [ctypes.POINTER(ServerOpts)]),
    "cwt_server_create": (ctypes.c_int, [ctypes.POINTER(_VP), _SZ, ctypes.POINTER(ServerOpts),
                                         _VP]),
    "cwt_server_destroy": (ctypes.c_int, [_VP]),
    "cwt_stream_open": (ctypes.c_int, [_VP, _VP, _I64, _I64, ctypes.POINTER(_VP)]),
    "cwt_stream_push": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_float), _I64, ctypes.c_uint64]),
    "cwt_stream_poll": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_float),
                                       ctypes.POINTER(ctypes.c_uint64),
                                       ctypes.POINTER(ctypes.c_uint64),
                                       ctypes.POINTER(ctypes.c_uint64)]),
    "cwt_server_flush": (ctypes.c_int, [_VP]),
    "cwt_stream_close": (ctypes.c_int, [_VP]),
    "cwt_server_get_stats": (ctypes.c_int, [_VP, ctypes.POINTER(ServerStats)]),
    "cwt_now_ns": (ctypes.c_uint64, []),
    "cwt_last_error": (ctypes.c_char_p, []),
}


def load():
    """Load libcwt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcwt.so is not built (%s); run "
                          "`python -c 'import __graft_entry__ as g; g.build()'`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc):
    if rc != CWT_OK:
        msg = load().cwt_last_error()
        raise CwtError(rc, msg.decode() if msg else "")
    return rc
