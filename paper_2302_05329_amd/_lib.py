"""ctypes binding of libphenomd_hip.so (the C ABI declared in include/phenomd.h).

Argument marshalling only.  The library must have been built (see build.py); a missing
library is an error, never a silent fallback.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libphenomd_hip.so")

PD_OK = 0
PD_EINVAL = -1
PD_EDOMAIN = -2
PD_EHIP = -3
PD_ENOMEM = -4
PD_EUNSUPPORTED = -5

PD_FN_SIN, PD_FN_COS, PD_FN_ATAN, PD_FN_EXP, PD_FN_RCP = 0, 1, 2, 3, 4

PD_FP64 = 0
PD_MIXED = 1

PD_PARAM_MC_ETA = 0
PD_PARAM_LNMC_ETA_LND = 1
PD_PARAM_MC_Q = 2
PD_PARAM_M1M2 = 3

PD_OP_WAVEFORM = 0
PD_OP_LOGLIKE = 1
PD_OP_LOGLIKE_GRAD = 2
PD_OP_FISHER = 3
PD_OP_MISMATCH_GRAD = 4

PD_K_LOGLIKE_GRAD = 0
PD_K_LOGLIKE = 1
PD_K_FISHER = 2
PD_K_WAVEFORM = 3
PD_K_MISMATCH_INPUT = 4
PD_K_MISMATCH_FFT = 5
PD_K_MISMATCH_ADJ = 6
PD_K_OVERLAP = 7
PD_OVERLAP_MAX_STREAMS = 64
PD_NOALLOC_SCRATCH_BYTES = 64 << 20
PD_FLOW_FP32, PD_FLOW_BF16 = 0, 1


class PdGrid(ctypes.Structure):
    _fields_ = [("f0", ctypes.c_double), ("df", ctypes.c_double), ("n_bins", ctypes.c_int64),
                ("f_min", ctypes.c_double), ("f_ref", ctypes.c_double)]


PD_NETWORK_MAX_DETECTORS = 8


class PdDetector(ctypes.Structure):
    _fields_ = [("vertex", ctypes.c_double * 3), ("xarm", ctypes.c_double * 3), ("yarm", ctypes.c_double * 3)]


PD_TARGET_GW = 0
PD_TARGET_GAUSS = 1
PD_TARGET_GW_NETWORK = 2


class PdPosterior(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("grid", PdGrid), ("lam", ctypes.c_void_p), ("data", ctypes.c_void_p),
                ("inv_psd", ctypes.c_void_p), ("lo", ctypes.c_double * 7), ("hi", ctypes.c_double * 7),
                ("mu", ctypes.c_double * 7), ("isig2", ctypes.c_double * 7), ("n_det", ctypes.c_int),
                ("detectors", PdDetector * PD_NETWORK_MAX_DETECTORS), ("gmst", ctypes.c_double),
                ("orient", ctypes.c_double * 4)]


class PdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"phenomd error {code}: {msg}")
        self.code = code


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_INT = ctypes.c_int
_SZ = ctypes.c_size_t
_GRID = ctypes.POINTER(PdGrid)

# name -> (restype, argtypes); mirrors include/phenomd.h
SIGNATURES = {
    "pd_workspace_bytes": (_SZ, [_INT, _I64, _I64]),
    "pd_waveform_eval": (_INT, [_P, _I64, _INT, _GRID, _P, _INT, _P, _P, _P, _SZ, _P]),
    "pd_loglike_and_grad": (_INT, [_P, _I64, _INT, _GRID, _P, _P, _P, _INT, _P, _P, _P, _P, _SZ, _P]),
    "pd_loglike_and_grad_noalloc": (_INT, [_P, _I64, _INT, _GRID, _P, _P, _P, _INT, _P, _P, _P, _P]),
    "pd_fisher": (_INT, [_P, _I64, _INT, _GRID, _P, _P, _P, _P, _P, _SZ, _P]),
    "pd_mismatch_grad": (_INT, [_P, _I64, _INT, _GRID, _P, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "pd_network_workspace_bytes": (_SZ, [_I64, _I64, _INT]),
    "pd_network_loglike_and_grad": (_INT, [_P, _I64, _INT, _GRID, _P, _INT, ctypes.POINTER(PdDetector), ctypes.c_double,
                                           _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "pd_network_strain_workspace_bytes": (_SZ, [_I64, _I64]),
    "pd_network_strain": (_INT, [_P, _I64, _INT, _GRID, _P, ctypes.POINTER(PdDetector), ctypes.c_double, _P, _P, _P,
                                 _SZ, _P]),
    "pd_network_fisher_workspace_bytes": (_SZ, [_I64, _I64, _INT]),
    "pd_network_fisher": (_INT, [_P, _I64, _INT, _GRID, _P, _INT, ctypes.POINTER(PdDetector), ctypes.c_double, _P, _P,
                                 _P, _P, _SZ, _P]),
    "pd_fit_lambda_step": (_INT, [_P, _I64, _INT, _GRID, _P, _P, _P, ctypes.c_double, _P, _P, _P, _P, _SZ, _P]),
    "pd_posterior_workspace_bytes": (_SZ, [ctypes.c_void_p, _I64]),
    "pd_posterior_logp": (_INT, [ctypes.c_void_p, _P, _I64, _P, _P, _P, _SZ, _P]),
    "pd_hmc_workspace_bytes": (_SZ, [ctypes.c_void_p, _I64]),
    "pd_hmc_step": (_INT, [ctypes.c_void_p, _I64, _P, _P, _P, _P, _P, _INT, ctypes.c_double,
                           ctypes.POINTER(ctypes.c_double), _P, _P, _P, _SZ, _P]),
    "pd_hmc_step_dense": (_INT, [ctypes.c_void_p, _I64, _P, _P, _P, _P, _P, _INT, ctypes.c_double,
                                 ctypes.POINTER(ctypes.c_double), _P, _P, _P, _SZ, _P]),
    "pd_independence_mh": (_INT, [_I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "pd_rwmh_workspace_bytes": (_SZ, [ctypes.c_void_p, _I64]),
    "pd_rwmh_step": (_INT, [ctypes.c_void_p, _I64, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_double), _P, _P, _SZ,
                            _P]),
    "pd_rwmh_step_dense": (_INT, [ctypes.c_void_p, _I64, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_double), _P, _P,
                                  _SZ, _P]),
    "pd_elementary_eval": (_INT, [_INT, _P, _I64, _P, _P]),
    "pd_overlap_workspace_bytes": (_SZ, [_I64, _I64, _I64]),
    "pd_overlap": (_INT, [_P, _I64, _INT, _GRID, _P, _P, _I64, _P, _P, _P, _P, _P, _SZ, _P]),
    "pd_flow_param_count": (_I64, []),
    "pd_flow_workspace_bytes": (_SZ, [_I64]),
    "pd_flow_forward": (_INT, [_P, _P, _I64, _P, _P, _INT, _P]),
    "pd_flow_sample": (_INT, [_P, _P, _I64, _P, _P, _INT, _P]),
    "pd_flow_loss_grad": (_INT, [_P, _P, _I64, _P, _P, _P, _SZ, _INT, _P]),
    "pd_adam_step": (_INT, [_P, _P, _P, _P, _I64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, _I64, _P]),
    "pd_transition_frequencies": (_INT, [_P, _I64, _INT, _GRID, _P, _P, _P, _SZ, _P]),
    "pd_profile_enable": (_INT, [_INT]),
    "pd_profile_read": (_INT, [_INT, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "pd_last_error": (ctypes.c_char_p, []),
    "pd_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2302_05329_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(code):
    if code != PD_OK:
        raise PdError(code, lib().pd_last_error().decode())
    return code


def make_grid(f0, df, n_bins, f_min, f_ref):
    return PdGrid(float(f0), float(df), int(n_bins), float(f_min), float(f_ref))
