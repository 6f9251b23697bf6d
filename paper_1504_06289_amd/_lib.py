"""ctypes loader for libtc.so (the HIP library declared in include/tc.h).

Loading fails loudly when the shared library has not been built: there is no
fallback implementation anywhere in this package.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtc.so")

TC_OK = 0
TC_ERR_INVALID_ARG = 1
TC_ERR_WORKSPACE = 2
TC_ERR_UNSUPPORTED = 3
TC_ERR_HIP = 4

TC_FP64 = 0
TC_FP32 = 1
TC_BF16X3 = 2
TC_BF16X6 = 3
TC_OZAKI_I8 = 4
PRECISIONS = {"fp64": TC_FP64, "fp32": TC_FP32, "ozaki8": TC_OZAKI_I8, "bf16x3": TC_BF16X3,
              "bf16x6": TC_BF16X6}

TC_OP_CONVOLVE = 0
TC_OP_TEI_GRAM = 1
TC_OP_TEI_GRAM_BACKWARD = 2
TC_OP_AUTOTUNE = 3
TC_NOALLOC_SCRATCH_BYTES = 268435456

# the ABI symbols declared in include/tc.h
EXPORTS = ("tc_newton_kernel", "tc_convolve", "tc_tei_gram", "tc_tei_gram_backward",
           "tc_tei_gram_noalloc", "tc_batch_tune_set", "tc_batch_tune_get",
           "tc_workspace_bytes", "tc_status_string", "tc_version", "tc_tune_set",
           "tc_tune_get", "tc_autotune", "tc_profile_enable", "tc_profile_read",
           "tc_term_classes", "tc_coulomb", "tc_coulomb_workspace_bytes", "tc_density_fit",
           "tc_density_fit_workspace_bytes", "tc_tei_cholesky",
           "tc_tei_cholesky_workspace_bytes", "tc_lattice_sum", "tc_lattice_energy", "tc_nuclear",
           "tc_nuclear_workspace_bytes", "tc_canonical_to_tucker",
           "tc_canonical_to_tucker_workspace_bytes")

BATCH_ROUTES = {"auto": 0, "fork_join": 1, "queue": 2, "queue_t64": 3, "queue_k2": 4,
                "queue_t64_k2": 5}

TC_ALGO_AUTO = 0
TC_ALGO_DIRECT = 1
TC_ALGO_FFT = 2
ALGORITHMS = {"auto": TC_ALGO_AUTO, "direct": TC_ALGO_DIRECT, "fft": TC_ALGO_FFT}


class TcInstance(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int * 3),
        ("R_f", ctypes.c_int),
        ("R_N", ctypes.c_int),
        ("c", ctypes.c_void_p),
        ("p", ctypes.c_void_p * 3),
        ("U", ctypes.c_void_p * 3),
        ("J", ctypes.c_void_p),
        ("G_saved", ctypes.c_void_p),
    ]


class TcDensity(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int * 3),
        ("R_f", ctypes.c_int),
        ("R_rho", ctypes.c_int),
        ("R_N", ctypes.c_int),
        ("c", ctypes.c_void_p),
        ("p", ctypes.c_void_p * 3),
        ("U", ctypes.c_void_p * 3),
        ("V", ctypes.c_void_p * 3),
        ("d", ctypes.c_void_p),
        ("Jd", ctypes.c_void_p),
    ]


class TcNuclear(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int * 3),
        ("h", ctypes.c_double * 3),
        ("R_f", ctypes.c_int),
        ("R_N", ctypes.c_int),
        ("M", ctypes.c_int),
        ("c", ctypes.c_void_p),
        ("p", ctypes.c_void_p * 3),
        ("U", ctypes.c_void_p * 3),
        ("Z", ctypes.c_void_p),
        ("pos", ctypes.c_void_p),
        ("V", ctypes.c_void_p),
    ]


class TcError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)}")


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -m paper_1504_06289_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        pd = ctypes.POINTER(ctypes.c_double)
        L.tc_newton_kernel.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_double, pd, pd, vp, vp]
        L.tc_newton_kernel.restype = ctypes.c_int
        L.tc_convolve.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp,
                                  ctypes.c_int, vp, ctypes.c_size_t, vp]
        L.tc_convolve.restype = ctypes.c_int
        L.tc_tei_gram.argtypes = [ctypes.POINTER(TcInstance), ctypes.c_int, ctypes.c_int, vp,
                                  ctypes.c_size_t, vp]
        L.tc_tei_gram.restype = ctypes.c_int
        L.tc_tei_gram_noalloc.argtypes = [ctypes.POINTER(TcInstance), ctypes.c_int, ctypes.c_int,
                                          vp]
        L.tc_tei_gram_noalloc.restype = ctypes.c_int
        L.tc_tei_gram_backward.argtypes = [ctypes.POINTER(TcInstance), ctypes.c_int,
                                           ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int,
                                           vp, ctypes.c_size_t, vp]
        L.tc_tei_gram_backward.restype = ctypes.c_int
        L.tc_workspace_bytes.argtypes = [ctypes.c_int, ctypes.POINTER(TcInstance), ctypes.c_int,
                                         ctypes.c_int]
        L.tc_workspace_bytes.restype = ctypes.c_size_t
        L.tc_status_string.argtypes = [ctypes.c_int]
        L.tc_status_string.restype = ctypes.c_char_p
        L.tc_version.argtypes = []
        L.tc_version.restype = ctypes.c_int
        L.tc_tune_set.argtypes = [ctypes.c_int] * 5
        L.tc_tune_set.restype = ctypes.c_int
        L.tc_tune_get.argtypes = [ctypes.c_int] * 4
        L.tc_tune_get.restype = ctypes.c_int
        L.tc_batch_tune_set.argtypes = [ctypes.POINTER(TcInstance), ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int]
        L.tc_batch_tune_set.restype = ctypes.c_int
        L.tc_batch_tune_get.argtypes = [ctypes.POINTER(TcInstance), ctypes.c_int, ctypes.c_int]
        L.tc_batch_tune_get.restype = ctypes.c_int
        L.tc_autotune.argtypes = [ctypes.POINTER(TcInstance), ctypes.c_int, ctypes.c_int, vp,
                                  ctypes.c_size_t, vp, pd]
        L.tc_autotune.restype = ctypes.c_int
        L.tc_profile_enable.argtypes = [ctypes.c_int]
        L.tc_profile_enable.restype = ctypes.c_int
        L.tc_profile_read.argtypes = [ctypes.c_int, ctypes.c_void_p, pd,
                                      ctypes.POINTER(ctypes.c_long)]
        L.tc_profile_read.restype = ctypes.c_int
        L.tc_term_classes.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, vp]
        L.tc_term_classes.restype = ctypes.c_int
        L.tc_coulomb_workspace_bytes.argtypes = [ctypes.POINTER(TcDensity), ctypes.c_int]
        L.tc_coulomb_workspace_bytes.restype = ctypes.c_size_t
        L.tc_coulomb.argtypes = [ctypes.POINTER(TcDensity), ctypes.c_int, vp, ctypes.c_size_t,
                                 vp]
        L.tc_coulomb.restype = ctypes.c_int
        pi = ctypes.POINTER(ctypes.c_int)
        L.tc_density_fit_workspace_bytes.argtypes = [ctypes.c_int] * 3
        L.tc_density_fit_workspace_bytes.restype = ctypes.c_size_t
        L.tc_density_fit.argtypes = [ctypes.c_int, ctypes.c_int, vp, ctypes.c_double,
                                     ctypes.c_int, vp, vp, pi, pi, pd, vp, ctypes.c_size_t, vp]
        L.tc_density_fit.restype = ctypes.c_int
        L.tc_tei_cholesky_workspace_bytes.argtypes = [ctypes.c_int] * 4
        L.tc_tei_cholesky_workspace_bytes.restype = ctypes.c_size_t
        L.tc_tei_cholesky.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp,
                                      ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_double,
                                      ctypes.c_int, vp, pi, pi, pd, vp, ctypes.c_size_t, vp]
        L.tc_tei_cholesky.restype = ctypes.c_int
        L.tc_canonical_to_tucker_workspace_bytes.argtypes = [pi, ctypes.c_int, pi]
        L.tc_canonical_to_tucker_workspace_bytes.restype = ctypes.c_size_t
        L.tc_canonical_to_tucker.argtypes = [pi, ctypes.c_int, vp, ctypes.POINTER(vp), pi,
                                             ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                             ctypes.POINTER(vp), vp, vp, pi, vp, ctypes.c_size_t,
                                             vp]
        L.tc_canonical_to_tucker.restype = ctypes.c_int
        L.tc_nuclear_workspace_bytes.argtypes = [ctypes.POINTER(TcNuclear)]
        L.tc_nuclear_workspace_bytes.restype = ctypes.c_size_t
        L.tc_nuclear.argtypes = [ctypes.POINTER(TcNuclear), vp, ctypes.c_size_t, vp]
        L.tc_nuclear.restype = ctypes.c_int
        L.tc_lattice_sum.argtypes = [ctypes.c_int, pi, ctypes.c_int, ctypes.POINTER(vp),
                                     ctypes.POINTER(vp), vp]
        L.tc_lattice_sum.restype = ctypes.c_int
        L.tc_lattice_energy.argtypes = [ctypes.c_int, pi, ctypes.c_int, vp, pd,
                                        ctypes.POINTER(vp), ctypes.c_double, pd, vp,
                                        ctypes.c_size_t, vp]
        L.tc_lattice_energy.restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().tc_status_string(s).decode()


def check(status: int, where: str):
    if status != TC_OK:
        raise TcError(status, where)
