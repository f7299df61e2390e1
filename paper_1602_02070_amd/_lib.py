"""ctypes view of libcpca.so (the C ABI declared in include/cpca.h)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcpca.so")

OK, EINVAL, ENOCONV, ENOTSPD, ENAN, EHIP, ENOMEM = range(7)
STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", ENOCONV: "ENOCONV", ENOTSPD: "ENOTSPD",
                ENAN: "ENAN", EHIP: "EHIP", ENOMEM: "ENOMEM"}
MODES = {"fp64": 0, "fp32": 1, "fp32_ir": 2}

EXPORTS = ["cpca_version", "cpca_last_error", "cpca_create", "cpca_destroy",
           "cpca_set_stream", "cpca_frpcag", "cpca_decode", "cpca_decode_backward",
           "cpca_apply", "cpca_check_csr_host", "cpca_check_index_set_host",
           "cpca_set_profiling", "cpca_get_profile", "cpca_set_apply_config",
           "cpca_solve_batched", "cpca_approx_decode", "cpca_cluster_decode",
           "cpca_laplacian_lmax", "cpca_apply_noalloc", "cpca_knn_graph",
           "cpca_approx_decode2", "cpca_approx_decode3", "cpca_kron_reduce"]


class CpcaCsr(ctypes.Structure):
    _fields_ = [("n", c_int64), ("nnz", c_int64), ("rowptr", c_void_p),
                ("colind", c_void_p), ("vals", c_void_p)]


class CpcaInfo(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("outer_iters", c_int32), ("status", c_int32),
                ("reserved", c_int32), ("rel_residual", c_double),
                ("objective", c_double), ("ms", c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class CpcaApproxInfo(ctypes.Structure):
    _fields_ = [("k", c_int32), ("svd_sweeps", c_int32), ("iters_r", c_int32),
                ("iters_c", c_int32), ("status", c_int32), ("reserved", c_int32),
                ("rel_residual_r", c_double), ("rel_residual_c", c_double),
                ("scale", c_double), ("ms", c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class CpcaClusterInfo(ctypes.Structure):
    _fields_ = [("kmeans_iters", c_int32), ("cg_iters", c_int32), ("status", c_int32),
                ("reserved", c_int32), ("rel_residual", c_double), ("ms", c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class CpcaInstance(ctypes.Structure):
    _fields_ = [("p", c_int64), ("n", c_int64), ("rho_r", c_int64), ("rho_c", c_int64),
                ("omega_r", c_void_p), ("omega_c", c_void_p),
                ("Lr", ctypes.POINTER(CpcaCsr)), ("Lc", ctypes.POINTER(CpcaCsr)),
                ("Lr_til", ctypes.POINTER(CpcaCsr)), ("Lc_til", ctypes.POINTER(CpcaCsr)),
                ("lmax_r_til", c_double), ("lmax_c_til", c_double), ("Ytil", c_void_p)]


class CpcaTask(ctypes.Structure):
    _fields_ = [("instance", c_int32), ("reserved", c_int32), ("gamma_r", c_double),
                ("gamma_c", c_double), ("X_out", c_void_p), ("Xtil_out", c_void_p)]


_lib = None


def _declare(lib):
    st = c_int32
    P = c_void_p
    csr = POINTER(CpcaCsr)
    info = POINTER(CpcaInfo)
    sig = {
        "cpca_version": (c_char_p, []),
        "cpca_last_error": (c_char_p, []),
        "cpca_create": (st, [POINTER(c_void_p), P]),
        "cpca_destroy": (st, [P]),
        "cpca_set_stream": (st, [P, P]),
        "cpca_frpcag": (st, [P, c_int32, P, c_int64, c_int64, csr, csr, c_double, c_double,
                             c_double, c_double, c_int32, c_double, P, info]),
        "cpca_laplacian_lmax": (st, [P, csr, c_double, c_int32, POINTER(c_double), info]),
        "cpca_kron_reduce": (st, [P, csr, P, c_int64, c_double, c_int32, P, info]),
        "cpca_knn_graph": (st, [P, P, c_int64, c_int64, c_int32, c_int32, P, P, P, c_int64,
                                POINTER(c_int64), POINTER(c_double), P, info]),
        "cpca_decode": (st, [P, c_int32, P, c_int64, c_int64, P, P, c_int64, c_int64, csr, csr,
                             c_double, c_double, c_double, c_int32, P, P, info]),
        "cpca_decode_backward": (st, [P, c_int32, P, P, c_int64, c_int64, P, P, c_int64, c_int64,
                                      csr, csr, c_double, c_double, c_double, c_int32, P,
                                      POINTER(c_double), POINTER(c_double), info]),
        "cpca_apply": (st, [P, c_int32, P, P, c_int64, c_int64, P, c_int64, P, c_int64, csr, csr,
                            c_double, c_double, POINTER(c_double)]),
        "cpca_apply_noalloc": (st, [P, c_int32, P, P, c_int64, c_int64, P, c_int64, P, c_int64,
                                    csr, csr, c_double, c_double, POINTER(c_double)]),
        "cpca_check_csr_host": (st, [c_int64, c_int64, P, P, P]),
        "cpca_check_index_set_host": (st, [c_int64, c_int64, P]),
        "cpca_set_profiling": (st, [P, c_int32]),
        "cpca_get_profile": (st, [P, c_char_p, POINTER(c_int64), POINTER(c_double)]),
        "cpca_set_apply_config": (st, [P, c_int32, c_int32, c_int32]),
        "cpca_solve_batched": (st, [P, c_int32, POINTER(CpcaInstance), c_int32, POINTER(CpcaTask),
                                    c_int32, c_int32, c_double, c_int32, POINTER(CpcaInfo)]),
        "cpca_approx_decode": (st, [P, c_int32, P, c_int64, c_int64, P, P, c_int64, c_int64, csr,
                                    csr, c_double, c_double, c_int32, c_double, c_int32, P,
                                    POINTER(c_double), POINTER(CpcaApproxInfo)]),
        "cpca_approx_decode2": (st, [P, c_int32, P, c_int64, c_int64, P, c_int64, c_int64, csr, P,
                                     c_double, c_int32, c_double, c_int32, P, POINTER(c_double),
                                     POINTER(CpcaApproxInfo)]),
        "cpca_approx_decode3": (st, [P, c_int32, P, c_int64, c_int64, P, c_int64, c_int64, csr, P,
                                     c_double, c_int32, c_double, c_int32, P, POINTER(c_double),
                                     POINTER(CpcaApproxInfo)]),
        "cpca_cluster_decode": (st, [P, c_int32, P, c_int64, c_int64, P, c_int64, csr, c_int32, P,
                                     c_int32, c_double, c_int32, P, P, P,
                                     POINTER(CpcaClusterInfo)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def load(path: str | None = None):
    """Load libcpca.so. Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    _lib = _declare(ctypes.CDLL(path))
    return _lib


def last_error() -> str:
    return load().cpca_last_error().decode()
