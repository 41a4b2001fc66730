"""ctypes declarations of the C ABI in include/gcge.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
import threading

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgcge.so")

GCGE_OK = 0
GCGE_NOT_CONVERGED = 1
GCGE_ERR_INVALID_ARG = -1
GCGE_ERR_NOT_SPD = -2
GCGE_ERR_OOM = -3
GCGE_ERR_HIP = -4
GCGE_ERR_INTERNAL = -5

B_IDENTITY, B_DIAG, B_CSR = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1

PROF_NAMES = ["cg_spmm", "cg_update_r", "cg_update_xp", "rotation_gemm", "p_gemm", "gram", "amg_vcycle", "cg_fold"]
STEP_NAMES = ["init", "step2_orth", "step3_rr", "step4_conv", "step5_p", "step6_cg", "final_check", "total"]

# Every symbol declared in include/gcge.h.
EXPORTED = [
    "gcge_create", "gcge_set_option_i", "gcge_set_option_d", "gcge_set_stream", "gcge_set_initial_vectors",
    "gcge_solve", "gcge_update_values", "gcge_eig_grad", "gcge_destroy", "gcge_last_error", "gcge_spmm",
    "gcge_spmm_f32", "gcge_shifted_spmm", "gcge_residual", "gcge_gram", "gcge_gemm_update", "gcge_cg",
    "gcge_orth", "gcge_orth_mbo", "gcge_small_eigh", "gcge_dense_eig", "gcge_p_hat", "gcge_pattern_grad",
    "gcge_amg_create", "gcge_amg_levels", "gcge_amg_aggregates", "gcge_amg_apply", "gcge_pcg", "gcge_amg_destroy",
    "gcge_gram_noalloc",
]

# Size of the library's device array behind gcge_gram_noalloc (GCGE_NOALLOC_SCRATCH_BYTES).
NOALLOC_SCRATCH_BYTES = 32 << 20


class GcgeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gcge error {code}: {msg}")
        self.code = code


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("rowptr", ctypes.c_void_p),
                ("colind", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("nconv", ctypes.c_int32), ("moves", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("cg_iterations", ctypes.c_int64),
                ("spmm_columns", ctypes.c_int64), ("time_ms", ctypes.c_double * 8),
                ("max_rel_residual", ctypes.c_double), ("orth_error", ctypes.c_double),
                ("prof_ms", ctypes.c_double * 8), ("prof_launches", ctypes.c_int64 * 8),
                ("prof_columns", ctypes.c_int64 * 8), ("prof_full_ms", ctypes.c_double * 4),
                ("prof_full_launches", ctypes.c_int64 * 4)]

    def as_dict(self):
        skip = ("time_ms", "reserved0", "prof_ms", "prof_launches", "prof_columns", "prof_full_ms",
                "prof_full_launches")
        d = {k: getattr(self, k) for k, _ in self._fields_ if k not in skip}
        d["time_ms"] = {name: self.time_ms[i] for i, name in enumerate(STEP_NAMES)}
        d["prof"] = {name: {"ms": self.prof_ms[i], "launches": self.prof_launches[i],
                            "columns": self.prof_columns[i]} for i, name in enumerate(PROF_NAMES)}
        for i, name in enumerate(PROF_NAMES[:3]):
            d["prof"][name]["full_ms"] = self.prof_full_ms[i]
            d["prof"][name]["full_launches"] = self.prof_full_launches[i]
        return d


_lock = threading.Lock()
_lib = None

c_int, c_int64, c_double, c_void_p = ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
P = ctypes.POINTER


def load():
    """Load libgcge.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                              f"g.build()'` (hipcc, gfx950)")
        lib = ctypes.CDLL(LIB_PATH)
        sig = {
            "gcge_create": (c_int, [P(Csr), c_int, c_void_p, c_int, c_double, P(c_void_p)]),
            "gcge_set_option_i": (c_int, [c_void_p, ctypes.c_char_p, c_int64]),
            "gcge_set_option_d": (c_int, [c_void_p, ctypes.c_char_p, c_double]),
            "gcge_set_stream": (c_int, [c_void_p, c_void_p]),
            "gcge_set_initial_vectors": (c_int, [c_void_p, c_void_p, c_int64, c_int]),
            "gcge_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_int64, P(Stats)]),
            "gcge_update_values": (c_int, [c_void_p, c_void_p, c_void_p]),
            "gcge_eig_grad": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
            "gcge_destroy": (None, [c_void_p]),
            "gcge_last_error": (ctypes.c_char_p, [c_void_p]),
            "gcge_spmm": (c_int, [P(Csr), c_void_p, c_int64, c_int, c_void_p, c_int64, c_void_p]),
            "gcge_spmm_f32": (c_int, [c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_int, c_void_p,
                                      c_int64, c_void_p]),
            "gcge_shifted_spmm": (c_int, [P(Csr), c_int, c_void_p, c_void_p, c_void_p, c_int64, c_int, c_void_p,
                                          c_int64, c_void_p]),
            "gcge_residual": (c_int, [P(Csr), c_int, c_void_p, c_void_p, c_void_p, c_int64, c_int, c_void_p,
                                      c_int64, c_void_p, c_void_p, c_void_p]),
            "gcge_gram": (c_int, [c_int64, c_void_p, c_int64, c_int, c_void_p, c_int64, c_int, c_void_p, c_void_p,
                                  c_void_p]),
            "gcge_gram_noalloc": (c_int, [c_int64, c_void_p, c_int64, c_int, c_void_p, c_int64, c_int, c_void_p,
                                          c_void_p, c_void_p]),
            "gcge_gemm_update": (c_int, [c_int64, c_void_p, c_int64, c_int, c_void_p, c_int, c_double, c_double,
                                         c_void_p, c_int64, c_void_p]),
            "gcge_cg": (c_int, [P(Csr), c_int, c_void_p, c_double, c_void_p, c_int64, c_int, c_int, c_double, c_int,
                                c_void_p, c_int64, c_void_p, c_void_p]),
            "gcge_orth": (c_int, [c_int64, c_int, c_void_p, c_void_p, c_int64, c_int, c_void_p, c_int64, c_int,
                                  c_void_p, c_void_p]),
            "gcge_orth_mbo": (c_int, [c_int64, c_int, c_void_p, c_void_p, c_int64, c_int, c_void_p, c_int64, c_int,
                                      c_int, c_void_p, c_void_p]),
            "gcge_small_eigh": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_int]),
            "gcge_dense_eig": (c_int, [c_int, c_void_p, c_int64, c_int, c_void_p, c_void_p, c_int64, c_void_p]),
            "gcge_p_hat": (c_int, [c_int, c_int, c_void_p, c_int, c_int, c_int, c_double, c_void_p, c_void_p]),
            "gcge_pattern_grad": (c_int, [c_int64, c_int64, c_void_p, c_void_p, c_void_p, c_int64, c_int, c_void_p,
                                          c_void_p, c_void_p]),
            "gcge_amg_create": (c_int, [P(Csr), c_int, c_int, c_double, c_void_p, P(c_void_p)]),
            "gcge_amg_levels": (c_int, [c_void_p, P(c_int), c_void_p, c_void_p, c_int]),
            "gcge_amg_aggregates": (c_int, [c_void_p, c_int, c_void_p]),
            "gcge_amg_apply": (c_int, [c_void_p, c_void_p, c_int64, c_int, c_void_p, c_int64, c_void_p]),
            "gcge_pcg": (c_int, [P(Csr), c_void_p, c_void_p, c_int64, c_int, c_int, c_double, c_void_p, c_int64,
                                 c_void_p, c_void_p]),
            "gcge_amg_destroy": (None, [c_void_p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
        return lib


def check(code: int, handle=None):
    if code < 0:
        msg = load().gcge_last_error(handle)
        raise GcgeError(code, msg.decode() if msg else "")
    return code
