"""ctypes binding of libgpp.so (declared in include/gpp.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  If the library is not built the import of any entry point fails
loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# the in-tree build, or a variant build (paper_2008_11326_amd.build --out)
# named by GPP_LIBRARY for measurements
LIB_PATH = os.environ.get("GPP_LIBRARY") or os.path.join(PKG, "libgpp.so")

GPP_OK = 0
STATUS = {0: "GPP_OK", 1: "GPP_ERR_INVALID", 2: "GPP_ERR_HIP",
          3: "GPP_ERR_NOMEM", 4: "GPP_ERR_WORKSPACE", 5: "GPP_ERR_UNSUPPORTED"}
MAX_NFREQ = 8
NOALLOC_SCRATCH_BYTES = 96 << 20  # GPP_NOALLOC_SCRATCH_BYTES of include/gpp.h


class GppError(RuntimeError):
    """A libgpp entry point returned a non-zero gpp_status."""

    def __init__(self, status: int, func: str, detail: str):
        self.status = status
        self.status_name = STATUS.get(status, str(status))
        super().__init__(f"{func}: {self.status_name}: {detail}")


class GppDims(C.Structure):
    _fields_ = [("number_bands", C.c_int64), ("nvband", C.c_int64),
                ("ncouls", C.c_int64), ("ngpown", C.c_int64),
                ("nfreq", C.c_int64)]


class GppInputs(C.Structure):
    _fields_ = [("aqsmtemp", C.c_void_p), ("aqsntemp", C.c_void_p),
                ("I_eps_array", C.c_void_p), ("wtilde_array", C.c_void_p),
                ("vcoul", C.c_void_p), ("wx_array", C.c_void_p)]


class GppPlanInfo(C.Structure):
    _fields_ = [("tuned", C.c_int32), ("from_cache", C.c_int32),
                ("bands_per_group", C.c_int32), ("schedule_order", C.c_int32),
                ("workgroups", C.c_int32), ("waves", C.c_int32),
                ("candidates", C.c_int32), ("schedule", C.c_int32),
                ("total_tiles", C.c_int64), ("tuned_ms", C.c_double)]


# (name, restype, argtypes) of every function include/*.h declares
_SIGNATURES = [
    ("gpp_sigma_fwd_workspace", C.c_size_t, [C.POINTER(GppDims)]),
    ("gpp_sigma_fwd", C.c_int,
     [C.POINTER(GppDims), C.POINTER(GppInputs), C.c_void_p, C.c_void_p,
      C.c_void_p, C.c_size_t, C.c_void_p]),
    ("gpp_sigma_fwd_noalloc", C.c_int,
     [C.POINTER(GppDims), C.POINTER(GppInputs), C.c_void_p, C.c_void_p, C.c_void_p]),
    ("gpp_sigma_qp", C.c_int,
     [C.POINTER(GppDims), C.POINTER(GppInputs), C.c_double, C.c_double, C.c_double,
      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    ("gpp_sigma_bwd_workspace", C.c_size_t, [C.POINTER(GppDims)]),
    ("gpp_sigma_bwd", C.c_int,
     [C.POINTER(GppDims), C.POINTER(GppInputs), C.c_void_p, C.c_void_p,
      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
      C.c_void_p]),
    ("gpp_plan_create", C.c_int,
     [C.c_int32, C.POINTER(GppDims), C.POINTER(C.c_void_p)]),
    ("gpp_plan_workspace", C.c_size_t, [C.c_void_p]),
    ("gpp_plan_get_info", C.c_int, [C.c_void_p, C.POINTER(GppPlanInfo)]),
    ("gpp_sigma_batched", C.c_int,
     [C.c_void_p, C.POINTER(GppInputs), C.c_void_p, C.c_void_p, C.c_void_p,
      C.c_size_t, C.c_void_p]),
    ("gpp_plan_destroy", None, [C.c_void_p]),
    ("gpp_status_string", C.c_char_p, [C.c_int]),
    ("gpp_last_error", C.c_char_p, []),
    ("gpp_version", C.c_int, []),
    # include/gpp_ladder.h
    ("gpp_ladder_steps", C.c_int32, []),
    ("gpp_ladder_name", C.c_char_p, [C.c_int32]),
    ("gpp_ladder_workspace", C.c_size_t, [C.c_int32, C.POINTER(GppDims)]),
    ("gpp_ladder_fwd", C.c_int,
     [C.c_int32, C.POINTER(GppDims), C.POINTER(GppInputs), C.c_void_p, C.c_void_p,
      C.c_void_p, C.c_size_t, C.c_void_p]),
    # include/gpp_microbench.h
    ("gpp_mb_fp64_fma", C.c_int,
     [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_double)]),
    ("gpp_mb_copy", C.c_int,
     [C.c_void_p, C.c_void_p, C.c_int64, C.c_int, C.c_void_p]),
    ("gpp_mb_read", C.c_int,
     [C.c_void_p, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]),
    ("gpp_mb_lds", C.c_int, [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]),
]
EXPORTED = [s[0] for s in _SIGNATURES]

_lib = None


def load():
    """Load libgpp.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; "
            "g.build()'` (the GPP path has no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, res, args in _SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, func: str):
    if status != GPP_OK:
        detail = load().gpp_last_error().decode(errors="replace")
        raise GppError(status, func, detail)


def dims_struct(number_bands, nvband, ncouls, ngpown, nfreq) -> GppDims:
    return GppDims(int(number_bands), int(nvband), int(ncouls), int(ngpown),
                   int(nfreq))
