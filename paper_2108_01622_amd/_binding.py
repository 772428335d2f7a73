"""ctypes binding of the C ABI in include/lhaf.h (argument marshalling only).

Every numeric step runs in the HIP library; PyTorch provides device memory
and the current HIP stream.  Loading fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LHAF_LIBRARY") or os.path.join(_HERE, "_lib", "liblhaf.so")

LH_SUM_ET, LH_SUM_FDS = 0, 1
LH_ACC_FP64, LH_ACC_DD, LH_ACC_DD_COMP = 0, 1, 2

_SUMS = {"et": LH_SUM_ET, "fds": LH_SUM_FDS}
# "ddc": double-double accumulation with compensated per-term recurrences
# (values only: lhaf, repeated, batched without saved/grads, noalloc, mixed)
_ACCS = {"fp64": LH_ACC_FP64, "dd": LH_ACC_DD, "ddc": LH_ACC_DD_COMP}


class LhOpts(ctypes.Structure):
    _fields_ = [
        ("sum", ctypes.c_int32),
        ("acc", ctypes.c_int32),
        ("term_begin", ctypes.c_int64),
        ("term_end", ctypes.c_int64),
        ("scaled", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
        ("workspace", ctypes.c_void_p),
        ("ws_bytes", ctypes.c_size_t),
        ("out_lo", ctypes.c_void_p),
        ("saved", ctypes.c_void_p),
        ("saved_count", ctypes.c_int64),
        ("grads", ctypes.c_void_p),
        ("grads_count", ctypes.c_int64),
    ]


class LhafError(RuntimeError):
    pass


_lib = None
TUNE_CACHE = os.path.join(_HERE, "tune", "mi355x.txt")


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LhafError(f"HIP library not built: {LIB_PATH} (run paper_2108_01622_amd.build)")
        if "LHAF_TUNE_CACHE" not in os.environ and os.path.exists(TUNE_CACHE):
            os.environ["LHAF_TUNE_CACHE"] = TUNE_CACHE  # read lazily by the library
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        P = ctypes.POINTER
        L.lh_opts_default.argtypes = [P(LhOpts)]
        L.lh_opts_default.restype = None
        L.lh_status_string.argtypes = [i32]
        L.lh_status_string.restype = ctypes.c_char_p
        L.lhaf_schedule_count.restype = i32
        L.lhaf_term_count.argtypes = [i32, vp, i32]
        L.lhaf_term_count.restype = i64
        L.lhaf_plan_pairs.argtypes = [i32, vp, vp, vp]
        L.lhaf_plan_pairs.restype = i32
        L.lhaf.argtypes = [vp, i64, vp, i32, vp, vp, P(LhOpts), vp]
        L.lhaf.restype = i32
        L.lhaf_repeated.argtypes = [vp, i64, vp, vp, i32, vp, vp, P(LhOpts), vp]
        L.lhaf_repeated.restype = i32
        L.lhaf_batched_workspace.argtypes = [i32, vp, vp, P(LhOpts)]
        L.lhaf_batched_workspace.restype = sz
        L.lhaf_batched.argtypes = [i32, vp, i64, i64, vp, i64, vp, vp, vp, vp, vp, vp, sz,
                                   P(LhOpts), vp]
        L.lhaf_batched.restype = i32
        L.lhaf_batched_noalloc.argtypes = [i32, vp, i64, i64, vp, i64, vp, vp, vp, vp, vp,
                                           P(LhOpts), vp]
        L.lhaf_batched_noalloc.restype = i32
        L.lhaf_noalloc_scratch_bytes.argtypes = []
        L.lhaf_noalloc_scratch_bytes.restype = sz
        L.lhaf_real.argtypes = [vp, i64, vp, vp, i32, vp, vp, P(LhOpts), vp]
        L.lhaf_real.restype = i32
        L.lhaf_mixed.argtypes = [vp, i64, vp, vp, i32, vp, vp, P(LhOpts), vp]
        L.lhaf_mixed.restype = i32
        L.lhaf_chain.argtypes = [vp, i64, vp, vp, i32, i32, i32, vp, vp, P(LhOpts), vp]
        L.lhaf_chain.restype = i32
        L.lhaf_gammas.argtypes = [vp, i64, vp, i64, vp, i32, i32, vp, vp, P(LhOpts), vp]
        L.lhaf_gammas.restype = i32
        L.lhaf_saved_count.argtypes = [i32, vp, vp, P(LhOpts)]
        L.lhaf_saved_count.restype = i64
        L.lhaf_grads_count.argtypes = [i32, vp, vp]
        L.lhaf_grads_count.restype = i64
        L.lhaf_backward_workspace.argtypes = [i32, vp, vp, i32, P(LhOpts)]
        L.lhaf_backward_workspace.restype = sz
        L.lhaf_backward.argtypes = [i32, vp, i64, i64, vp, i64, vp, vp, vp, vp, vp, vp, i32, vp,
                                    sz, P(LhOpts), vp]
        L.lhaf_backward.restype = i32
        _lib = L
    return _lib


EXPORTED = ["lh_opts_default", "lh_status_string", "lhaf_schedule_count", "lhaf_term_count",
            "lhaf_plan_pairs", "lhaf", "lhaf_repeated", "lhaf_batched_workspace", "lhaf_batched",
            "lhaf_batched_noalloc", "lhaf_noalloc_scratch_bytes",
            "lhaf_real", "lhaf_mixed", "lhaf_chain", "lhaf_gammas", "lhaf_saved_count", "lhaf_grads_count", "lhaf_backward_workspace",
            "lhaf_backward"]


def check(status: int) -> None:
    if status != 0:
        raise LhafError(f"lhaf status {status}: {lib().lh_status_string(status).decode()}")


def make_opts(sum="fds", acc="dd", term_begin=0, term_end=-1, scaled=True, schedule=-1,
              workspace=None, out_lo=None, saved=None, grads=None) -> LhOpts:
    o = LhOpts()
    lib().lh_opts_default(ctypes.byref(o))
    o.sum = _SUMS[sum]
    o.acc = _ACCS[acc]
    o.term_begin = int(term_begin)
    o.term_end = int(term_end)
    o.scaled = 1 if scaled else 0
    o.schedule = int(schedule)
    if workspace is not None:
        o.workspace = ctypes.c_void_p(workspace.data_ptr())
        o.ws_bytes = workspace.numel() * workspace.element_size()
    if out_lo is not None:
        o.out_lo = ctypes.c_void_p(out_lo.data_ptr())
    if saved is not None:
        o.saved = ctypes.c_void_p(saved.data_ptr())
        o.saved_count = saved.numel()
    if grads is not None:
        o.grads = ctypes.c_void_p(grads.data_ptr())
        o.grads_count = grads.numel()
    return o


def host_ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def term_count(N: int, r=None, sum="fds") -> int:
    if r is not None:
        r = np.ascontiguousarray(r, dtype=np.int32)
        N = len(r)
    v = int(lib().lhaf_term_count(int(N), host_ptr(r) if r is not None else None, _SUMS[sum]))
    if v < 0:
        check(-v)
    return v


def plan_pairs(N: int, r=None):
    """Host planner output: (pos[2H], eta[H]) -- pos entries index the
    problem's index list, -1 is the padding vertex."""
    if r is not None:
        r = np.ascontiguousarray(r, dtype=np.int32)
        N = len(r)
    pos = np.zeros(128, dtype=np.int32)
    eta = np.zeros(64, dtype=np.int32)
    H = int(lib().lhaf_plan_pairs(int(N), host_ptr(r) if r is not None else None,
                                  host_ptr(pos), host_ptr(eta)))
    if H < 0:
        check(-H)
    return pos[: 2 * H].copy(), eta[:H].copy()
