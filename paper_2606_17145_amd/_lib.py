"""ctypes binding of libsrgrav.so: argument marshalling only.

Every step of the computation runs in the HIP library; this module converts
torch tensors to device pointers and C structs and turns error codes into
exceptions.  There is no fallback: if the library is missing, every call
raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsrgrav.so")

SR_OPEN_BH, SR_OPEN_RELATIVE = 0, 1
SR_FP64, SR_FP32, SR_FP32_ACC64 = 0, 1, 2
PRECISIONS = {"fp64": SR_FP64, "fp32": SR_FP32, "fp32_acc64": SR_FP32_ACC64}
CRITERIA = {"bh": SR_OPEN_BH, "relative": SR_OPEN_RELATIVE}
EXPORTED = ("tree_build", "tree_drift", "shortrange_accel", "shortrange_accel_noalloc", "shortrange_accel_adjoint", "tree_node_count",
            "tree_export", "tree_free", "srgrav_last_error", "sr_axpy", "srgrav_timing",
            "srgrav_timing_read", "srgrav_inject_alloc_failure", "tree_walk_stats", "pm_create", "pm_accel", "pm_accel_adjoint", "pm_free", "sph_density")
PHASES = ("tree_build", "traverse", "eval", "reduce", "adjoint_eval", "adjoint_reduce", "pushdown",
          "pm_deposit", "pm_fft", "pm_green", "pm_interp", "pm_stencil", "pm_adj_gather", "pm_sort", "sph_iter", "drift")


class SrgravError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"srgrav error {code}: {msg}")
        self.code = code


class SrParams(C.Structure):
    _fields_ = [("G", C.c_double), ("r_s", C.c_double), ("r_cut", C.c_double),
                ("criterion", C.c_int32), ("theta", C.c_double), ("alpha", C.c_double),
                ("precision", C.c_int32)]


class SrTreeExport(C.Structure):
    _fields_ = [(name, C.c_void_p) for name in
                ("key_hi", "key_lo", "perm", "level", "first", "count", "parent", "skip", "corner",
                 "M", "com", "M32", "comX", "side")]


_lib = None


def lib():
    """Load libsrgrav.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        vp, i64, d = C.c_void_p, C.c_int64, C.c_double
        L.tree_build.argtypes = [vp, vp, vp, d, i64, d, C.c_int32, vp, C.POINTER(vp)]
        L.tree_drift.argtypes = [vp, vp, vp]
        L.tree_drift.restype = C.c_int
        L.shortrange_accel.argtypes = [vp, C.POINTER(SrParams), vp, i64, vp, vp, vp, C.POINTER(i64), vp]
        L.shortrange_accel_noalloc.argtypes = [vp, C.POINTER(SrParams), vp, i64, vp, vp, vp, vp]
        L.shortrange_accel_adjoint.argtypes = [vp, C.POINTER(SrParams), vp, i64, vp, vp, vp, vp, i64, vp]
        L.tree_node_count.argtypes = [vp, C.POINTER(i64)]
        L.tree_export.argtypes = [vp, C.POINTER(SrTreeExport), vp]
        L.sr_axpy.argtypes = [vp, C.c_int32, vp, C.c_int32, d, i64, vp]
        L.sr_axpy.restype = C.c_int
        L.srgrav_timing.argtypes = [C.c_int32]
        L.srgrav_timing.restype = C.c_int
        L.srgrav_timing_read.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.srgrav_timing_read.restype = C.c_int
        L.srgrav_inject_alloc_failure.argtypes = [C.c_int64]
        L.srgrav_inject_alloc_failure.restype = C.c_int
        L.tree_walk_stats.argtypes = [vp, C.POINTER(C.c_int64)]
        L.tree_walk_stats.restype = C.c_int
        L.tree_free.argtypes = [vp]
        L.tree_free.restype = None
        L.pm_create.argtypes = [C.c_int32, C.POINTER(vp)]
        L.pm_create.restype = C.c_int
        L.pm_accel.argtypes = [vp, vp, vp, i64, d, d, d, vp, vp]
        L.pm_accel.restype = C.c_int
        L.pm_accel_adjoint.argtypes = [vp, vp, vp, i64, d, d, d, vp, vp, vp, vp]
        L.pm_accel_adjoint.restype = C.c_int
        L.sph_density.argtypes = [vp, d, vp, vp, C.POINTER(i64), vp]
        L.sph_density.restype = C.c_int
        L.pm_free.argtypes = [vp]
        L.pm_free.restype = None
        L.srgrav_last_error.restype = C.c_char_p
        for name in ("tree_build", "shortrange_accel", "shortrange_accel_noalloc", "shortrange_accel_adjoint", "tree_node_count",
                     "tree_export"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(rc: int):
    if rc != 0:
        raise SrgravError(rc, lib().srgrav_last_error().decode())


def ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def stream_handle():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_params(params: dict) -> SrParams:
    return SrParams(float(params.get("G", 1.0)), float(params["r_s"]), float(params["r_cut"]),
                    CRITERIA[params.get("criterion", "bh")], float(params.get("theta", 0.5)),
                    float(params.get("alpha", 0.0)), PRECISIONS[params.get("precision", "fp64")])


def timing(enable: bool):
    """Start (resetting) or stop phase timing with HIP events in the library."""
    check(lib().srgrav_timing(1 if enable else 0))


def timing_read() -> dict:
    """{phase: (total_ms, launches)} of the phases timed since timing(True)."""
    ms = (C.c_double * len(PHASES))()
    calls = (C.c_int64 * len(PHASES))()
    check(lib().srgrav_timing_read(ms, calls))
    return {name: (ms[k], calls[k]) for k, name in enumerate(PHASES)}
