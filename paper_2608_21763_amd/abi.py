"""ctypes binding of the C-ABI in ``include/s2w.h`` (argument marshalling only).

Every entry point maps one-to-one onto an ``s2w_*`` function.  Nothing here
computes any part of the map; a missing library raises instead of falling back.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libs2w.so")

DTYPES = {"f32": 0, "bf16": 1, "f16": 2}
DIFF_NONE = 0
DIFF_BACKWARD = 1
LAYOUTS = {"auto": 0, "single": 1, "batched": 2, "direct": 3}
PRODUCTS = {"auto": 0, "bf16": 1, "f16": 2}

STATUS = {0: "S2W_OK", 1: "S2W_EINVAL", 2: "S2W_ENOMEM", 3: "S2W_ESTATE", 4: "S2W_EUNSUPPORTED", 5: "S2W_EHIP"}


class S2WError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        self.code = STATUS.get(status, str(status))
        super().__init__(f"{where}: {self.code}" + (f" ({detail})" if detail else ""))


class Desc(ctypes.Structure):
    _fields_ = [("nsub", ctypes.c_int32), ("ngrid", ctypes.c_int32), ("nobs", ctypes.c_int32),
                ("nt", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("diff", ctypes.c_int32),
                ("g_dtype", ctypes.c_int32), ("f_dtype", ctypes.c_int32), ("dt", ctypes.c_double),
                ("layout", ctypes.c_int32), ("products", ctypes.c_int32)]


class BlttDesc(ctypes.Structure):
    _fields_ = [("nrow", ctypes.c_int32), ("ncol", ctypes.c_int32), ("nt", ctypes.c_int32),
                ("max_batch", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("fused_wg_per_cu", ctypes.c_int32), ("fused_rows", ctypes.c_int32), ("adj_cols", ctypes.c_int32),
                ("adj_splits", ctypes.c_int32), ("batch_path_min_b", ctypes.c_int32), ("gemm_cfg", ctypes.c_int32),
                ("fgemm_splits", ctypes.c_int32), ("fgemm_lds", ctypes.c_int32), ("gemm32_cfg", ctypes.c_int32),
                ("gemm32_cfg_k", ctypes.c_int32), ("gemm32_splits", ctypes.c_int32), ("adj32_splits", ctypes.c_int32),
                ("hadj_tile_f", ctypes.c_int32), ("hadj_tile_g", ctypes.c_int32), ("mid_rupts", ctypes.c_int32),
                ("adj32_cfg", ctypes.c_int32)]


EXPORTS = ["s2w_abi_version", "s2w_status_string", "s2w_last_error", "s2w_plan_create", "s2w_plan_destroy",
           "s2w_query_sizes", "s2w_bind_memory", "s2w_set_operators", "s2w_forward", "s2w_adjoint",
           "s2w_set_tuning", "s2w_get_tuning", "s2w_transform_length", "s2w_set_profile_events", "s2w_plan_layout",
           "s2w_bltt_create", "s2w_bltt_destroy", "s2w_bltt_query_sizes", "s2w_bltt_bind_memory",
           "s2w_bltt_set_blocks", "s2w_bltt_apply", "s2w_bltt_adjoint", "s2w_bltt_last_error", "s2w_forward_noalloc",
           "s2w_forward_displacement"]

_lib = None


def load_library(path: str | None = None):
    """Load ``libs2w.so``; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with paper_2608_21763_amd/build_lib.py (or __graft_entry__.build())")
    lib = ctypes.CDLL(p)
    P, vp, i32, i64, u64 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    plan_p = vp
    lib.s2w_abi_version.restype = i32
    lib.s2w_status_string.restype = ctypes.c_char_p
    lib.s2w_status_string.argtypes = [i32]
    lib.s2w_last_error.restype = ctypes.c_char_p
    lib.s2w_last_error.argtypes = [plan_p]
    lib.s2w_plan_create.argtypes = [P(Desc), i32, P(plan_p)]
    lib.s2w_plan_destroy.argtypes = [plan_p]
    lib.s2w_query_sizes.argtypes = [plan_p, P(u64), P(u64)]
    lib.s2w_bind_memory.argtypes = [plan_p, vp, u64, vp, u64]
    lib.s2w_set_operators.argtypes = [plan_p, vp, vp, i64, i64, vp]
    lib.s2w_forward.argtypes = [plan_p, vp, i32, vp, vp]
    lib.s2w_adjoint.argtypes = [plan_p, vp, i32, vp, vp]
    lib.s2w_forward_noalloc.argtypes = [plan_p, vp, i32, vp, vp]
    lib.s2w_forward_displacement.argtypes = [plan_p, vp, i32, vp, vp, P(i32), i32, vp]
    lib.s2w_set_tuning.argtypes = [plan_p, P(Tuning)]
    lib.s2w_get_tuning.argtypes = [plan_p, P(Tuning)]
    lib.s2w_transform_length.argtypes = [plan_p, P(i32)]
    lib.s2w_set_profile_events.argtypes = [plan_p, vp, vp]
    lib.s2w_plan_layout.argtypes = [plan_p, P(i32)]
    lib.s2w_bltt_create.argtypes = [P(BlttDesc), i32, P(vp)]
    lib.s2w_bltt_destroy.argtypes = [vp]
    lib.s2w_bltt_query_sizes.argtypes = [vp, P(u64), P(u64)]
    lib.s2w_bltt_bind_memory.argtypes = [vp, vp, u64, vp, u64]
    lib.s2w_bltt_set_blocks.argtypes = [vp, vp, i64, i64, vp]
    lib.s2w_bltt_apply.argtypes = [vp, vp, i32, vp, vp]
    lib.s2w_bltt_adjoint.argtypes = [vp, vp, i32, vp, vp]
    lib.s2w_bltt_last_error.restype = ctypes.c_char_p
    lib.s2w_bltt_last_error.argtypes = [vp]
    for name in EXPORTS:
        if name not in ("s2w_abi_version", "s2w_status_string", "s2w_last_error", "s2w_bltt_last_error"):
            getattr(lib, name).restype = i32
    if path is None:
        _lib = lib
    return lib


class Plan:
    """Thin owner of an ``s2w_plan*``; methods mirror the C entry points."""

    def __init__(self, nsub: int, ngrid: int, nobs: int, nt: int, max_batch: int = 1, dt: float = 1.0,
                 diff: int = DIFF_BACKWARD, g_dtype: str = "f32", f_dtype: str = "f32", device: int = 0,
                 layout: str = "auto", products: str = "auto"):
        self.lib = load_library()
        self.desc = Desc(nsub, ngrid, nobs, nt, max_batch, diff, DTYPES[g_dtype], DTYPES[f_dtype], dt,
                         LAYOUTS[layout], PRODUCTS[products])
        self.handle = ctypes.c_void_p()
        st = self.lib.s2w_plan_create(ctypes.byref(self.desc), device, ctypes.byref(self.handle))
        if st != 0:
            raise S2WError(st, "s2w_plan_create")

    def _check(self, st: int, where: str):
        if st != 0:
            msg = self.lib.s2w_last_error(self.handle)
            raise S2WError(st, where, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self.lib.s2w_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query_sizes(self):
        op, ws = ctypes.c_uint64(), ctypes.c_uint64()
        self._check(self.lib.s2w_query_sizes(self.handle, ctypes.byref(op), ctypes.byref(ws)), "s2w_query_sizes")
        return op.value, ws.value

    def transform_length(self) -> int:
        L = ctypes.c_int32()
        self._check(self.lib.s2w_transform_length(self.handle, ctypes.byref(L)), "s2w_transform_length")
        return L.value

    def layout(self) -> str:
        v = ctypes.c_int32()
        self._check(self.lib.s2w_plan_layout(self.handle, ctypes.byref(v)), "s2w_plan_layout")
        return {1: "single", 2: "batched", 3: "direct"}[v.value]

    def bind(self, op_ptr: int, op_bytes: int, ws_ptr: int, ws_bytes: int):
        self._check(self.lib.s2w_bind_memory(self.handle, op_ptr, op_bytes, ws_ptr, ws_bytes), "s2w_bind_memory")

    def set_operators(self, g_ptr: int, f_ptr: int, row0: int, nrows: int, stream: int = 0):
        self._check(self.lib.s2w_set_operators(self.handle, g_ptr, f_ptr, row0, nrows, stream), "s2w_set_operators")

    def forward(self, s_ptr: int, B: int, y_ptr: int, stream: int = 0):
        self._check(self.lib.s2w_forward(self.handle, s_ptr, B, y_ptr, stream), "s2w_forward")

    def adjoint(self, r_ptr: int, B: int, gs_ptr: int, stream: int = 0):
        self._check(self.lib.s2w_adjoint(self.handle, r_ptr, B, gs_ptr, stream), "s2w_adjoint")

    def forward_noalloc(self, s_ptr: int, B: int, y_ptr: int, stream: int = 0):
        self._check(self.lib.s2w_forward_noalloc(self.handle, s_ptr, B, y_ptr, stream), "s2w_forward_noalloc")

    def forward_displacement(self, s_ptr: int, B: int, y_ptr: int, m_ptr: int, times=None, ntimes: int = 0,
                             stream: int = 0):
        """times: a sequence of steps (marshalled to an int32 array), or None with ntimes = nt."""
        arr = None
        if times is not None:
            arr = (ctypes.c_int32 * len(times))(*[int(t) for t in times])
            ntimes = len(times)
        self._check(self.lib.s2w_forward_displacement(self.handle, s_ptr, B, y_ptr, m_ptr, arr, ntimes, stream),
                    "s2w_forward_displacement")

    def set_profile_events(self, begin: int = 0, end: int = 0):
        """hipEvent_t handles (ints) recorded around the dominant kernel of later calls; 0, 0 stops."""
        self._check(self.lib.s2w_set_profile_events(self.handle, begin or None, end or None), "s2w_set_profile_events")

    def get_tuning(self) -> dict:
        t = Tuning()
        self._check(self.lib.s2w_get_tuning(self.handle, ctypes.byref(t)), "s2w_get_tuning")
        return {n: getattr(t, n) for n, _ in Tuning._fields_}

    def set_tuning(self, **kw):
        t = Tuning(**{n: int(kw.get(n, 0)) for n, _ in Tuning._fields_})
        self._check(self.lib.s2w_set_tuning(self.handle, ctypes.byref(t)), "s2w_set_tuning")


class Bltt:
    """Thin owner of an ``s2w_bltt*`` (one block lower-triangular Toeplitz operator)."""

    def __init__(self, nrow: int, ncol: int, nt: int, max_batch: int = 1, device: int = 0):
        self.lib = load_library()
        self.desc = BlttDesc(nrow, ncol, nt, max_batch)
        self.handle = ctypes.c_void_p()
        st = self.lib.s2w_bltt_create(ctypes.byref(self.desc), device, ctypes.byref(self.handle))
        if st != 0:
            raise S2WError(st, "s2w_bltt_create")

    def _check(self, st: int, where: str):
        if st != 0:
            msg = self.lib.s2w_bltt_last_error(self.handle)
            raise S2WError(st, where, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self.lib.s2w_bltt_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query_sizes(self):
        op, ws = ctypes.c_uint64(), ctypes.c_uint64()
        self._check(self.lib.s2w_bltt_query_sizes(self.handle, ctypes.byref(op), ctypes.byref(ws)),
                    "s2w_bltt_query_sizes")
        return op.value, ws.value

    def bind(self, op_ptr: int, op_bytes: int, ws_ptr: int, ws_bytes: int):
        self._check(self.lib.s2w_bltt_bind_memory(self.handle, op_ptr, op_bytes, ws_ptr, ws_bytes),
                    "s2w_bltt_bind_memory")

    def set_blocks(self, f_ptr: int, row0: int, nrows: int, stream: int = 0):
        self._check(self.lib.s2w_bltt_set_blocks(self.handle, f_ptr, row0, nrows, stream), "s2w_bltt_set_blocks")

    def apply(self, x_ptr: int, B: int, y_ptr: int, stream: int = 0):
        self._check(self.lib.s2w_bltt_apply(self.handle, x_ptr, B, y_ptr, stream), "s2w_bltt_apply")

    def adjoint(self, y_ptr: int, B: int, x_ptr: int, stream: int = 0):
        self._check(self.lib.s2w_bltt_adjoint(self.handle, y_ptr, B, x_ptr, stream), "s2w_bltt_adjoint")
