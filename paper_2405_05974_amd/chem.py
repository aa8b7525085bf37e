"""Python binding of libchem (ctypes; argument marshalling only).

Every step of the integration runs in the HIP kernels of libchem.so; this
module only turns torch CUDA tensors into device pointers and the current
stream into a hipStream_t.  Importing it does not load the library; the first
Mechanism() does, and raises if the built library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchem.so")

CHEM_OK = 0
CHEM_WARN_CELLS_FAILED = 1
CHEM_ERR_ARG = -1
CHEM_ERR_PARSE = -2
CHEM_ERR_DEVICE = -3
CHEM_ERR_OOM = -4
CHEM_ERR_UNSUPPORTED = -5

OPT_MAX_STEPS = 1
OPT_Q_MAX = 2
OPT_FIXED_T = 3
OPT_FIXED_STEP = 4
OPT_LU_FP32 = 5
OPT_IR_MAX = 6

RECORD_ROWS = 9   # per-cell record rows of chem_integrate_ex

OPT_GRAPH = 7
OPT_WAVES_PER_CU = 8
OPT_GROUP_WIDTH = 9
OPT_KERNEL = 10          # 0 auto, 1 group kernels, 2 lane-per-cell kernels (generated, hipRTC)
KERNEL_AUTO, KERNEL_GROUP, KERNEL_LANE = 0, 1, 2
OPT_JAC = 11             # 0 analytic, 1 difference quotients, 2 difference-quotient T column
JAC_ANALYTIC, JAC_FD, JAC_FD_T = 0, 1, 2
OPT_RETRY = 13           # failed cells retried with dt split into 2, 4, ... 2^k substeps
OPT_JAC_REUSE = 12       # 1: keep the factored Newton matrix while recent; 0 (default): fresh every attempt
OPT_PROGRESS = 14        # s > 0: progress lines from chem_integrate_boxes every s seconds (per-box times on)

EXPORTED = ("chem_mech_load", "chem_mech_load_str", "chem_mech_free", "chem_mech_info", "chem_set_stream",
            "chem_set_option", "chem_integrate", "chem_integrate_ex", "chem_integrate_noalloc", "chem_integrate_boxes",
            "chem_autotune",
            "chem_rates",
            "chem_last_error", "chem_server_create", "chem_server_submit", "chem_server_poll", "chem_server_drain",
            "chem_server_stats_get", "chem_server_destroy")


NOALLOC_MAX_CELLS = 1048576   # CHEM_NOALLOC_MAX_CELLS in chem.h


class ChemStats(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_steps_total", C.c_int64), ("n_steps_max", C.c_int64),
                ("n_attempts", C.c_int64), ("n_rhs", C.c_int64), ("n_jac", C.c_int64), ("n_lu", C.c_int64),
                ("n_newton_iters", C.c_int64), ("n_err_test_fails", C.c_int64), ("n_newton_fails", C.c_int64),
                ("n_cells_failed", C.c_int64), ("n_ir_sweeps", C.c_int64), ("wall_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ChemBox(C.Structure):
    _fields_ = [("T", C.c_void_p), ("Y", C.c_void_p), ("n_cells", C.c_int64), ("dt", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("submitted", "completed", "cells_completed", "launches", "bytes_in_use",
                                         "bytes_peak", "budget_bytes", "queued", "in_flight")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ChemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libchem error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: Optional[str] = None):
    """Load libchem.so with typed signatures (raises if it is not built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libchem.so not built at {p}; build it with python -m paper_2405_05974_amd.build")
    # torch ships its own HIP runtime under the same soname as the system one;
    # loading torch first makes libchem bind to that copy, so the process has
    # one runtime and device pointers/streams from torch are valid here.
    import torch  # noqa: F401
    lib = C.CDLL(p)
    vp, dp, i64, i32p = C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p
    lib.chem_mech_load.argtypes = [C.c_char_p, C.POINTER(C.c_void_p)]
    lib.chem_mech_load_str.argtypes = [C.c_char_p, C.POINTER(C.c_void_p)]
    lib.chem_mech_free.argtypes = [vp]
    lib.chem_mech_free.restype = None
    lib.chem_mech_info.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.chem_set_stream.argtypes = [vp, vp]
    lib.chem_set_option.argtypes = [vp, C.c_int, C.c_double]
    lib.chem_integrate.argtypes = [vp, i64, dp, dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                   C.POINTER(ChemStats)]
    lib.chem_integrate_ex.argtypes = [vp, i64, dp, dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                      C.POINTER(ChemStats), i32p]
    lib.chem_integrate_noalloc.argtypes = [vp, i64, dp, dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                           C.POINTER(ChemStats)]
    lib.chem_integrate_boxes.argtypes = [vp, C.c_int, C.POINTER(ChemBox), C.c_double, C.c_double, C.c_double,
                                         C.POINTER(ChemStats), C.POINTER(C.c_double)]
    lib.chem_autotune.argtypes = [vp, i64, dp, dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                  C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.chem_rates.argtypes = [vp, i64, dp, dp, C.c_double, dp, dp, dp]
    lib.chem_server_create.argtypes = [i64, C.c_int, C.POINTER(C.c_void_p)]
    lib.chem_server_submit.argtypes = [vp, vp, i64, dp, dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                       C.POINTER(C.c_int64)]
    lib.chem_server_poll.argtypes = [vp, i64, dp, dp, C.POINTER(C.c_double), C.POINTER(C.c_int)]
    lib.chem_server_drain.argtypes = [vp]
    lib.chem_server_stats_get.argtypes = [vp, C.POINTER(ServerStats)]
    lib.chem_server_destroy.argtypes = [vp]
    lib.chem_server_destroy.restype = None
    lib.chem_last_error.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("chem_mech_free", "chem_last_error", "chem_server_destroy"):
            getattr(lib, name).restype = C.c_int
    if path is None:
        _lib = lib
    return lib


def _check(lib, rc: int) -> int:
    if rc < 0:
        raise ChemError(rc, lib.chem_last_error().decode())
    return rc


def _ptr(t) -> int:
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return t.data_ptr()


def _ptr_i32(t) -> int:
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int32 or not t.is_contiguous():
        raise TypeError("expected a contiguous int32 CUDA tensor")
    return t.data_ptr()


def _stream_handle(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Mechanism:
    """A mechanism loaded into libchem (tables resident on the current device)."""

    def __init__(self, text: Optional[str] = None, path: Optional[str] = None):
        self.lib = load_library()
        h = C.c_void_p()
        if path is not None:
            rc = self.lib.chem_mech_load(path.encode(), C.byref(h))
        else:
            rc = self.lib.chem_mech_load_str(text.encode(), C.byref(h))
        _check(self.lib, rc)
        self.h = h
        S, R, E = C.c_int(), C.c_int(), C.c_int()
        _check(self.lib, self.lib.chem_mech_info(h, C.byref(S), C.byref(R), C.byref(E)))
        self.S, self.R, self.E = S.value, R.value, E.value
        self.N = self.S + 1

    def close(self):
        if getattr(self, "h", None):
            self.lib.chem_mech_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, key: int, value: float):
        _check(self.lib, self.lib.chem_set_option(self.h, int(key), float(value)))

    def set_options(self, max_steps=None, q_max=None, fixed_T=None, fixed_step_n=None, lu_fp32=None, ir_max=None,
                    graph=None, waves_per_cu=None, group_width=None, kernel=None, jac=None, jac_reuse=None, retry=None,
                    progress=None):
        for key, val in ((OPT_MAX_STEPS, max_steps), (OPT_Q_MAX, q_max), (OPT_FIXED_T, fixed_T),
                         (OPT_FIXED_STEP, fixed_step_n), (OPT_LU_FP32, lu_fp32), (OPT_IR_MAX, ir_max),
                         (OPT_GRAPH, graph), (OPT_WAVES_PER_CU, waves_per_cu), (OPT_GROUP_WIDTH, group_width),
                         (OPT_KERNEL, kernel), (OPT_JAC, jac), (OPT_JAC_REUSE, jac_reuse), (OPT_RETRY, retry),
                         (OPT_PROGRESS, progress)):
            if val is not None:
                self.set_option(key, float(val))

    def integrate(self, T, Y, p: float, dt: float, rtol: float, atol: float, records=None, stream=None) -> dict:
        """Advance every cell in place.  T: [n] and Y: [S, n] float64 CUDA
        tensors; records: optional int32 CUDA tensor [9, n] for per-cell
        records.  Returns the stats dict (plus 'rc')."""
        n = T.numel()
        if Y.numel() != self.S * n:
            raise ValueError("Y must hold S * n values")
        if records is not None and records.numel() != RECORD_ROWS * n:
            raise ValueError(f"records must hold {RECORD_ROWS} x n int32 values")
        _check(self.lib, self.lib.chem_set_stream(self.h, _stream_handle(stream)))
        st = ChemStats()
        rc = self.lib.chem_integrate_ex(self.h, n, _ptr(T), _ptr(Y), float(p), float(dt), float(rtol),
                                        float(atol), C.byref(st), _ptr_i32(records))
        _check(self.lib, rc)
        out = st.as_dict()
        out["rc"] = rc
        return out

    def integrate_noalloc(self, T, Y, p: float, dt: float, rtol: float, atol: float, stream=None) -> dict:
        """As integrate() without records, through the allocation-free entry
        point (fixed per-device scratch, at most NOALLOC_MAX_CELLS cells)."""
        n = T.numel()
        if Y.numel() != self.S * n:
            raise ValueError("Y must hold S * n values")
        _check(self.lib, self.lib.chem_set_stream(self.h, _stream_handle(stream)))
        st = ChemStats()
        rc = self.lib.chem_integrate_noalloc(self.h, n, _ptr(T), _ptr(Y), float(p), float(dt), float(rtol),
                                             float(atol), C.byref(st))
        _check(self.lib, rc)
        out = st.as_dict()
        out["rc"] = rc
        return out

    def autotune(self, T, Y, p: float, dt: float, rtol: float, atol: float, stream=None):
        """Time the candidate launch shapes on a sample (unchanged) and keep the
        fastest; returns (group_width, waves_per_cu)."""
        _check(self.lib, self.lib.chem_set_stream(self.h, _stream_handle(stream)))
        w, v = C.c_int(), C.c_int()
        _check(self.lib, self.lib.chem_autotune(self.h, T.numel(), _ptr(T), _ptr(Y), float(p), float(dt),
                                                float(rtol), float(atol), C.byref(w), C.byref(v)))
        return w.value, v.value

    def integrate_boxes(self, boxes, p: float, rtol: float, atol: float, box_ms: bool = False, stream=None):
        """boxes: list of (T, Y, dt) with T [n_b] and Y [S, n_b] float64 CUDA
        tensors, updated in place.  Returns (stats dict, per-box completion
        times in ms or None)."""
        arr = (ChemBox * max(len(boxes), 1))()
        for i, (T, Y, dt) in enumerate(boxes):
            n = T.numel()
            if Y.numel() != self.S * n:
                raise ValueError("Y must hold S * n values")
            arr[i] = ChemBox(_ptr(T) if n else None, _ptr(Y) if n else None, n, float(dt))
        ms = (C.c_double * max(len(boxes), 1))() if box_ms else None
        _check(self.lib, self.lib.chem_set_stream(self.h, _stream_handle(stream)))
        st = ChemStats()
        rc = self.lib.chem_integrate_boxes(self.h, len(boxes), arr, float(p), float(rtol), float(atol),
                                           C.byref(st), ms)
        _check(self.lib, rc)
        out = st.as_dict()
        out["rc"] = rc
        return out, (list(ms)[:len(boxes)] if box_ms else None)

    def rates(self, T, Y, p: float, wdot, f=None, jac=None, stream=None):
        """Production rates (mol/m^3/s), optionally the ODE rhs and Jacobian."""
        n = T.numel()
        _check(self.lib, self.lib.chem_set_stream(self.h, _stream_handle(stream)))
        _check(self.lib, self.lib.chem_rates(self.h, n, _ptr(T), _ptr(Y), float(p), _ptr(wdot), _ptr(f),
                                             _ptr(jac)))


class Server:
    """Continuous-batching request server (host arrays in, host arrays out)."""

    def __init__(self, budget_bytes: int, streams: int = 4):
        self.lib = load_library()
        h = C.c_void_p()
        _check(self.lib, self.lib.chem_server_create(int(budget_bytes), int(streams), C.byref(h)))
        self.h = h
        self._meta = {}

    def submit(self, mech: "Mechanism", T, Y, p: float, dt: float, rtol: float, atol: float) -> int:
        import numpy as np
        T = np.ascontiguousarray(T, dtype=np.float64)
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        n = T.size
        if Y.size != mech.S * n:
            raise ValueError("Y must hold S * n values")
        rid = C.c_int64()
        _check(self.lib, self.lib.chem_server_submit(self.h, mech.h, n, T.ctypes.data, Y.ctypes.data, float(p),
                                                     float(dt), float(rtol), float(atol), C.byref(rid)))
        self._meta[rid.value] = (mech.S, n)
        return rid.value

    def poll(self, rid: int):
        """None while pending, else (T, Y, latency_ms, status)."""
        import numpy as np
        S, n = self._meta[rid]
        T = np.full(n, np.nan)              # left as NaN when the request failed
        Y = np.full((S, n), np.nan)
        lat = C.c_double()
        status = C.c_int()
        rc = _check(self.lib, self.lib.chem_server_poll(self.h, rid, T.ctypes.data if n else None,
                                                        Y.ctypes.data if n else None, C.byref(lat),
                                                        C.byref(status)))
        if rc == 0:
            return None
        del self._meta[rid]
        return T, Y, lat.value, status.value

    def drain(self):
        _check(self.lib, self.lib.chem_server_drain(self.h))

    def stats(self) -> dict:
        st = ServerStats()
        _check(self.lib, self.lib.chem_server_stats_get(self.h, C.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "h", None):
            self.lib.chem_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
