"""CPU oracle (test infrastructure only).

Plain scalar FP64 reference for per-cell stiff chemistry integration, written
in C (``oracle.c``) and loaded here through ctypes.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import this package;
the GPU library never touches it.  See ``oracle.c`` for what it computes and
which passages of the paper each part follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BUILD_CMD = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
             "-fno-fast-math", "-Wall", "-Wno-unused-result", _SRC, "-o", _LIB, "-lm"]


def build(extra_flags=(), out: Optional[str] = None) -> str:
    """Compile oracle.c into liboracle.so, or into `out` (always recompiles)."""
    cmd = BUILD_CMD[:1] + list(extra_flags) + BUILD_CMD[1:]
    if out is not None:
        cmd[cmd.index(_LIB)] = out
    subprocess.run(cmd, check=True)
    return out or _LIB


def build_native(out_dir: str) -> str:
    """The same oracle built for the host it runs on (-march=native) into
    out_dir, for timing: rounding is unchanged (no contraction, no fast-math)."""
    return build(["-march=native"], out=os.path.join(out_dir, "liboracle_native.so"))


class OrcOpts(C.Structure):
    _fields_ = [("max_steps", C.c_int), ("q_max", C.c_int), ("fixed_T", C.c_int),
                ("fixed_step_n", C.c_int), ("jac_mode", C.c_int), ("jac_reuse", C.c_int)]


class OrcCellStats(C.Structure):
    _fields_ = [("status", C.c_int), ("steps", C.c_int), ("attempts", C.c_int), ("n_rhs", C.c_int),
                ("n_jac", C.c_int), ("n_newton", C.c_int), ("n_etf", C.c_int), ("n_nnf", C.c_int),
                ("n_clip", C.c_int), ("clip_mass", C.c_double)]


_lib = None


def _load(path: Optional[str] = None):
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or _LIB
    if not os.path.exists(p):
        build()
    lib = C.CDLL(p)
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int)
    lib.orc_load.restype = C.c_void_p
    lib.orc_load.argtypes = [C.c_char_p, C.c_char_p, C.c_int]
    lib.orc_free.argtypes = [C.c_void_p]
    lib.orc_info.argtypes = [C.c_void_p, ip, ip, ip]
    lib.orc_weights.argtypes = [C.c_void_p, dp]
    lib.orc_nu.argtypes = [C.c_void_p, ip]
    lib.orc_thermo.argtypes = [C.c_void_p, C.c_double, dp, dp, dp, dp]
    lib.orc_rates.argtypes = [C.c_void_p, C.c_double, dp, C.c_double, dp, dp, dp, dp]
    lib.orc_rhs.argtypes = [C.c_void_p, dp, C.c_double, C.c_int, dp]
    lib.orc_jac.argtypes = [C.c_void_p, dp, C.c_double, C.c_int, dp]
    lib.orc_jac_fd.argtypes = [C.c_void_p, dp, C.c_double, C.c_int, dp, C.c_double, dp]
    lib.orc_jac_fd.restype = C.c_int
    lib.orc_lu.argtypes = [C.c_int, dp, ip]
    lib.orc_lu.restype = C.c_int
    lib.orc_lu_solve.argtypes = [C.c_int, dp, ip, dp]
    lib.orc_enthalpy.restype = C.c_double
    lib.orc_enthalpy.argtypes = [C.c_void_p, C.c_double, dp]
    lib.orc_temperature_from_h.restype = C.c_double
    lib.orc_temperature_from_h.argtypes = [C.c_void_p, C.c_double, dp]
    lib.orc_integrate.restype = C.c_int64
    lib.orc_integrate.argtypes = [C.c_void_p, C.c_int64, dp, dp, C.c_double, C.c_double, C.c_double,
                                  C.c_double, C.POINTER(OrcOpts), C.POINTER(OrcCellStats), C.c_int]
    lib.orc_qss_info.restype = C.c_int
    lib.orc_qss_info.argtypes = [C.c_void_p, ip, ip]
    lib.orc_qss_rates.restype = C.c_int
    lib.orc_qss_rates.argtypes = [C.c_void_p, C.c_double, dp, C.c_double, dp, dp]
    lib.orc_max_threads.restype = C.c_int
    if path is None:
        _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int))


class Mech:
    """An oracle-side mechanism parsed from the text format."""

    def __init__(self, text: str, lib_path: Optional[str] = None):
        self.lib = _load(lib_path)
        err = C.create_string_buffer(256)
        h = self.lib.orc_load(text.encode(), err, 256)
        if not h:
            raise ValueError("oracle could not parse mechanism: " + err.value.decode())
        self.h = h
        S, R, E = C.c_int(), C.c_int(), C.c_int()
        self.lib.orc_info(h, C.byref(S), C.byref(R), C.byref(E))
        self.S, self.R, self.E = S.value, R.value, E.value
        # quasi-steady-state species: the state holds the ST transported ones
        nq = C.c_int()
        qsp = np.zeros(max(self.S, 1), dtype=np.int32)
        self.ST = int(self.lib.orc_qss_info(h, C.byref(nq), _ip(qsp)))
        self.qss = [int(k) for k in qsp[:nq.value]]
        self.N = self.ST + 1

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.orc_free(self.h)
                self.h = None
        except Exception:
            pass

    # -- per-cell building blocks ------------------------------------------
    def weights(self) -> np.ndarray:
        W = np.zeros(self.S)
        self.lib.orc_weights(self.h, _dp(W))
        return W

    def nu(self) -> np.ndarray:
        nu = np.zeros(self.S * self.R, dtype=np.int32)
        self.lib.orc_nu(self.h, _ip(nu))
        return nu.reshape(self.S, self.R)

    def thermo(self, T: float):
        H, Sm, Cp, G = (np.zeros(self.S) for _ in range(4))
        self.lib.orc_thermo(self.h, float(T), _dp(H), _dp(Sm), _dp(Cp), _dp(G))
        return H, Sm, Cp, G

    def rates(self, T: float, Y: np.ndarray, p: float):
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        kf, kr, Q = np.zeros(self.R), np.zeros(self.R), np.zeros(self.R)
        wdot = np.zeros(self.S)
        self.lib.orc_rates(self.h, float(T), _dp(Y), float(p), _dp(kf), _dp(kr), _dp(Q), _dp(wdot))
        return kf, kr, Q, wdot

    def qss_rates(self, T: float, Y: np.ndarray, p: float):
        """QSS concentrations (mol/cm^3) and transported production rates
        (mol/cm^3/s) at a state of the transported species."""
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        Cq, wd = np.zeros(max(len(self.qss), 1)), np.zeros(self.ST)
        bad = self.lib.orc_qss_rates(self.h, float(T), _dp(Y), float(p), _dp(Cq), _dp(wd))
        return Cq[:len(self.qss)], wd, bool(bad)

    def rhs(self, y: np.ndarray, p: float, fixed_T: bool = False) -> np.ndarray:
        y = np.ascontiguousarray(y, dtype=np.float64)
        f = np.zeros(self.N)
        self.lib.orc_rhs(self.h, _dp(y), float(p), int(fixed_T), _dp(f))
        return f

    def jac(self, y: np.ndarray, p: float, fixed_T: bool = False) -> np.ndarray:
        y = np.ascontiguousarray(y, dtype=np.float64)
        J = np.zeros(self.N * self.N)
        self.lib.orc_jac(self.h, _dp(y), float(p), int(fixed_T), _dp(J))
        return J.reshape(self.N, self.N)

    def jac_fd(self, y: np.ndarray, p: float, w: np.ndarray, h: float, fixed_T: bool = False) -> np.ndarray:
        """The one-sided difference-quotient Jacobian (increment rule of the
        integrator's finite-difference mode) at y, with error weights w and step h."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        J = np.zeros(self.N * self.N)
        self.lib.orc_jac_fd(self.h, _dp(y), float(p), int(fixed_T), _dp(w), float(h), _dp(J))
        return J.reshape(self.N, self.N)

    def enthalpy(self, T: float, Y: np.ndarray) -> float:
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        return self.lib.orc_enthalpy(self.h, float(T), _dp(Y))

    def temperature_from_h(self, h: float, Y: np.ndarray) -> float:
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        return self.lib.orc_temperature_from_h(self.h, float(h), _dp(Y))

    # -- whole-batch integration ---------------------------------------------
    def integrate(self, T: np.ndarray, Y: np.ndarray, p: float, dt: float, rtol: float, atol: float,
                  max_steps: int = 100000, q_max: int = 5, fixed_T: bool = False, fixed_step_n: int = 0,
                  nthreads: int = 0, want_stats: bool = True, jac_mode: int = 0, jac_reuse: bool = False):
        """Returns (T_out, Y_out, stats) where stats is a structured numpy array
        (one record per cell) or None.  Inputs are not modified."""
        T = np.array(T, dtype=np.float64, copy=True).ravel()
        n = T.shape[0]
        Y = np.array(Y, dtype=np.float64, copy=True).reshape(self.ST, n)
        Y = np.ascontiguousarray(Y)
        o = OrcOpts(int(max_steps), int(q_max), int(fixed_T), int(fixed_step_n), int(jac_mode), int(jac_reuse))
        st = (OrcCellStats * n)() if want_stats else None
        self.lib.orc_integrate(self.h, n, _dp(T), _dp(Y), float(p), float(dt), float(rtol), float(atol),
                               C.byref(o), st, int(nthreads))
        stats = None
        if want_stats:
            dt_ = np.dtype([(name, np.float64 if ty is C.c_double else np.int32)
                            for name, ty in OrcCellStats._fields_], align=True)
            assert dt_.itemsize == C.sizeof(OrcCellStats)
            stats = np.frombuffer(st, dtype=dt_).copy()
        return T, Y, stats


def lu(A: np.ndarray):
    lib = _load()
    a = np.ascontiguousarray(A, dtype=np.float64).copy()
    n = a.shape[0]
    piv = np.zeros(n, dtype=np.int32)
    info = lib.orc_lu(n, _dp(a), _ip(piv))
    return a, piv, info


def lu_solve(a: np.ndarray, piv: np.ndarray, b: np.ndarray) -> np.ndarray:
    lib = _load()
    x = np.ascontiguousarray(b, dtype=np.float64).copy()
    lib.orc_lu_solve(a.shape[0], _dp(np.ascontiguousarray(a)), _ip(np.ascontiguousarray(piv, dtype=np.int32)), _dp(x))
    return x


def max_threads() -> int:
    return int(_load().orc_max_threads())
