"""Plain FP64 CPU oracle for SG-WLS filtering (Liu et al., ICCV 2017, arXiv 1705.01674).

TEST INFRASTRUCTURE ONLY: the correctness reference for the GPU library.  Only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the GPU library
(``paper_1705_01674_amd``) and that library never imports it.

The arithmetic lives in ``sgwls_oracle.c`` (plain C, double precision, OpenMP
over independent subsystems); this module is only ctypes marshalling.  Every
function follows a passage of the paper:

* ``centres``       -- strip centres k, k+tau, ... (Sec. 2.1 and the sliding step of Sec. 2.3)
* ``snake_pixel``   -- neighbourhood construction along the column direction (Sec. 2.1)
* ``weight``        -- guidance weights omega^exp / omega^frac (Eq. 2)
* ``strip_band``    -- the band of A_s = I + lambda L on the 1D vector (Eqs. 4-5)
* ``band_solve``    -- exact solve of A_s u = f (Eq. 5) by banded LDL^T
* ``col_pass`` / ``row_pass`` -- construct, solve, inverse-construct, average (Sec. 2.3)
* ``filter``        -- T alternating column/row iterations (Sec. 2.3)
* ``filter_backward`` -- the adjoint of ``filter`` (not in the paper; gradients of the above)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sgwls_oracle.c")
_LIB = os.path.join(_HERE, "_sgwls_oracle.so")


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into ``oracle/_sgwls_oracle.so``.

    Optimised for the x86-64-v3 level (AVX2, FMA) rather than the building
    host: the library is built on one host and run on another (the GPU
    machine), whose CPU may lack the builder's newer extensions.  Products
    are not contracted into fused multiply-adds, so the oracle's arithmetic
    is the source's, operation by operation."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp",
                               "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_double), ("r", ctypes.c_int), ("iters", ctypes.c_int),
                ("stride", ctypes.c_int), ("kind", ctypes.c_int),
                ("sigma_s", ctypes.c_double), ("sigma_r", ctypes.c_double),
                ("alpha_s", ctypes.c_double), ("alpha_r", ctypes.c_double),
                ("eps", ctypes.c_double)]


@dataclass(frozen=True)
class OracleParams:
    """Filter parameters (Eq. 1-2, Sec. 2.3).  kind: "exp" or "frac"."""
    lam: float = 1.0
    r: int = 1
    iters: int = 1
    stride: int = 1
    kind: str = "exp"
    sigma_s: float = 1.0
    sigma_r: float = 0.1
    alpha_s: float = 1.2
    alpha_r: float = 1.2
    eps: float = 1e-4

    def c(self) -> _Params:
        return _Params(float(self.lam), int(self.r), int(self.iters), int(self.stride),
                       {"exp": 0, "frac": 1}[self.kind], float(self.sigma_s),
                       float(self.sigma_r), float(self.alpha_s), float(self.alpha_r),
                       float(self.eps))


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Params)
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = None
        lib.orc_centres.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _I]
        lib.orc_snake_pixel.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _I, _I]
        lib.orc_weight.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        lib.orc_weight.restype = ctypes.c_double
        lib.orc_weight_dga.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        lib.orc_weight_dga.restype = ctypes.c_double
        lib.orc_strip_band.argtypes = [ctypes.c_int, ctypes.c_int, _D, P, ctypes.c_int, _D, _D, _D]
        lib.orc_band_solve.argtypes = [ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_int, _D]
        for name in ("orc_col_pass", "orc_row_pass"):
            getattr(lib, name).argtypes = [ctypes.c_int] * 3 + [_D, _D, _D, P, _D]
        lib.orc_filter.argtypes = [ctypes.c_int] * 3 + [_D, _D, _D, P, _D]
        for name in ("orc_col_pass_backward", "orc_row_pass_backward"):
            getattr(lib, name).argtypes = [ctypes.c_int] * 3 + [_D] * 6 + [P]
        lib.orc_filter_backward.argtypes = [ctypes.c_int] * 3 + [_D] * 6 + [P]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _chw(x):
    x = _f64(x)
    if x.ndim == 2:
        return x[None], True
    if x.ndim != 3:
        raise ValueError("expected (M, N) or (C, M, N)")
    return x, False


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads used by later oracle calls."""
    _load().orc_set_threads(int(n))


def centres(n: int, r: int, stride: int) -> np.ndarray:
    lib = _load()
    cnt = lib.orc_centres(n, r, stride, None)
    _check(0 if cnt > 0 else cnt, "centres")
    out = np.zeros(cnt, dtype=np.int32)
    lib.orc_centres(n, r, stride, out.ctypes.data_as(_I))
    return out


def snake_pixel(k: int, r: int, p: int):
    i, j = ctypes.c_int(), ctypes.c_int()
    _load().orc_snake_pixel(k, r, p, ctypes.byref(i), ctypes.byref(j))
    return i.value, j.value


def weight(params: OracleParams, d: int, ga: float, gb: float) -> float:
    return float(_load().orc_weight(ctypes.byref(params.c()), d, ga, gb))


def weight_dga(params: OracleParams, d: int, ga: float, gb: float) -> float:
    return float(_load().orc_weight_dga(ctypes.byref(params.c()), d, ga, gb))


def strip_band(g, params: OracleParams, k: int):
    """Band of A_s for the column-direction vector centred at column k:
    (diag[s], off[s, r], w[s, r]) with off[p, d-1] = A_s(p, p+d)."""
    g = _f64(g)
    M, N = g.shape
    s = (2 * params.r + 1) * M
    diag = np.zeros(s)
    off = np.zeros((s, params.r))
    w = np.zeros((s, params.r))
    _check(_load().orc_strip_band(M, N, _ptr(g), ctypes.byref(params.c()), k,
                                  _ptr(diag), _ptr(off), _ptr(w)), "strip_band")
    return diag, off, w


def band_solve(diag, off, rhs):
    diag, off = _f64(diag), _f64(off)
    rhs = _f64(rhs).copy()
    squeeze = rhs.ndim == 1
    if squeeze:
        rhs = rhs[:, None].copy()
    s, r = off.shape
    _check(_load().orc_band_solve(s, r, _ptr(diag), _ptr(off), rhs.shape[1], _ptr(rhs)),
           "band_solve")
    return rhs[:, 0] if squeeze else rhs


def _pass(name, X, g, params):
    X, sq = _chw(X)
    g = _f64(g)
    C, M, N = X.shape
    Y = np.zeros_like(X)
    cnt = np.zeros((M, N))
    _check(getattr(_load(), name)(C, M, N, _ptr(X), _ptr(g), _ptr(Y),
                                  ctypes.byref(params.c()), _ptr(cnt)), name)
    return (Y[0] if sq else Y), cnt


def col_pass(X, g, params: OracleParams):
    """One column-direction pass; returns (Y, cnt)."""
    return _pass("orc_col_pass", X, g, params)


def row_pass(X, g, params: OracleParams):
    """One row-direction pass; returns (Y, cnt)."""
    return _pass("orc_row_pass", X, g, params)


def filter(F, g, params: OracleParams, save: bool = False):
    """SG-WLS filter.  Returns U, or (U, saved) with the 2T pass inputs."""
    F, sq = _chw(F)
    g = _f64(g)
    C, M, N = F.shape
    U = np.zeros_like(F)
    saved = np.zeros((2 * params.iters, C, M, N)) if save else None
    _check(_load().orc_filter(C, M, N, _ptr(F), _ptr(g), _ptr(U), ctypes.byref(params.c()),
                              _ptr(saved)), "filter")
    U = U[0] if sq else U
    return (U, saved) if save else U


def pass_backward(direction, X, g, Yb, params: OracleParams):
    """Adjoint of one pass; returns (Xb, gb, lb)."""
    X, sq = _chw(X)
    Yb, _ = _chw(Yb)
    g = _f64(g)
    C, M, N = X.shape
    Xb = np.zeros_like(X)
    gb = np.zeros((M, N))
    lb = np.zeros(1)
    name = {"col": "orc_col_pass_backward", "row": "orc_row_pass_backward"}[direction]
    _check(getattr(_load(), name)(C, M, N, _ptr(X), _ptr(g), _ptr(Yb), _ptr(Xb), _ptr(gb),
                                  _ptr(lb), ctypes.byref(params.c())), name)
    return (Xb[0] if sq else Xb), gb, float(lb[0])


def filter_backward(g, saved, Ub, params: OracleParams):
    """Adjoint of ``filter``; returns (Fb, gb, lb)."""
    Ub, sq = _chw(Ub)
    g = _f64(g)
    saved = _f64(saved)
    C, M, N = Ub.shape
    Fb = np.zeros_like(Ub)
    gb = np.zeros((M, N))
    lb = np.zeros(1)
    _check(_load().orc_filter_backward(C, M, N, _ptr(g), _ptr(saved), _ptr(Ub), _ptr(Fb),
                                       _ptr(gb), _ptr(lb), ctypes.byref(params.c())),
           "filter_backward")
    return (Fb[0] if sq else Fb), gb, float(lb[0])


def sparse_interpolate(F, H, g, params: OracleParams):
    """Guided sparse interpolation of Eq. (21): U = S(F) / S(H), where S is the
    SG-WLS filter standing in for A^{-1}, F the sparse input (zero where
    unknown) and H the index map (1 where F is known, 0 elsewhere)."""
    num = filter(F, g, params)
    den = filter(H, g, params)
    return num / den
