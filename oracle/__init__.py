"""FP64 CPU oracle for the EbV LU path -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
this package.  The GPU product path never imports it, and it imports nothing
from the GPU path.  The arithmetic lives in ``ebv_oracle.c`` (plain C, double
precision, no FMA contraction); this file only marshals numpy arrays.

Every function follows the paper's definitions (Hashemi, Lahooti, Shirani,
arXiv:1907.05767): Eq. (1) forward/backward substitution, Eq. (3) the
triangular factors, Eq. (6-a)/(6-c) the elimination step.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)


def _declare(lib):
    vp = ctypes.c_void_p
    lib.oracle_lu_factor.argtypes = [_i64, vp, _i64]
    lib.oracle_lu_factor.restype = ctypes.c_int
    for name in ("oracle_forward", "oracle_backward", "oracle_lu_solve"):
        getattr(lib, name).argtypes = [_i64, _i64, vp, _i64, vp, _i64]
        getattr(lib, name).restype = None
    lib.oracle_lu_factor_band.argtypes = [_i64, _i64, _i64, vp, _i64]
    lib.oracle_lu_factor_band.restype = ctypes.c_int
    lib.oracle_lu_solve_band.argtypes = [_i64, _i64, _i64, _i64, vp, _i64, vp, _i64]
    lib.oracle_lu_solve_band.restype = None
    lib.oracle_lu_solve_adjoint.argtypes = [_i64, _i64, vp, _i64, vp, _i64, vp, _i64, vp, _i64]
    lib.oracle_lu_solve_adjoint.restype = None
    lib.oracle_lu_factor_solve_batched.argtypes = [_i64, vp, vp, vp, vp, vp, _i64, vp]
    lib.oracle_lu_factor_solve_batched.restype = None
    lib.oracle_refine_mixed.argtypes = [_i64, _i64, vp, _i64, vp, _i64, vp, _i64,
                                        ctypes.c_int, ctypes.c_double, vp, vp]
    lib.oracle_refine_mixed.restype = ctypes.c_int
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_lu_factor_skyline.argtypes = [_i64, vp, vp, vp, vp, vp, vp]
    lib.oracle_lu_factor_skyline.restype = ctypes.c_int
    lib.oracle_lu_solve_skyline.argtypes = [_i64, _i64, vp, vp, vp, vp, vp, vp, vp, _i64]
    lib.oracle_lu_solve_skyline.restype = None
    return lib


def _load():
    """The library this module's functions call (``use_library`` swaps it)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(os.path.join(_HERE, "ebv_oracle.c"))
    ):
        from . import build as _b
        _b.build()
    _lib = _declare(ctypes.CDLL(_LIB_PATH))
    return _lib


def use_library(path):
    """Point this module at another build of ``ebv_oracle.c`` (the test-suite
    uses it to show that the pins reject deliberately broken copies).
    ``None`` restores the default build.  Returns the previous library."""
    global _lib
    prev = _lib
    _lib = None if path is None else _declare(ctypes.CDLL(path))
    return prev


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c64(a) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    return np.ascontiguousarray(a).copy()


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def lu_factor(A):
    """Doolittle LU (Eq. 6-a/6-c) of a copy of A. Returns (LU, info)."""
    lu = _c64(A)
    n = lu.shape[0]
    assert lu.shape == (n, n)
    info = _load().oracle_lu_factor(n, _p(lu), n)
    return lu, int(info)


def split_lu(LU):
    """Unit-lower L and upper U from the packed in-place factor."""
    LU = np.asarray(LU)
    n = LU.shape[0]
    L = np.tril(LU, -1) + np.eye(n, dtype=LU.dtype)
    U = np.triu(LU)
    return L, U


def _as2d(B):
    b = _c64(B)
    vec = b.ndim == 1
    if vec:
        b = b[:, None].copy()
    return b, vec


def forward(LU, B):
    lu = np.ascontiguousarray(LU, dtype=np.float64)
    b, vec = _as2d(B)
    _load().oracle_forward(lu.shape[0], b.shape[1], _p(lu), lu.shape[0], _p(b), b.shape[1])
    return b[:, 0] if vec else b


def backward(LU, B):
    lu = np.ascontiguousarray(LU, dtype=np.float64)
    b, vec = _as2d(B)
    _load().oracle_backward(lu.shape[0], b.shape[1], _p(lu), lu.shape[0], _p(b), b.shape[1])
    return b[:, 0] if vec else b


def lu_solve(LU, B):
    """Eq. (1): LY = B forward, then UX = Y backward."""
    lu = np.ascontiguousarray(LU, dtype=np.float64)
    b, vec = _as2d(B)
    _load().oracle_lu_solve(lu.shape[0], b.shape[1], _p(lu), lu.shape[0], _p(b), b.shape[1])
    return b[:, 0] if vec else b


def solve(A, B):
    """Factor then solve. Returns (X, LU, info)."""
    lu, info = lu_factor(A)
    if info:
        raise ZeroDivisionError(f"zero pivot at step {info}")
    return lu_solve(lu, B), lu, info


def inverse(A):
    """Explicit inverse (Eq. 4-c: the product of the elementary upper factors
    and the elementary lower factors is A^{-1}), computed by its definition:
    the solution X of A X = I, column by column through the oracle's factor
    and its forward and backward substitutions (Eq. 1).  Returns (X, LU)."""
    a = _c64(A)
    n = a.shape[0]
    lu, info = lu_factor(a)
    if info:
        raise ZeroDivisionError(f"zero pivot at step {info}")
    return lu_solve(lu, np.eye(n)), lu


def _sky(f, rp, g, cp):
    return (np.ascontiguousarray(f, dtype=np.int32), np.ascontiguousarray(rp, dtype=np.int64),
            np.ascontiguousarray(g, dtype=np.int32), np.ascontiguousarray(cp, dtype=np.int64))


def lu_factor_skyline(f, rp, AL, g, cp, AU):
    """Doolittle LU in skyline (profile) storage: L by rows, U with the
    diagonal by columns (layout of inputs.skyline).  Returns (LL, UU, info)."""
    f, rp, g, cp = _sky(f, rp, g, cp)
    al, au = _c64(AL), _c64(AU)
    info = _load().oracle_lu_factor_skyline(len(f), _p(f), _p(rp), _p(al), _p(g), _p(cp), _p(au))
    return al, au, int(info)


def lu_solve_skyline(f, rp, LL, g, cp, UU, B):
    """Eq. (1) on skyline factors (forward by rows, backward by rows)."""
    f, rp, g, cp = _sky(f, rp, g, cp)
    ll = np.ascontiguousarray(LL, dtype=np.float64)
    uu = np.ascontiguousarray(UU, dtype=np.float64)
    b, vec = _as2d(B)
    _load().oracle_lu_solve_skyline(len(f), b.shape[1], _p(f), _p(rp), _p(ll), _p(g), _p(cp), _p(uu), _p(b),
                                    b.shape[1])
    return b[:, 0] if vec else b


def lu_factor_band(AB, kl: int, ku: int):
    """Band Doolittle LU in row-wise band storage AB[i, j - i + kl]. Returns (LUB, info)."""
    ab = _c64(AB)
    n, w = ab.shape
    assert w >= kl + ku + 1
    info = _load().oracle_lu_factor_band(n, kl, ku, _p(ab), w)
    return ab, int(info)


def lu_solve_band(LUB, kl: int, ku: int, B):
    ab = np.ascontiguousarray(LUB, dtype=np.float64)
    b, vec = _as2d(B)
    _load().oracle_lu_solve_band(ab.shape[0], kl, ku, b.shape[1], _p(ab), ab.shape[1], _p(b), b.shape[1])
    return b[:, 0] if vec else b


def lu_solve_adjoint(LU, X, Xbar, want_abar: bool = True):
    """Adjoint of X = A^{-1} B: returns (Bbar, Abar) with Bbar = A^{-T} Xbar, Abar = -Bbar X^T."""
    lu = np.ascontiguousarray(LU, dtype=np.float64)
    x, vec = _as2d(X)
    bb, _ = _as2d(Xbar)
    n = lu.shape[0]
    abar = np.empty((n, n), dtype=np.float64) if want_abar else None
    _load().oracle_lu_solve_adjoint(n, bb.shape[1], _p(lu), n, _p(x), x.shape[1], _p(bb), bb.shape[1],
                                    _p(abar) if abar is not None else None, n)
    return (bb[:, 0] if vec else bb), abar


def factor_solve_batched(ns, offA, A, offB, B, nrhs: int = 1):
    """Ragged batch: factor + solve each packed system. Returns (LU_packed, X_packed, info)."""
    ns = np.ascontiguousarray(ns, dtype=np.int32)
    offA = np.ascontiguousarray(offA, dtype=np.int64)
    offB = np.ascontiguousarray(offB, dtype=np.int64)
    a = _c64(A)
    b = _c64(B)
    info = np.zeros(len(ns), dtype=np.int32)
    _load().oracle_lu_factor_solve_batched(len(ns), _p(ns), _p(offA), _p(a), _p(offB), _p(b), nrhs, _p(info))
    return a, b, info


def refine_mixed(A, B, max_iter: int = 10, tol: float = 1e-12):
    """Mixed-precision reference: float factor/solves, double residual/update.
    Returns (X, iters, relres, status)."""
    a = np.ascontiguousarray(A, dtype=np.float64)
    b, vec = _as2d(B)
    n, nrhs = b.shape
    x = np.zeros((n, nrhs), dtype=np.float64)
    iters = np.zeros(nrhs, dtype=np.int32)
    relres = np.zeros(nrhs, dtype=np.float64)
    st = _load().oracle_refine_mixed(n, nrhs, _p(a), n, _p(b), nrhs, _p(x), nrhs, max_iter, tol,
                                     _p(iters), _p(relres))
    return (x[:, 0] if vec else x), iters, relres, int(st)
