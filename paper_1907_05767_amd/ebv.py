"""Python binding of libebv.so (argument marshalling only).

Every function hands device pointers of torch tensors, the sizes, and the
current HIP stream to the C ABI declared in ``include/ebv.h``; all arithmetic
runs in the library's HIP kernels.  PyTorch provides device memory and the
stream.  The library must be built (``paper_1907_05767_amd/build.py``); a
missing library raises immediately, there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libebv.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "ebv.h")

F64, F32 = 0, 1
OP_FACTOR, OP_SOLVE, OP_BATCHED, OP_ADJOINT, OP_MIXED, OP_BAND, OP_BATCHED_MIXED, OP_FACTOR_SOLVE = range(8)

_lib = None


class EbvError(RuntimeError):
    """A libebv entry point returned a nonzero status."""


def _declare(lib):
    i64, i32, vp, sz, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_double
    ci = ctypes.c_int
    sig = {
        "ebv_version": ([], ci),
        "ebv_status_string": ([ci], ctypes.c_char_p),
        "ebv_init": ([], ci),
        "ebv_workspace_status_offset": ([], sz),
        "ebv_workspace_size": ([ci, ci, i64, i64, i64], sz),
        "ebv_set_dense_tuning": ([ci, ci, ci, ci], ci),
        "ebv_profile_update_enable": ([ci], ci),
        "ebv_profile_update_read": ([ctypes.POINTER(dbl), ctypes.POINTER(i64), ctypes.POINTER(dbl)], ci),
        "ebv_lu_factor": ([ci, i64, vp, i64, i64, i64, vp, vp, sz, vp], ci),
        "ebv_lu_solve": ([ci, i64, i64, vp, i64, vp, i64, i64, i64, i64, vp, sz, vp], ci),
        "ebv_lu_factor_solve": ([ci, i64, i64, vp, i64, vp, i64, vp, vp, sz, vp], ci),
        "ebv_lu_factor_band": ([i64, i64, i64, vp, i64, vp, vp], ci),
        "ebv_lu_solve_band": ([i64, i64, i64, i64, vp, i64, vp, i64, vp], ci),
        "ebv_lu_factor_batched": ([ci, i64, vp, vp, vp, i64, vp, vp, i64, vp, vp, ci, i32, dbl, vp, i32, vp, sz, vp], ci),
        "ebv_batched_order": ([i64, vp, vp], ci),
        "ebv_lu_solve_adjoint": ([ci, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, i64, i64, i64, i64, i64, vp, sz, vp], ci),
        "ebv_lu_solve_mixed": ([i64, i64, vp, i64, vp, i64, vp, i64, i32, dbl, vp, vp, vp, vp, sz, vp], ci),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


def lib():
    """The loaded libebv.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise EbvError(f"{LIB_PATH} is missing: build it with paper_1907_05767_amd/build.py")
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def header_symbols():
    """Names of the functions declared in include/ebv.h."""
    text = open(HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ebv_\w+)\s*\(", text)))


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().ebv_status_string(rc).decode()
        raise EbvError(f"{what} failed: status {rc} ({msg})")


def _dt(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need_gpu(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("tensors must be contiguous and on the GPU")


def workspace(op: int, dtype: int, n: int, nrhs: int = 0, batch: int = 1, device=None) -> Optional[torch.Tensor]:
    """Device workspace for an operation (None when it needs none)."""
    nbytes = lib().ebv_workspace_size(op, dtype, n, nrhs, batch)
    if nbytes == 0:
        return None
    return torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")


def _ws_args(ws: Optional[torch.Tensor]):
    if ws is None:
        return None, 0
    base = ws.data_ptr()
    pad = (-base) % 256
    return ctypes.c_void_p(base + pad), ws.numel() - pad


def workspace_status(ws: Optional[torch.Tensor]) -> int:
    """Device-side error word of a workspace (synchronizes)."""
    if ws is None:
        return 0
    base = ws.data_ptr()
    pad = (-base) % 256
    return int(ws[pad:pad + 4].view(torch.int32).item())


def set_dense_tuning(small_update_below: int = 0, lookahead: bool = True, defer_group: int = 3,
                     defer_above: int = 1024):
    """Process-wide tuning of the single-system factor (see ebv_set_dense_tuning)."""
    _check(lib().ebv_set_dense_tuning(int(small_update_below), int(bool(lookahead)), int(defer_group),
                                      int(defer_above)), "ebv_set_dense_tuning")


def profile_update_enable(max_launches: int):
    """Bracket the next single-system update launches with HIP events (0 = off)."""
    _check(lib().ebv_profile_update_enable(int(max_launches)), "ebv_profile_update_enable")


def profile_update_read():
    """(summed ms, launches, summed algorithmic flops) of the bracketed update launches."""
    ms, n, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    _check(lib().ebv_profile_update_read(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl)),
           "ebv_profile_update_read")
    return ms.value, n.value, fl.value


# ----------------------------------------------------------------- dense ---
def lu_factor_(A: torch.Tensor, info: Optional[torch.Tensor] = None,
               ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """In-place Doolittle LU of A (n x n, or batch x n x n). Returns info (int32[batch])."""
    _need_gpu(A)
    batched = A.dim() == 3
    batch = A.shape[0] if batched else 1
    n = A.shape[-1]
    assert A.shape[-2] == n
    if info is None:
        info = torch.zeros(batch, dtype=torch.int32, device=A.device)
    if ws is None:
        ws = workspace(OP_FACTOR, _dt(A), n, 0, batch, A.device)
    w, wb = _ws_args(ws)
    rc = lib().ebv_lu_factor(_dt(A), n, _p(A), n, batch, n * n, _p(info), w, wb, _stream())
    _check(rc, "ebv_lu_factor")
    return info


def lu_factor(A: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
    LU = A.clone()
    info = lu_factor_(LU)
    return LU, info


def lu_solve_(LU: torch.Tensor, B: torch.Tensor, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """In-place solve: B (n x nrhs, or batch x n x nrhs) <- A^{-1} B from the packed factor."""
    _need_gpu(LU, B)
    batched = LU.dim() == 3
    batch = LU.shape[0] if batched else 1
    n = LU.shape[-1]
    nrhs = B.shape[-1]
    if ws is None:
        ws = workspace(OP_SOLVE, _dt(LU), n, nrhs, batch, LU.device)
    w, wb = _ws_args(ws)
    rc = lib().ebv_lu_solve(_dt(LU), n, nrhs, _p(LU), n, _p(B), nrhs, batch, n * n, n * nrhs, w, wb, _stream())
    _check(rc, "ebv_lu_solve")
    return B


def lu_solve(LU: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
    return lu_solve_(LU, B.clone())


def lu_factor_solve_(A: torch.Tensor, B: torch.Tensor, info: Optional[torch.Tensor] = None,
                     ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """In place: A (n x n) <- L\\U and B (n x nrhs) <- A^{-1} B, the forward
    substitution carried inside the factorization. Returns info (int32[1])."""
    _need_gpu(A, B)
    n, nrhs = A.shape[0], B.shape[-1]
    assert A.dim() == 2 and A.shape[1] == n and B.shape[0] == n
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    if ws is None:
        ws = workspace(OP_FACTOR_SOLVE, _dt(A), n, nrhs, 1, A.device)
    w, wb = _ws_args(ws)
    rc = lib().ebv_lu_factor_solve(_dt(A), n, nrhs, _p(A), n, _p(B), nrhs, _p(info), w, wb, _stream())
    _check(rc, "ebv_lu_factor_solve")
    return info


# ------------------------------------------------------------------ band ---
def lu_factor_band_(AB: torch.Tensor, kl: int, ku: int, info: Optional[torch.Tensor] = None) -> torch.Tensor:
    """In-place band LU of row-wise band storage AB[i, j - i + kl] (n x (kl+ku+1), float64)."""
    _need_gpu(AB)
    n, w = AB.shape
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=AB.device)
    _check(lib().ebv_lu_factor_band(n, kl, ku, _p(AB), w, _p(info), _stream()), "ebv_lu_factor_band")
    return info


def lu_solve_band_(LUB: torch.Tensor, kl: int, ku: int, B: torch.Tensor) -> torch.Tensor:
    _need_gpu(LUB, B)
    n, w = LUB.shape
    nrhs = B.shape[-1]
    _check(lib().ebv_lu_solve_band(n, kl, ku, nrhs, _p(LUB), w, _p(B), nrhs, _stream()), "ebv_lu_solve_band")
    return B


# --------------------------------------------------------------- batched ---
def batched_order(ns) -> np.ndarray:
    """EbV schedule (host): costliest system first, then the cheapest, ..."""
    ns = np.ascontiguousarray(ns, dtype=np.int32)
    order = np.empty_like(ns)
    _check(lib().ebv_batched_order(len(ns), ns.ctypes.data_as(ctypes.c_void_p),
                                   order.ctypes.data_as(ctypes.c_void_p)), "ebv_batched_order")
    return order


class RaggedBatch:
    """Device-side description of a packed ragged batch (sizes, offsets, order)."""

    def __init__(self, ns, offA, offB, device="cuda", ebv_order: bool = True):
        ns = np.ascontiguousarray(ns, dtype=np.int32)
        self.count = len(ns)
        self.ns_host = ns
        self.n = torch.from_numpy(ns).to(device)
        self.offA = torch.from_numpy(np.ascontiguousarray(offA, dtype=np.int64)).to(device)
        self.offB = torch.from_numpy(np.ascontiguousarray(offB, dtype=np.int64)).to(device)
        self.totA = int((np.asarray(offA, dtype=np.int64) + ns.astype(np.int64) ** 2).max()) if self.count else 0
        self.totB = int((np.asarray(offB, dtype=np.int64) + ns.astype(np.int64)).max()) if self.count else 0
        self.order = torch.from_numpy(batched_order(ns)).to(device) if ebv_order else None
        self.device = device


def factor_solve_batched_(rb: RaggedBatch, A: torch.Tensor, B: Optional[torch.Tensor], mixed: bool = False,
                          max_iter: int = 10, tol: float = 1e-12, info: Optional[torch.Tensor] = None,
                          iters: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
                          wg_per_cu: int = 0):
    """Factor + solve every system of a packed ragged batch in one persistent launch.
    Plain: A <- LU and B <- X in A's dtype.  mixed: float factor of each system
    in the workspace, A unchanged, B <- X refined in double."""
    _need_gpu(A, B)
    dt = _dt(A)
    if info is None:
        info = torch.zeros(rb.count, dtype=torch.int32, device=A.device)
    if mixed and iters is None:
        iters = torch.zeros(rb.count, dtype=torch.int32, device=A.device)
    if ws is None:
        ws = workspace(OP_BATCHED_MIXED if mixed else OP_BATCHED, dt, rb.totA, rb.totB, rb.count, A.device)
    w, wb = _ws_args(ws)
    rc = lib().ebv_lu_factor_batched(dt, rb.count, _p(rb.n), _p(rb.offA), _p(A), A.numel(), _p(rb.offB), _p(B),
                                     0 if B is None else B.numel(), _p(rb.order), _p(info), int(mixed),
                                     int(max_iter), float(tol), _p(iters), int(wg_per_cu), w, wb, _stream())
    _check(rc, "ebv_lu_factor_batched")
    return info, iters


# --------------------------------------------------------------- adjoint ---
def lu_solve_adjoint(LU: torch.Tensor, X: torch.Tensor, Xbar: torch.Tensor, want_abar: bool = True,
                     ws: Optional[torch.Tensor] = None):
    """Reverse-mode of X = A^{-1} B: returns (Bbar, Abar) = (A^{-T} Xbar, -Bbar X^T)."""
    _need_gpu(LU, X, Xbar)
    batched = LU.dim() == 3
    batch = LU.shape[0] if batched else 1
    n = LU.shape[-1]
    nrhs = Xbar.shape[-1]
    Bbar = Xbar.clone()
    Abar = torch.empty_like(LU) if want_abar else None
    if ws is None:
        ws = workspace(OP_ADJOINT, _dt(LU), n, nrhs, batch, LU.device)
    w, wb = _ws_args(ws)
    rc = lib().ebv_lu_solve_adjoint(_dt(LU), n, nrhs, _p(LU), n, _p(X), nrhs, _p(Bbar), nrhs, _p(Abar), n, batch,
                                    n * n, n * nrhs, n * nrhs, n * n, w, wb, _stream())
    _check(rc, "ebv_lu_solve_adjoint")
    return Bbar, Abar


class EbvSolve(torch.autograd.Function):
    """X = A^{-1} B with the EbV factor; backward reuses the factor (U^T and L^T
    solves, Abar = -Bbar X^T) through the library's adjoint entry point."""

    @staticmethod
    def forward(ctx, A, B):
        LU = A.detach().contiguous().clone()
        X = B.detach().contiguous().clone()
        if LU.dim() == 2:
            info = lu_factor_solve_(LU, X)
        else:
            info = lu_factor_(LU)
            lu_solve_(LU, X)
        ctx.save_for_backward(LU, X)
        ctx.info = info
        return X

    @staticmethod
    def backward(ctx, Xbar):
        LU, X = ctx.saved_tensors
        Bbar, Abar = lu_solve_adjoint(LU, X, Xbar.contiguous(), want_abar=ctx.needs_input_grad[0])
        return Abar, Bbar


def solve(A: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
    """Differentiable X = A^{-1} B (A: n x n or batch x n x n)."""
    return EbvSolve.apply(A, B)


# ------------------------------------------------------- mixed precision ---
def solve_mixed(A: torch.Tensor, B: torch.Tensor, tol: float = 1e-12, max_iter: int = 10,
                ws: Optional[torch.Tensor] = None):
    """Float factor + double refinement. Returns (X, iters, relres, info) as device tensors."""
    _need_gpu(A, B)
    n = A.shape[0]
    nrhs = B.shape[-1]
    X = torch.empty_like(B)
    iters = torch.empty(nrhs, dtype=torch.int32, device=A.device)
    relres = torch.empty(nrhs, dtype=torch.float64, device=A.device)
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    if ws is None:
        ws = workspace(OP_MIXED, F64, n, nrhs, 1, A.device)
    w, wb = _ws_args(ws)
    rc = lib().ebv_lu_solve_mixed(n, nrhs, _p(A), n, _p(B), nrhs, _p(X), nrhs, int(max_iter), float(tol),
                                  _p(iters), _p(relres), _p(info), w, wb, _stream())
    _check(rc, "ebv_lu_solve_mixed")
    return X, iters, relres, info
