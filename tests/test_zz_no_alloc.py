"""GPU: the allocation-free factor + solve (static scratch inside the
library) against ebv_lu_factor_solve with a caller workspace, through the
C ABI, on consecutive calls of decreasing size (each call must see nothing
the previous one left in the shared array)."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1907_05767_amd import ebv, inputs
from tests.gpu_util import case, dev, fwd_err, host

pytestmark = pytest.mark.gpu


def _noalloc(A: torch.Tensor, B: torch.Tensor, info: torch.Tensor) -> int:
    n, nrhs = A.shape[0], B.shape[1]
    return ebv.lib().ebv_lu_factor_solve_noalloc(
        ebv.handle(), ebv.F64 if A.dtype == torch.float64 else ebv.F32, n, nrhs, ctypes.c_void_p(A.data_ptr()),
        A.stride(0), ctypes.c_void_p(B.data_ptr()), B.stride(0), ctypes.c_void_p(info.data_ptr()),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def _with_workspace(A: torch.Tensor, B: torch.Tensor, info: torch.Tensor) -> int:
    n, nrhs = A.shape[0], B.shape[1]
    dt = ebv.F64 if A.dtype == torch.float64 else ebv.F32
    ws = ebv.workspace(ebv.OP_FACTOR_SOLVE, dt, n, nrhs, 1)
    w, wb = ebv._ws_args(ws)  # 256-byte aligned start and its usable size
    rc = ebv.lib().ebv_lu_factor_solve(
        ebv.handle(), dt, n, nrhs, ctypes.c_void_p(A.data_ptr()), A.stride(0), ctypes.c_void_p(B.data_ptr()),
        B.stride(0), ctypes.c_void_p(info.data_ptr()), w, wb, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return rc


def _compare(n: int, nrhs: int, seed: int, with_oracle: bool):
    A = inputs.dense(n, 0.5, seed)
    B = inputs.rhs(n, nrhs, seed)
    a1, b1 = dev(A), dev(B)
    a2, b2 = dev(A), dev(B)
    i1 = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    i2 = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    case(f"no-alloc factor+solve n={n} nrhs={nrhs} seed={seed}")
    assert _noalloc(a1, b1, i1) == 0
    torch.cuda.synchronize()
    case(f"workspace factor+solve n={n} nrhs={nrhs} seed={seed}")
    assert _with_workspace(a2, b2, i2) == 0
    assert int(i1.item()) == 0 and int(i2.item()) == 0
    # same launches and tuning: the results agree to the parity bar (and are
    # expected to be bitwise equal)
    assert fwd_err(host(b1), host(b2)) <= 1e-12
    assert np.max(np.abs(host(a1) - host(a2))) <= 1e-12
    if with_oracle:
        X_ref, LU_ref, info_ref = oracle.solve(A, B)
        assert info_ref == 0
        assert fwd_err(host(b1), X_ref) <= 1e-12
        assert np.max(np.abs(host(a1) - LU_ref)) <= 1e-12


def test_noalloc_matches_workspace_entry_point_twice():
    # two calls in a row on the shared array, the second smaller
    _compare(1000, 5, 71, with_oracle=True)
    _compare(300, 2, 72, with_oracle=True)


def test_noalloc_largest_size_then_small():
    n = int(ebv.lib().ebv_noalloc_max_n())
    _compare(n, 4, 73, with_oracle=False)
    _compare(129, 3, 74, with_oracle=True)


def test_noalloc_rejects_oversize_before_any_work():
    n = int(ebv.lib().ebv_noalloc_max_n()) + 1
    a = torch.zeros(1, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc = ebv.lib().ebv_lu_factor_solve_noalloc(ebv.handle(), ebv.F64, n, 1, ctypes.c_void_p(a.data_ptr()), n,
                                               ctypes.c_void_p(a.data_ptr()), 1, ctypes.c_void_p(info.data_ptr()),
                                               None)
    assert rc == 8  # EBV_ERR_TOO_LARGE
