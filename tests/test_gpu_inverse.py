"""GPU parity: the explicit inverse from the factors (the paper's product
form of the inverse, Eq. 4-c) against the oracle's inverse, element by
element, and at full size on sampled columns."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1907_05767_amd import ebv, inputs
from tests.gpu_util import case, dev, host

pytestmark = pytest.mark.gpu


def _rel(x, ref) -> float:
    return float(np.max(np.abs(np.asarray(x, np.float64) - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [1, 2, 3, 16, 17, 63, 64, 65, 130, 200, 257, 513])
def test_inverse_parity(n):
    case(f"inverse n={n}")
    A = inputs.dense(n, 0.5, 600 + n)
    X_ref, _ = oracle.inverse(A)
    t = dev(A)
    assert int(ebv.lu_factor_(t).item()) == 0
    X = ebv.lu_inverse(t)
    torch.cuda.synchronize()
    assert _rel(host(X), X_ref) <= 1e-12


def test_inverse_row_dominance_09_and_float():
    case("inverse s=0.9 fp64, and fp32")
    n = 300
    A = inputs.dense(n, 0.9, 611)
    X_ref, _ = oracle.inverse(A)
    t = dev(A)
    ebv.lu_factor_(t)
    assert _rel(host(ebv.lu_inverse(t)), X_ref) <= 1e-12
    t32 = dev(A, torch.float32)
    ebv.lu_factor_(t32)
    assert _rel(host(ebv.lu_inverse(t32)), X_ref) <= 1e-4


def test_inverse_padded_leading_dimensions():
    case("inverse lda > n, ldai > n")
    n, pa, px = 150, 7, 5
    A = inputs.dense(n, 0.5, 612)
    X_ref, _ = oracle.inverse(A)
    big = np.zeros((n, n + pa))
    big[:, :n] = A
    t = dev(big)
    h = ebv.handle()
    ws = ebv.workspace(ebv.OP_FACTOR, ebv.F64, n, 0, 1)
    w, wb = ebv._ws_args(ws)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert ebv.lib().ebv_lu_factor(h, ebv.F64, n, ctypes.c_void_p(t.data_ptr()), n + pa, 1, 0,
                                   ctypes.c_void_p(info.data_ptr()), w, wb, st) == 0
    out = torch.full((n, n + px), 7.0, dtype=torch.float64, device="cuda")
    wsi = ebv.workspace(ebv.OP_INVERSE, ebv.F64, n, 0, 1)
    wi, wib = ebv._ws_args(wsi)
    assert ebv.lib().ebv_lu_inverse(h, ebv.F64, n, ctypes.c_void_p(t.data_ptr()), n + pa,
                                    ctypes.c_void_p(out.data_ptr()), n + px, wi, wib, st) == 0
    torch.cuda.synchronize()
    o = host(out)
    assert int(info.item()) == 0
    assert _rel(o[:, :n], X_ref) <= 1e-12
    assert np.all(o[:, n:] == 7.0)  # padding untouched


def test_inverse_full_size_4096_sampled_columns():
    case("inverse n=4096 sampled columns")
    n = 4096
    A = inputs.dense(n, 0.5, 2)
    t = dev(A)
    assert int(ebv.lu_factor_(t).item()) == 0
    X = host(ebv.lu_inverse(t))
    LU_ref, info = oracle.lu_factor(A)
    assert info == 0
    cols = np.array([0, 1, 15, 16, 777, 2048, 3071, 4095])
    E = np.zeros((n, len(cols)))
    E[cols, np.arange(len(cols))] = 1.0
    Xc = oracle.lu_solve(LU_ref, E)
    assert _rel(X[:, cols], Xc) <= 1e-12
    # and every column through A X = I on sampled rows
    rows = np.array([0, 5, 1000, 4095])
    R = A[rows] @ X
    I = np.zeros_like(R)
    I[np.arange(len(rows)), rows] = 1.0
    assert np.max(np.abs(R - I)) <= 1e-12
