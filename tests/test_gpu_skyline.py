"""GPU parity: skyline (profile) LU and solve -- the stand-in for the paper's
sparse systems (Table 1) -- against the skyline oracle, element by element
on the envelope, on variable-bandwidth profiles up to the full size."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_1907_05767_amd import ebv, inputs
from tests.gpu_util import case, fwd_err, host

pytestmark = pytest.mark.gpu


def _run(f, rp, AL, g, cp, AU, nrhs, seed):
    n = len(f)
    B = inputs.rhs(n, nrhs, seed)
    LL, UU, info_ref = oracle.lu_factor_skyline(f, rp, AL, g, cp, AU)
    assert info_ref == 0
    X_ref = oracle.lu_solve_skyline(f, rp, LL, g, cp, UU, B)
    sk = ebv.Skyline(f, rp, AL, g, cp, AU)
    info = sk.factor_()
    tB = torch.from_numpy(B).cuda()
    sk.solve_(tB)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    scale = max(np.abs(LL).max(initial=0.0), np.abs(UU).max(initial=0.0), 1.0)
    assert np.max(np.abs(host(sk.AL) - LL), initial=0.0) <= 1e-12 * scale
    assert np.max(np.abs(host(sk.AU) - UU), initial=0.0) <= 1e-12 * scale
    assert fwd_err(host(tB), X_ref) <= 1e-12


@pytest.mark.parametrize("n,ws,wl,pl,nrhs", [(1, 1, 1, 0.0, 1), (2, 1, 2, 0.5, 2), (65, 3, 40, 0.2, 1),
                                             (300, 8, 100, 0.1, 3), (1000, 64, 500, 0.1, 8),
                                             (777, 130, 700, 0.3, 5)])
def test_skyline_parity(n, ws, wl, pl, nrhs):
    case(f"skyline n={n} ws={ws} wl={wl} pl={pl}")
    _run(*inputs.skyline(n, ws, wl, pl, 0.5, 900 + n), nrhs, 900 + n)


def test_skyline_extreme_profiles():
    case("skyline tridiagonal and full profiles")
    for n, full in ((200, False), (130, True)):
        idx = np.arange(n)
        f = np.zeros(n, np.int32) if full else np.maximum(0, idx - 1).astype(np.int32)
        g = f.copy()
        rp = np.zeros(n + 1, np.int64)
        cp = np.zeros(n + 1, np.int64)
        rp[1:] = np.cumsum(idx - f)
        cp[1:] = np.cumsum(idx - g + 1)
        A = inputs.dense(n, 0.5, 950 + n)
        AL = np.concatenate([A[i, f[i]:i] for i in range(n)])
        AU = np.concatenate([A[g[j]:j + 1, j] for j in range(n)])
        _run(f, rp, AL, g, cp, AU, 2, 950 + n)


def test_skyline_full_size_16384():
    case("skyline n=16384 full size")
    _run(*inputs.skyline(16384, 64, 1024, 0.1, 0.5, 7), 8, 7)


def test_skyline_repeated_solves_two_blocks():
    """Several solves on one factorization give the same result: every
    workspace region the solve writes (the diagonal tiles' inverse packs)
    lies inside the workspace the library asks for."""
    case("skyline n=65 two blocks, repeated solves")
    f, rp, AL, g, cp, AU = inputs.skyline(65, 3, 40, 0.2, 0.5, 965)
    B = inputs.rhs(65, 1, 965)
    LL, UU, _ = oracle.lu_factor_skyline(f, rp, AL, g, cp, AU)
    X_ref = oracle.lu_solve_skyline(f, rp, LL, g, cp, UU, B)
    sk = ebv.Skyline(f, rp, AL, g, cp, AU)
    sk.factor_()
    for _ in range(4):
        tB = torch.from_numpy(B).cuda()
        sk.solve_(tB)
        torch.cuda.synchronize()
        assert fwd_err(host(tB), X_ref) <= 1e-12
