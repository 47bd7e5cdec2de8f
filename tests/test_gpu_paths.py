"""GPU parity: band, ragged batched (plain FP64, FP32, mixed), adjoint and
mixed-precision paths against the FP64 oracle."""
from __future__ import annotations

import os

import numpy as np
import pytest
import torch

import oracle
from paper_1907_05767_amd import ebv, inputs
from tests.gpu_util import case, dev, fwd_err, host

pytestmark = pytest.mark.gpu


# ------------------------------------------------------------------- band ---
@pytest.mark.parametrize("n,kl,ku,nrhs", [(1, 0, 0, 1), (5, 1, 1, 2), (64, 64, 64, 1), (65, 3, 5, 3),
                                          (200, 64, 64, 8), (300, 64, 7, 2), (1000, 17, 64, 9), (777, 1, 1, 1)])
def test_band_parity(n, kl, ku, nrhs):
    case(f"band n={n} kl={kl} ku={ku} nrhs={nrhs}")
    AB = inputs.band(n, kl, ku, 0.5, 3 + n)
    B = inputs.rhs(n, nrhs, 4 + n)
    LUB_ref, info_ref = oracle.lu_factor_band(AB, kl, ku)
    X_ref = oracle.lu_solve_band(LUB_ref, kl, ku, B)
    t = dev(AB)
    info = ebv.lu_factor_band_(t, kl, ku)
    X = dev(B)
    ebv.lu_solve_band_(t, kl, ku, X)
    torch.cuda.synchronize()
    assert int(info.item()) == info_ref == 0
    # compare the in-band slots only (slots outside the matrix are unspecified)
    mask = inputs.band(n, kl, ku, 0.5, 3 + n) != 0
    mask[:, kl] = True
    assert np.max(np.abs(np.where(mask, host(t) - LUB_ref, 0.0))) <= 1e-12
    assert fwd_err(host(X), X_ref) <= 1e-12


def test_band_full_size_16384():
    n, kl, ku, nrhs = 16384, 64, 64, 8
    case("band n=16384 kl=ku=64 nrhs=8 full size")
    AB = inputs.band(n, kl, ku, 0.5, 3)
    B = inputs.rhs(n, nrhs, 3)
    LUB_ref, _ = oracle.lu_factor_band(AB, kl, ku)
    X_ref = oracle.lu_solve_band(LUB_ref, kl, ku, B)
    t = dev(AB)
    ebv.lu_factor_band_(t, kl, ku)
    X = dev(B)
    ebv.lu_solve_band_(t, kl, ku, X)
    torch.cuda.synchronize()
    mask = AB != 0
    assert np.max(np.abs(np.where(mask, host(t) - LUB_ref, 0.0))) <= 1e-12
    assert fwd_err(host(X), X_ref) <= 1e-12


# ---------------------------------------------------------------- batched ---
def _ragged(count, nmin, nmax, seed):
    ns, offA, A, offB, B = inputs.ragged(count, nmin, nmax, 0.5, seed)
    return ns, offA, A, offB, B


@pytest.mark.parametrize("ebv_order", [True, False])
def test_batched_fp64_parity(ebv_order):
    case(f"ragged batched fp64 ebv_order={ebv_order}")
    ns, offA, A, offB, B = _ragged(48, 1, 300, 11)
    LU_ref, X_ref, info_ref = oracle.factor_solve_batched(ns, offA, A, offB, B)
    rb = ebv.RaggedBatch(ns, offA, offB, ebv_order=ebv_order)
    tA, tB = dev(A), dev(B)
    info, _ = ebv.factor_solve_batched_(rb, tA, tB)
    torch.cuda.synchronize()
    assert np.array_equal(host(info), info_ref)
    LUh, Xh = host(tA), host(tB)
    for k in range(len(ns)):
        n = int(ns[k])
        a, b = slice(offA[k], offA[k] + n * n), slice(offB[k], offB[k] + n)
        assert np.max(np.abs(LUh[a] - LU_ref[a])) <= 1e-12, k
        assert fwd_err(Xh[b], X_ref[b]) <= 1e-12, k


def test_batched_matches_uniform_path_bitwise():
    """Same workgroup-level factor code: the ragged batch and the uniform
    batch give identical bits for the factors of the same system; the
    solutions (forward substitution fused into the ragged batch's factor,
    separate in the uniform solve) agree to rounding."""
    case("ragged vs uniform bitwise")
    n = 150
    A, B = inputs.uniform_batch(3, n, 0.5, 8)
    ns = np.full(3, n, dtype=np.int32)
    offA = np.arange(3, dtype=np.int64) * n * n
    offB = np.arange(3, dtype=np.int64) * n
    rb = ebv.RaggedBatch(ns, offA, offB)
    tA, tB = dev(A.reshape(-1)), dev(B.reshape(-1))
    ebv.factor_solve_batched_(rb, tA, tB)
    uA, uB = dev(A), dev(B)
    ebv.lu_factor_(uA)
    ebv.lu_solve_(uA, uB)
    torch.cuda.synchronize()
    assert torch.equal(tA, uA.reshape(-1))
    assert fwd_err(host(tB).reshape(3, n).T, host(uB).reshape(3, n).T) <= 1e-13


def test_batched_fp32_plain():
    case("ragged batched fp32 plain")
    ns, offA, A, offB, B = _ragged(24, 1, 200, 12)
    _, X_ref, _ = oracle.factor_solve_batched(ns, offA, A, offB, B)
    rb = ebv.RaggedBatch(ns, offA, offB)
    tA, tB = dev(A, torch.float32), dev(B, torch.float32)
    ebv.factor_solve_batched_(rb, tA, tB)
    torch.cuda.synchronize()
    Xh = host(tB).astype(np.float64)
    for k in range(len(ns)):
        b = slice(offB[k], offB[k] + int(ns[k]))
        assert fwd_err(Xh[b], X_ref[b]) <= 1e-4, k


def test_batched_mixed_parity():
    case("ragged batched mixed fp32+fp64 refinement small")
    ns, offA, A, offB, B = _ragged(40, 1, 260, 13)
    _, X_ref, _ = oracle.factor_solve_batched(ns, offA, A, offB, B)
    rb = ebv.RaggedBatch(ns, offA, offB)
    tA, tB = dev(A), dev(B)
    info, iters = ebv.factor_solve_batched_(rb, tA, tB, mixed=True, max_iter=10, tol=1e-12)
    torch.cuda.synchronize()
    assert np.array_equal(host(tA), A)  # A untouched
    it = host(iters)
    assert np.all(it >= 0) and np.all(it <= 10)
    assert np.all(host(info) == 0)
    Xh = host(tB)
    for k in range(len(ns)):
        b = slice(offB[k], offB[k] + int(ns[k]))
        assert fwd_err(Xh[b], X_ref[b]) <= 1e-12, k


def _full_ragged():
    ns, offA, A, offB, B = _ragged(4096, 16, 512, 4)
    _, X_ref, info_ref = oracle.factor_solve_batched(ns, offA, A, offB, B)
    assert np.all(info_ref == 0)
    return ns, offA, A, offB, B, X_ref


@pytest.fixture(scope="module")
def full_ragged():
    return _full_ragged()


def _per_system_err(ns, offB, X, X_ref):
    errs = np.empty(len(ns))
    for k in range(len(ns)):
        b = slice(offB[k], offB[k] + int(ns[k]))
        errs[k] = fwd_err(X[b], X_ref[b])
    return errs


def test_batched_full_size_every_system(full_ragged):
    """4096 systems with n ~ U{16..512}, plain FP64: every system's solution
    against the oracle's factor + solve."""
    ns, offA, A, offB, B, X_ref = full_ragged
    case("ragged batched full size 4096 x U{16..512} fp64, every system")
    rb = ebv.RaggedBatch(ns, offA, offB)
    tA, tB = dev(A), dev(B)
    info, _ = ebv.factor_solve_batched_(rb, tA, tB)
    torch.cuda.synchronize()
    assert np.all(host(info) == 0)
    errs = _per_system_err(ns, offB, host(tB), X_ref)
    print(f"plain fp64: max rel forward error over 4096 systems {errs.max():.3e}")
    assert errs.max() <= 1e-12, (int(errs.argmax()), errs.max())


def test_batched_mixed_full_size_every_system(full_ragged):
    """The same 4096 systems with the FP32 factor and FP64 refinement: every
    system's solution against the oracle's FP64 solution, each within
    1e-12 (the refinement stops on a forward-error bound)."""
    ns, offA, A, offB, B, X_ref = full_ragged
    case("ragged batched full size 4096 x U{16..512} mixed, every system")
    rb = ebv.RaggedBatch(ns, offA, offB)
    tA, tB = dev(A), dev(B)
    info, iters = ebv.factor_solve_batched_(rb, tA, tB, mixed=True, max_iter=10, tol=1e-12)
    torch.cuda.synchronize()
    assert np.all(host(info) == 0)
    it = host(iters)
    assert np.all(it >= 1) and np.all(it <= 10), (it.min(), it.max())
    errs = _per_system_err(ns, offB, host(tB), X_ref)
    print(f"mixed: max rel forward error over 4096 systems {errs.max():.3e}, corrections {it.min()}..{it.max()}")
    assert errs.max() <= 1e-12, (int(errs.argmax()), errs.max())


# ---------------------------------------------------------------- adjoint ---
@pytest.mark.parametrize("n,nrhs", [(1, 1), (70, 1), (300, 2), (513, 3)])
def test_adjoint_single_parity(n, nrhs):
    case(f"adjoint single n={n} nrhs={nrhs}")
    A = inputs.dense(n, 0.5, 600 + n)
    B = inputs.rhs(n, nrhs, 601 + n)
    W = inputs.rhs(n, nrhs, 602 + n)
    X_ref, LU_ref, _ = oracle.solve(A, B)
    bbar_ref, abar_ref = oracle.lu_solve_adjoint(LU_ref, X_ref, W)
    bbar, abar = ebv.lu_solve_adjoint(dev(LU_ref), dev(X_ref), dev(W))
    torch.cuda.synchronize()
    assert fwd_err(host(bbar), bbar_ref) <= 1e-12
    assert np.max(np.abs(host(abar) - abar_ref)) <= 1e-12 * max(1.0, np.abs(abar_ref).max())


def test_autograd_batched_vs_oracle():
    batch, n = 4, 130
    case(f"autograd batched {batch}x{n}")
    A, B = inputs.uniform_batch(batch, n, 0.5, 6)
    W = np.stack([inputs.rhs(n, 1, 900 + b) for b in range(batch)])
    tA = dev(A).requires_grad_(True)
    tB = dev(B).requires_grad_(True)
    X = ebv.solve(tA, tB)
    loss = (X * dev(W)).sum()
    loss.backward()
    torch.cuda.synchronize()
    gA, gB = host(tA.grad), host(tB.grad)
    for b in range(batch):
        X_ref, LU_ref, _ = oracle.solve(A[b], B[b])
        bbar_ref, abar_ref = oracle.lu_solve_adjoint(LU_ref, X_ref, W[b])
        assert np.linalg.norm(gB[b] - bbar_ref) <= 1e-12 * np.linalg.norm(bbar_ref)
        assert np.linalg.norm(gA[b] - abar_ref) <= 1e-12 * np.linalg.norm(abar_ref)


@pytest.mark.parametrize("n", [130, 1024])
def test_adjoint_central_differences(n):
    """Central differences (h = 1e-6) of the per-system loss L_s = w_s . x_s
    against the adjoint, on 4 systems: 64 sampled entries of A and 64 of b
    per system, normwise relative error <= 1e-8 with no absolute slack.

    L(A +- hE) - L(A) is evaluated without cancellation: the perturbed
    solution is x + d with A' d = b' - A' x (A', b' the perturbed system, the
    residual formed in float64 on the host, d from the GPU solve), so
    (L+ - L-) / 2h = w . (d+ - d-) / 2h carries the solve's relative error
    of about 1e-15 instead of that error times |L| / h.  All perturbed
    systems of a system are solved in one uniform batch."""
    batch, h, per = 4, 1e-6, 64
    case(f"adjoint vs central differences n={n}")
    A, B = inputs.uniform_batch(batch, n, 0.5, 60 + n)
    W = np.stack([inputs.rhs(n, 1, 950 + b) for b in range(batch)])
    tA = dev(A).requires_grad_(True)
    tB = dev(B).requires_grad_(True)
    X = ebv.solve(tA, tB)
    (X * dev(W)).sum().backward()
    torch.cuda.synchronize()
    gA, gB, Xh = host(tA.grad), host(tB.grad), host(X)
    rng = np.random.default_rng(n)
    worst = 0.0
    for s in range(batch):
        x, w = Xh[s], W[s]
        ij = rng.integers(0, n, size=(per, 2))
        bi = rng.choice(n, per, replace=False)
        # perturbed copies: 2 per sampled A entry (+h, -h), then 2 per b entry
        Ap = np.repeat(A[s][None], 4 * per, axis=0)
        Bp = np.repeat(B[s][None], 4 * per, axis=0)
        for k, (i, j) in enumerate(ij):
            Ap[2 * k, i, j] += h
            Ap[2 * k + 1, i, j] -= h
        for k, i in enumerate(bi):
            Bp[2 * per + 2 * k, i, 0] += h
            Bp[2 * per + 2 * k + 1, i, 0] -= h
        R = Bp - Ap @ x[None]                 # b' - A' x
        D = host(ebv.solve(dev(Ap), dev(R)))  # A' d = b' - A' x
        dL = (D * w[None]).sum(axis=(1, 2))   # L(A', b') - L(A, b)
        fd = (dL[0::2] - dL[1::2]) / (2 * h)
        fdA, fdB = fd[:per], fd[per:]
        anA = gA[s][ij[:, 0], ij[:, 1]]
        anB = gB[s][bi, 0]
        eA = np.linalg.norm(fdA - anA) / np.linalg.norm(anA)
        eB = np.linalg.norm(fdB - anB) / np.linalg.norm(anB)
        # for context: the rounding part of the plain quotient (L+ - L-) / 2h
        plain = np.finfo(np.float64).eps * abs(float((x * w).sum())) / h
        print(f"n={n} system {s}: FD rel err A {eA:.2e}, b {eB:.2e} "
              f"(a plain quotient would carry ~{plain:.1e} absolute per entry)")
        worst = max(worst, eA, eB)
    assert worst <= 1e-8, worst


def test_adjoint_full_size_sampled():
    """512 systems of n = 1024: forward factor + solve and the adjoint through
    autograd; sampled systems against the oracle adjoint."""
    batch, n = 512, 1024
    case("adjoint full size 512 x 1024")
    A, B = inputs.uniform_batch(batch, n, 0.5, 6)
    W = np.random.default_rng(6).standard_normal((batch, n, 1))
    tA = dev(A).requires_grad_(True)
    tB = dev(B).requires_grad_(True)
    X = ebv.solve(tA, tB)
    (X * dev(W)).sum().backward()
    torch.cuda.synchronize()
    for b in (0, 137, 511):
        X_ref, LU_ref, _ = oracle.solve(A[b], B[b])
        bbar_ref, abar_ref = oracle.lu_solve_adjoint(LU_ref, X_ref, W[b])
        assert fwd_err(host(X[b]), X_ref) <= 1e-12
        assert np.linalg.norm(host(tB.grad[b]) - bbar_ref) <= 1e-12 * np.linalg.norm(bbar_ref)
        assert np.linalg.norm(host(tA.grad[b]) - abar_ref) <= 1e-12 * np.linalg.norm(abar_ref)


@pytest.mark.parametrize("n", [4160, 4161])
def test_one_rhs_batched_solves_at_lds_limit(n):
    """One right-hand side per system: n = 4160 is the largest vector the
    batched solves hold in LDS, n = 4161 takes the block-staged path.  The
    plain solves (L then U) and the adjoint's transposed solves (U^T then
    L^T) of a batch of two, on the GPU's own factor, against the oracle's
    substitutions on that same factor."""
    batch = 2
    case(f"one-rhs batched solves n={n}")
    A, B = inputs.uniform_batch(batch, n, 0.5, 70 + n % 7)
    W = np.stack([inputs.rhs(n, 1, 80 + b) for b in range(batch)])
    LU = dev(A)
    info = ebv.lu_factor_(LU)
    X = dev(B)
    ebv.lu_solve_(LU, X)
    bbar, _ = ebv.lu_solve_adjoint(LU, X, dev(W), want_abar=False)
    torch.cuda.synchronize()
    assert np.all(host(info) == 0)
    LUh, Xh, Bh = host(LU), host(X), host(bbar)
    for b in range(batch):
        assert fwd_err(Xh[b], oracle.lu_solve(LUh[b], B[b])) <= 1e-12, b
        bbar_ref, _ = oracle.lu_solve_adjoint(LUh[b], Xh[b], W[b], want_abar=False)
        assert fwd_err(Bh[b], bbar_ref) <= 1e-12, b


# -------------------------------------------------------- mixed precision ---
@pytest.mark.parametrize("n,s,nrhs", [(1, 0.5, 1), (100, 0.9, 4), (1000, 0.9, 4), (700, 0.5, 9), (1500, 0.9, 3)])
def test_mixed_parity(n, s, nrhs):
    case(f"mixed n={n} s={s} nrhs={nrhs}")
    A = inputs.dense(n, s, 5 + n)
    B = inputs.rhs(n, nrhs, 6 + n)
    X_ref, _, _ = oracle.solve(A, B)
    X, iters, ferr, info = ebv.solve_mixed(dev(A), dev(B), tol=1e-12, max_iter=10)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    it, fe = host(iters), host(ferr)
    assert np.all(it >= 0) and np.all(it <= 10) and np.all(fe <= 1e-12)
    assert fwd_err(host(X), X_ref) <= 1e-12


def test_mixed_forced_class_path():
    """n = 1500 with the column-class split forced on every launch of the
    float factor (defer_above = 0): refinement to the oracle within 1e-12."""
    n, s, nrhs = 1500, 0.9, 4
    case(f"mixed n={n} s={s} nrhs={nrhs} class path forced")
    A = inputs.dense(n, s, 71)
    B = inputs.rhs(n, nrhs, 72)
    X_ref, _, _ = oracle.solve(A, B)
    ebv.set_dense_tuning(0, True, 3, 0)
    try:
        X, iters, ferr, info = ebv.solve_mixed(dev(A), dev(B), tol=1e-12, max_iter=10)
        torch.cuda.synchronize()
    finally:
        ebv.set_dense_tuning()
    assert int(info.item()) == 0 and np.all(host(ferr) <= 1e-12)
    assert fwd_err(host(X), X_ref) <= 1e-12


GOLDEN_MIXED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "mixed_n16384_s0.9_seed5_X.npy")


def test_mixed_full_size_16384():
    """n = 16384, row sum 0.9, 4 right-hand sides: the mixed-precision
    solution against the FP64 oracle's (stored by
    tests/golden/make_mixed_reference.py), every column within 1e-12; the
    residual recomputed on the host, and agreement with the plain FP64 solve."""
    n, nrhs = 16384, 4
    case("mixed full size n=16384")
    X_ref = np.load(GOLDEN_MIXED)
    A = inputs.dense(n, 0.9, 5)
    B = inputs.rhs(n, nrhs, 5)
    tA, tB = dev(A), dev(B)
    X, iters, ferr, info = ebv.solve_mixed(tA, tB, tol=1e-12, max_iter=10)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    Xh = host(X)
    err = fwd_err(Xh, X_ref)
    print(f"mixed n=16384: rel forward error vs oracle {err:.3e}, bound {host(ferr)}, iters {host(iters)}")
    assert err <= 1e-12
    assert np.all(host(ferr) <= 1e-12) and np.all(host(iters) >= 0)
    R = B - A @ Xh
    rel = np.abs(R).max(axis=0) / np.abs(B).max(axis=0)
    assert np.all(rel <= 1e-12), rel
    LU = tA.clone()
    ebv.lu_factor_(LU)
    X64 = ebv.lu_solve(LU, tB)
    torch.cuda.synchronize()
    assert fwd_err(host(X64), X_ref) <= 1e-12
