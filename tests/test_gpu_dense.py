"""GPU parity: dense factor and solves (single system and uniform batches)
against the FP64 oracle, element by element."""
from __future__ import annotations

import os

import numpy as np
import pytest
import torch

import oracle
from paper_1907_05767_amd import ebv, inputs
from tests.gpu_util import case, dev, fwd_err, host

pytestmark = pytest.mark.gpu

# sizes spanning one tile, several tiles and ragged tails
SIZES = [1, 2, 3, 17, 63, 64, 65, 127, 128, 129, 200, 256, 257, 300, 513]


@pytest.mark.parametrize("n", SIZES)
def test_factor_parity(n):
    case(f"dense factor n={n}")
    A = inputs.dense(n, 0.5, 1000 + n)
    LU_ref, info_ref = oracle.lu_factor(A)
    t = dev(A)
    info = ebv.lu_factor_(t)
    torch.cuda.synchronize()
    assert int(info.item()) == info_ref == 0
    err = np.max(np.abs(host(t) - LU_ref))
    assert err <= 1e-12, err


# (small_update_below, lookahead, defer_group, defer_above): 128-row update
# tiles everywhere, both launch schemes, column-class updates of every
# group size (forced at small n by defer_above = 0)
TUNINGS = [(0, True, 1, 2048), (0, True, 2, 0), (0, True, 3, 0), (0, True, 4, 0), (0, False, 1, 2048),
           (2048, True, 4, 0)]


@pytest.mark.parametrize("cfg", TUNINGS)
@pytest.mark.parametrize("n", [300, 700])
def test_factor_parity_tunings(n, cfg):
    case(f"dense factor n={n} tuning={cfg}")
    A = inputs.dense(n, 0.5, 7 + n)
    B = inputs.rhs(n, 5, 8 + n)
    X_ref, LU_ref, _ = oracle.solve(A, B)
    ebv.set_dense_tuning(*cfg)
    try:
        t = dev(A)
        ebv.lu_factor_(t)
        LU2, X2 = dev(A), dev(B)
        info = ebv.lu_factor_solve_(LU2, X2)
        torch.cuda.synchronize()
    finally:
        ebv.set_dense_tuning()
    assert np.max(np.abs(host(t) - LU_ref)) <= 1e-12
    assert int(info.item()) == 0
    assert np.max(np.abs(host(LU2) - LU_ref)) <= 1e-12
    assert fwd_err(host(X2), X_ref) <= 1e-12


@pytest.mark.parametrize("n,nrhs", [(1, 1), (64, 2), (65, 3), (129, 8), (300, 70)])
def test_factor_solve_phases_scheme(n, nrhs):
    """The launch-per-phase scheme (panel and update launches) against the
    oracle, and against the default look-ahead scheme."""
    case(f"dense factor_solve phases n={n} nrhs={nrhs}")
    A = inputs.dense(n, 0.5, 4500 + n)
    B = inputs.rhs(n, nrhs, 4600 + n)
    X_ref, LU_ref, _ = oracle.solve(A, B)
    ebv.set_dense_tuning(2048, False, 1, 2048)
    try:
        LU, X = dev(A), dev(B)
        info = ebv.lu_factor_solve_(LU, X)
        torch.cuda.synchronize()
    finally:
        ebv.set_dense_tuning()
    LU2, X2 = dev(A), dev(B)
    ebv.lu_factor_solve_(LU2, X2)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    assert fwd_err(host(X), X_ref) <= 1e-12
    assert np.max(np.abs(host(LU) - LU_ref)) <= 1e-12
    assert np.max(np.abs(host(LU2) - host(LU))) <= 1e-13


@pytest.mark.parametrize("n,nrhs", [(1, 1), (64, 1), (65, 3), (200, 8), (257, 9), (513, 2)])
def test_solve_parity(n, nrhs):
    case(f"dense solve n={n} nrhs={nrhs}")
    A = inputs.dense(n, 0.5, 2000 + n)
    B = inputs.rhs(n, nrhs, 3000 + n)
    X_ref, LU_ref, _ = oracle.solve(A, B)
    LU = dev(A)
    ebv.lu_factor_(LU)
    X = dev(B)
    ebv.lu_solve_(LU, X)
    torch.cuda.synchronize()
    assert fwd_err(host(X), X_ref) <= 1e-12
    # the solve alone, on the oracle's own factor
    X2 = dev(B)
    ebv.lu_solve_(dev(LU_ref), X2)
    torch.cuda.synchronize()
    assert fwd_err(host(X2), X_ref) <= 1e-13


@pytest.mark.parametrize("n,nrhs", [(1, 1), (64, 1), (65, 3), (200, 8), (257, 70), (513, 2), (700, 130)])
def test_factor_solve_parity(n, nrhs):
    """ebv_lu_factor_solve: forward substitution carried inside the factor
    (B as extra columns), then the backward substitution."""
    case(f"dense factor_solve n={n} nrhs={nrhs}")
    A = inputs.dense(n, 0.5, 2500 + n)
    B = inputs.rhs(n, nrhs, 3500 + n)
    X_ref, LU_ref, _ = oracle.solve(A, B)
    LU, X = dev(A), dev(B)
    ws = ebv.workspace(ebv.OP_FACTOR_SOLVE, ebv.F64, n, nrhs, 1)
    info = ebv.lu_factor_solve_(LU, X, ws=ws)
    LU2 = dev(A)
    ws2 = ebv.workspace(ebv.OP_FACTOR, ebv.F64, n, 0, 1)
    ebv.lu_factor_(LU2, ws=ws2)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    # no bounded wait gave up: the status word sits at the documented offset
    assert ebv.lib().ebv_workspace_status_offset() == 0
    assert ebv.workspace_status(ws) == 0 and ebv.workspace_status(ws2) == 0
    assert fwd_err(host(X), X_ref) <= 1e-12
    assert np.max(np.abs(host(LU) - LU_ref)) <= 1e-12
    assert torch.equal(LU, LU2)  # the factor is the same computation either way


def test_forward_backward_separately():
    """Forward substitution alone matches the oracle's forward (Eq. 1, LY = B)."""
    n, nrhs = 150, 4
    case("dense forward/backward split")
    A = inputs.dense(n, 0.5, 77)
    LU_ref, _ = oracle.lu_factor(A)
    B = inputs.rhs(n, nrhs, 78)
    Y_ref = oracle.forward(LU_ref, B)
    ws = ebv.workspace(ebv.OP_SOLVE, ebv.F64, n, nrhs, 1)
    w, wb = ebv._ws_args(ws)
    LU = dev(LU_ref)
    Y = dev(B)
    from paper_1907_05767_amd.ebv import _p, _stream, lib
    # solve with an identity upper factor isolates the forward sweep
    LUf = (torch.tril(LU, -1) + torch.eye(n, dtype=LU.dtype, device=LU.device)).contiguous()
    rc = lib().ebv_lu_solve(ebv.handle(), 0, n, nrhs, _p(LUf), n, _p(Y), nrhs, 1, 0, 0, None, w, wb, _stream())
    assert rc == 0
    torch.cuda.synchronize()
    assert fwd_err(host(Y), Y_ref) <= 1e-13


def test_full_size_4096x8():
    """The n=4096, 8 right-hand-side workload at full size."""
    n, nrhs = 4096, 8
    case("dense n=4096 nrhs=8 full size")
    A = inputs.dense(n, 0.5, 2)
    B = inputs.rhs(n, nrhs, 2)
    LU = dev(A)
    info = ebv.lu_factor_(LU)
    X = dev(B)
    ebv.lu_solve_(LU, X)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    LUh, Xh = host(LU), host(X)
    # sampled entries of L U against A (each an O(n) dot product)
    rng = np.random.default_rng(5)
    ii, jj = rng.integers(0, n, 2000), rng.integers(0, n, 2000)
    for i, j in zip(ii, jj):
        k = min(i, j)
        lu = np.dot(LUh[i, :k], LUh[:k, j]) + (LUh[i, j] if i <= j else LUh[i, k] * LUh[k, j])
        assert abs(lu - A[i, j]) <= 1e-13
    # solution against the oracle at full size
    X_ref, LU_ref, _ = oracle.solve(A, B)
    assert fwd_err(Xh, X_ref) <= 1e-12
    assert np.max(np.abs(LUh - LU_ref)) <= 1e-12
    # the fused entry point the benchmark times, in its launch configuration
    case("dense n=4096 nrhs=8 factor_solve full size")
    LU2, X2 = dev(A), dev(B)
    ws = ebv.workspace(ebv.OP_FACTOR_SOLVE, ebv.F64, n, nrhs, 1)
    info2 = ebv.lu_factor_solve_(LU2, X2, ws=ws)
    torch.cuda.synchronize()
    assert int(info2.item()) == 0
    assert fwd_err(host(X2), X_ref) <= 1e-12
    assert torch.equal(LU2, LU)


def test_zero_pivot_info():
    case("zero pivot info")
    A = np.array([[0.0, 1.0], [1.0, 1.0]])
    info = ebv.lu_factor_(dev(A))
    torch.cuda.synchronize()
    assert int(info.item()) == 1
    A = inputs.dense(100, 0.5, 1)
    A[:2, :2] = 1.0  # singular leading 2x2 minor: second pivot is exactly zero
    info = ebv.lu_factor_(dev(A))
    torch.cuda.synchronize()
    assert int(info.item()) == oracle.lu_factor(A)[1] == 2
    info = ebv.lu_factor_solve_(dev(A), dev(np.ones((100, 2))))
    torch.cuda.synchronize()
    assert int(info.item()) == 2


def test_bitwise_deterministic():
    case("determinism n=300")
    A = inputs.dense(300, 0.5, 9)
    t1, t2 = dev(A), dev(A)
    ebv.lu_factor_(t1)
    ebv.lu_factor_(t2)
    torch.cuda.synchronize()
    assert torch.equal(t1, t2)


@pytest.mark.parametrize("batch,n,nrhs", [(3, 1, 1), (7, 50, 2), (5, 64, 1), (3, 200, 1), (4, 130, 3), (2, 300, 8), (2, 700, 2)])
def test_uniform_batch_parity(batch, n, nrhs):
    case(f"uniform batch {batch}x{n} nrhs={nrhs}")
    A, B = inputs.uniform_batch(batch, n, 0.5, 40 + n, nrhs)
    LU = dev(A)
    info = ebv.lu_factor_(LU)
    X = dev(B)
    ebv.lu_solve_(LU, X)
    torch.cuda.synchronize()
    assert np.all(host(info) == 0)
    LUh, Xh = host(LU), host(X)
    for b in range(batch):
        X_ref, LU_ref, _ = oracle.solve(A[b], B[b])
        assert np.max(np.abs(LUh[b] - LU_ref)) <= 1e-12
        assert fwd_err(Xh[b], X_ref) <= 1e-12


def test_float32_factor():
    """The float factor (used by the mixed-precision path) against the oracle
    run on the float-rounded matrix: agreement to float accuracy."""
    n = 257
    case("float32 dense factor")
    A = inputs.dense(n, 0.5, 5)
    A32 = A.astype(np.float32)
    LU_ref, _ = oracle.lu_factor(A32.astype(np.float64))
    t = dev(A32, torch.float32)
    ebv.lu_factor_(t)
    torch.cuda.synchronize()
    assert np.max(np.abs(host(t).astype(np.float64) - LU_ref)) <= 2e-5


def _lu_abs(LU):
    """|L| |U| of a packed factor (the scale of its rounding errors)."""
    L = np.abs(np.tril(LU, -1)) + np.eye(len(LU))
    U = np.abs(np.triu(LU))
    return L @ U


@pytest.mark.parametrize("n,forced", [(1100, True), (2112, False)])
def test_float32_factor_class_path(n, forced):
    """The float factor through the column-class block steps (forced on every
    launch at n = 1100; engaged by the default split at n = 2112, whose
    trailing region exceeds 1024) against the oracle run on the
    float-rounded matrix, element by element within 16 sqrt(n) u (|L||U|)_ij,
    u = 2^-24.  A dropped 64-step update or a wrong operand would leave
    errors of order (|L||U|)_ij itself."""
    case(f"float32 dense factor n={n} class path forced={forced}")
    A = inputs.dense(n, 0.5, 31 + n)
    A32 = A.astype(np.float32)
    LU_ref, _ = oracle.lu_factor(A32.astype(np.float64))
    if forced:
        ebv.set_dense_tuning(0, True, 3, 0)
    try:
        t = dev(A32, torch.float32)
        info = ebv.lu_factor_(t)
        torch.cuda.synchronize()
    finally:
        ebv.set_dense_tuning()
    assert int(info.item()) == 0
    diff = np.abs(host(t).astype(np.float64) - LU_ref)
    scale = _lu_abs(LU_ref)
    ratio = (diff / scale).max() / (np.sqrt(n) * 2.0 ** -24)
    print(f"float factor n={n}: max |dLU| / (sqrt(n) u |L||U|) = {ratio:.3f}")
    assert ratio <= 16.0


def _set_f32_group(g, tmp_path):
    """The FP32 factor's column-class group through a one-key tuning table
    (a table updates only the keys it names)."""
    path = tmp_path / f"f32_group_{g}.txt"
    path.write_text(f"dense.f32.defer_group {g}\n")
    assert ebv.lib().ebv_load_tuning(ebv.handle(), str(path).encode()) == 0


@pytest.mark.parametrize("g", [1, 2, 3])
def test_float32_factor_groups(g, tmp_path):
    """The float factor with each other column-class group size (the default
    is 4), the class path forced on every launch, against the oracle run on
    the float-rounded matrix as in the test above."""
    n = 1100
    case(f"float32 dense factor n={n} f32 group {g}")
    A = inputs.dense(n, 0.5, 31 + n)
    A32 = A.astype(np.float32)
    LU_ref, _ = oracle.lu_factor(A32.astype(np.float64))
    ebv.set_dense_tuning(0, True, 3, 0)
    _set_f32_group(g, tmp_path)
    try:
        t = dev(A32, torch.float32)
        info = ebv.lu_factor_(t)
        torch.cuda.synchronize()
    finally:
        ebv.set_dense_tuning()
        _set_f32_group(4, tmp_path)  # the library default, then the table's value if there is one
        if os.path.exists(ebv.TUNING_PATH):
            assert ebv.lib().ebv_load_tuning(ebv.handle(), ebv.TUNING_PATH.encode()) == 0
    assert int(info.item()) == 0
    diff = np.abs(host(t).astype(np.float64) - LU_ref)
    ratio = (diff / _lu_abs(LU_ref)).max() / (np.sqrt(n) * 2.0 ** -24)
    assert ratio <= 16.0, ratio


def test_dense_n256_single_rhs():
    """The n = 256, 1 right-hand-side workload (factor + solve through the
    fused entry point) against the oracle."""
    n, nrhs = 256, 1
    case("dense n=256 nrhs=1")
    A = inputs.dense(n, 0.5, 1)
    B = inputs.rhs(n, nrhs, 1)
    X_ref, LU_ref, _ = oracle.solve(A, B)
    LU, X = dev(A), dev(B)
    info = ebv.lu_factor_solve_(LU, X)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    assert fwd_err(host(X), X_ref) <= 1e-12
    assert np.max(np.abs(host(LU) - LU_ref)) <= 1e-12


def _padded(a, ld):
    """a (rows x cols) inside a rows x ld device buffer, padding filled with a sentinel."""
    rows, cols = a.shape
    buf = np.full((rows, ld), 12345.0)
    buf[:, :cols] = a
    return dev(buf)


@pytest.mark.parametrize("n,nrhs,lda,ldb", [(100, 3, 131, 7), (300, 8, 320, 16), (65, 1, 65, 3)])
def test_leading_dimensions(n, nrhs, lda, ldb):
    """lda > n and ldb > nrhs through the C ABI: the factor, the solves, the
    fused factor + solve, the adjoint and mixed precision read and write only
    the n x n and n x nrhs parts (the padding keeps its sentinel)."""
    from paper_1907_05767_amd.ebv import _p, _stream, _ws_args, handle, lib
    case(f"leading dimensions n={n} nrhs={nrhs} lda={lda} ldb={ldb}")
    A = inputs.dense(n, 0.5, 90 + n)
    B = inputs.rhs(n, nrhs, 91 + n)
    W = inputs.rhs(n, nrhs, 92 + n)
    X_ref, LU_ref, _ = oracle.solve(A, B)
    bbar_ref, abar_ref = oracle.lu_solve_adjoint(LU_ref, X_ref, W)
    h = handle()
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    # fused factor + solve
    tA, tB = _padded(A, lda), _padded(B, ldb)
    w, wb = _ws_args(ebv.workspace(ebv.OP_FACTOR_SOLVE, ebv.F64, n, nrhs, 1))
    assert lib().ebv_lu_factor_solve(h, 0, n, nrhs, _p(tA), lda, _p(tB), ldb, _p(info), w, wb, _stream()) == 0
    # factor, then solve
    tA2, tB2 = _padded(A, lda), _padded(B, ldb)
    w2, wb2 = _ws_args(ebv.workspace(ebv.OP_FACTOR, ebv.F64, n, 0, 1))
    assert lib().ebv_lu_factor(h, 0, n, _p(tA2), lda, 1, 0, _p(info), w2, wb2, _stream()) == 0
    w3, wb3 = _ws_args(ebv.workspace(ebv.OP_SOLVE, ebv.F64, n, nrhs, 1))
    assert lib().ebv_lu_solve(h, 0, n, nrhs, _p(tA2), lda, _p(tB2), ldb, 1, 0, 0, _p(info), w3, wb3, _stream()) == 0
    # adjoint with padded LU, X, Bbar and Abar
    tLU, tX, tW = _padded(LU_ref, lda), _padded(X_ref, ldb + 1), _padded(W, ldb)
    tAb = _padded(np.zeros((n, n)), lda + 2)
    w4, wb4 = _ws_args(ebv.workspace(ebv.OP_ADJOINT, ebv.F64, n, nrhs, 1))
    assert lib().ebv_lu_solve_adjoint(h, 0, n, nrhs, _p(tLU), lda, _p(tX), ldb + 1, _p(tW), ldb, _p(tAb), lda + 2,
                                      1, 0, 0, 0, 0, _p(info), w4, wb4, _stream()) == 0
    # mixed precision with padded A, B and X
    tAm, tBm, tXm = _padded(A, lda), _padded(B, ldb), _padded(np.zeros((n, nrhs)), ldb + 3)
    w5, wb5 = _ws_args(ebv.workspace(ebv.OP_MIXED, ebv.F64, n, nrhs, 1))
    assert lib().ebv_lu_solve_mixed(h, n, nrhs, _p(tAm), lda, _p(tBm), ldb, _p(tXm), ldb + 3, 10, 1e-12, None, None,
                                    _p(info), w5, wb5, _stream()) == 0
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    for t, ld, cols, ref in ((tA, lda, n, LU_ref), (tB, ldb, nrhs, X_ref), (tA2, lda, n, LU_ref),
                             (tB2, ldb, nrhs, X_ref), (tW, ldb, nrhs, bbar_ref), (tAb, lda + 2, n, abar_ref),
                             (tXm, ldb + 3, nrhs, X_ref)):
        hv = host(t)
        assert np.all(hv[:, cols:] == 12345.0), "padding written"
        if ref is X_ref or ref is bbar_ref:
            assert fwd_err(hv[:, :cols], ref) <= 1e-12
        else:
            assert np.max(np.abs(hv[:, :cols] - ref)) <= 1e-12 * max(1.0, np.abs(ref).max())
    assert np.array_equal(host(tAm)[:, :n], A) and np.array_equal(host(tBm)[:, :nrhs], B)


def test_strided_uniform_batch():
    """batch > 1 with strideA > n * lda and strideB > n * ldb."""
    from paper_1907_05767_amd.ebv import _p, _stream, handle, lib
    batch, n, nrhs, lda, ldb = 3, 90, 2, 97, 5
    case("strided uniform batch")
    A, B = inputs.uniform_batch(batch, n, 0.5, 93, nrhs)
    sA, sB = n * lda + 11, n * ldb + 7
    bufA = np.full(batch * sA, 7.0)
    bufB = np.full(batch * sB, 7.0)
    for k in range(batch):
        bufA[k * sA:k * sA + n * lda].reshape(n, lda)[:, :n] = A[k]
        bufB[k * sB:k * sB + n * ldb].reshape(n, ldb)[:, :nrhs] = B[k]
    tA, tB = dev(bufA), dev(bufB)
    info = torch.zeros(batch, dtype=torch.int32, device="cuda")
    h = handle()
    assert lib().ebv_lu_factor(h, 0, n, _p(tA), lda, batch, sA, _p(info), None, 0, _stream()) == 0
    assert lib().ebv_lu_solve(h, 0, n, nrhs, _p(tA), lda, _p(tB), ldb, batch, sA, sB, None, None, 0, _stream()) == 0
    torch.cuda.synchronize()
    assert np.all(host(info) == 0)
    hA, hB = host(tA), host(tB)
    for k in range(batch):
        X_ref, LU_ref, _ = oracle.solve(A[k], B[k])
        lu = hA[k * sA:k * sA + n * lda].reshape(n, lda)
        x = hB[k * sB:k * sB + n * ldb].reshape(n, ldb)
        assert np.max(np.abs(lu[:, :n] - LU_ref)) <= 1e-12 and np.all(lu[:, n:] == 7.0)
        assert fwd_err(x[:, :nrhs], X_ref) <= 1e-12 and np.all(x[:, nrhs:] == 7.0)


def test_bounded_wait_give_up_is_reported():
    """With a one-spin wait budget every wait that does not find its data at
    once gives up: all launches still end, info reports -1 (the status word
    holds bit 1), and the next call with the default budget on the same
    workspace is correct again."""
    n, nrhs = 1024, 4
    case("bounded-wait give-up reported through info")
    A = inputs.dense(n, 0.5, 44)
    B = inputs.rhs(n, nrhs, 45)
    X_ref, _, _ = oracle.solve(A, B)
    ws = ebv.workspace(ebv.OP_FACTOR_SOLVE, ebv.F64, n, nrhs, 1)
    ebv.set_wait_limit(1)
    try:
        info = ebv.lu_factor_solve_(dev(A), dev(B), ws=ws)
        torch.cuda.synchronize()
    finally:
        ebv.set_wait_limit(0)
    assert int(info.item()) == -1
    assert ebv.workspace_status(ws) & 1
    with pytest.raises(ebv.EbvError):
        ebv.check_info(info, "factor_solve")
    LU, X = dev(A), dev(B)
    info = ebv.lu_factor_solve_(LU, X, ws=ws)
    torch.cuda.synchronize()
    assert int(info.item()) == 0 and ebv.workspace_status(ws) == 0
    assert fwd_err(host(X), X_ref) <= 1e-12
