"""Independent checks ("pins") of the FP64 oracle.

Each check compares the oracle with something it does not compute itself:
classical determinant identities evaluated in exact rational arithmetic,
Cramer's rule, a closed form, a library routine on a case where it reduces to
the same factorization, or an invariant the mathematics fixes.  The functions
raise AssertionError on disagreement so the mutation tests can reuse them
against deliberately broken builds of the oracle.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np

import oracle
from paper_1907_05767_amd import inputs

EPS = np.finfo(np.float64).eps


# ------------------------------------------------------------ exact helpers --
def det_leibniz(M):
    """Determinant by the Leibniz permutation expansion (exact for Fractions)."""
    n = len(M)
    if n == 0:
        return Fraction(1)
    total = Fraction(0)
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for a in range(n) for b in range(a + 1, n) if perm[a] > perm[b])
        p = Fraction(1)
        for i in range(n):
            p *= M[i][perm[i]]
            if p == 0:
                break
        total += -p if inv % 2 else p
    return total


def to_frac(A):
    return [[Fraction(float(v)) for v in row] for row in np.asarray(A)]


def minor(F, rows, cols):
    return det_leibniz([[F[r][c] for c in cols] for r in rows])


def doolittle_by_minors(F):
    """Exact Doolittle factors from determinant identities (no elimination):
    u_ij = det(A[0..i, (0..i-1) + j]) / det(A[0..i-1, 0..i-1])   (i <= j)
    l_ij = det(A[(0..j-1) + i, 0..j]) / det(A[0..j, 0..j])       (i >  j)."""
    n = len(F)
    lead = [minor(F, range(k), range(k)) for k in range(n + 1)]
    L = [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    U = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        for j in range(i, n):
            U[i][j] = minor(F, list(range(i + 1)), list(range(i)) + [j]) / lead[i]
        for r in range(i + 1, n):
            L[r][i] = minor(F, list(range(i)) + [r], list(range(i + 1))) / lead[i + 1]
    return L, U, lead[n]


def cramer(F, b):
    n = len(F)
    d = det_leibniz(F)
    out = []
    for i in range(n):
        Mi = [[(b[r] if c == i else F[r][c]) for c in range(n)] for r in range(n)]
        out.append(det_leibniz(Mi) / d)
    return out


# ------------------------------------------------------------------- pins ---
def pin_minors(n: int, seed: int, s: float = 0.5):
    """Oracle L, U against the determinant-identity factors, exact arithmetic."""
    A = inputs.dense(n, s, seed)
    LU, info = oracle.lu_factor(A)
    assert info == 0
    L, U = oracle.split_lu(LU)
    Le, Ue, det = doolittle_by_minors(to_frac(A))
    Lx = np.array([[float(v) for v in r] for r in Le])
    Ux = np.array([[float(v) for v in r] for r in Ue])
    scale = 1.0
    tol = 8 * n * EPS * scale
    assert np.max(np.abs(L - Lx)) <= tol, np.max(np.abs(L - Lx))
    assert np.max(np.abs(U - Ux)) <= tol, np.max(np.abs(U - Ux))
    assert abs(np.prod(np.diag(U)) - float(det)) <= tol * abs(float(det))


def pin_cramer(n: int, seed: int, nrhs: int = 2):
    A = inputs.dense(n, 0.5, seed)
    B = inputs.rhs(n, nrhs, seed + 1000)
    X, _, _ = oracle.solve(A, B)
    F = to_frac(A)
    for c in range(nrhs):
        xe = np.array([float(v) for v in cramer(F, [Fraction(float(v)) for v in B[:, c]])])
        err = np.max(np.abs(X[:, c] - xe)) / max(np.max(np.abs(xe)), 1e-300)
        assert err <= 16 * n * EPS, err


def tridiag_closed_form(n: int, a: float, b: float, c: float):
    """Doolittle factors of the constant tridiagonal matrix (sub b, diag a, super c).
    With D_i the leading minors, D_i = (r+^(i+1) - r-^(i+1)) / (r+ - r-),
    r+- = (a +- sqrt(a^2 - 4bc)) / 2;  U_ii = D_i / D_(i-1), U_(i,i+1) = c,
    L_(i+1,i) = b D_(i-1) / D_i.  Written with q = r-/r+ to stay in range."""
    disc = math.sqrt(a * a - 4 * b * c)
    rp, rm = (a + disc) / 2, (a - disc) / 2
    q = rm / rp
    i = np.arange(1, n + 1, dtype=np.float64)
    # U_ii (1-based i) = r+ (1 - q^(i+1)) / (1 - q^i)
    udiag = rp * (1 - q ** (i + 1)) / (1 - q ** i)
    lsub = b / udiag[:-1]
    det_log = np.sum(np.log(np.abs(udiag)))
    return udiag, lsub, det_log


def tridiag_dense(n, a, b, c):
    A = np.diag(np.full(n, a)) + np.diag(np.full(n - 1, b), -1) + np.diag(np.full(n - 1, c), 1)
    return A


def pin_tridiag(n: int, a=1.0, b=0.25, c=0.25, use_band=False):
    udiag, lsub, _ = tridiag_closed_form(n, a, b, c)
    if use_band:
        AB = np.zeros((n, 3))
        AB[:, 0] = b
        AB[:, 1] = a
        AB[:, 2] = c
        AB[0, 0] = 0.0
        AB[-1, 2] = 0.0
        LUB, info = oracle.lu_factor_band(AB, 1, 1)
        assert info == 0
        u = LUB[:, 1]
        l = LUB[1:, 0]
        sup = LUB[:-1, 2]
    else:
        LU, info = oracle.lu_factor(tridiag_dense(n, a, b, c))
        assert info == 0
        u = np.diag(LU)
        l = np.diag(LU, -1)
        sup = np.diag(LU, 1)
        # elimination must not create fill outside the tridiagonal band
        assert np.all(np.triu(LU, 2) == 0.0) and np.all(np.tril(LU, -2) == 0.0)
    tol = 64 * EPS
    assert np.max(np.abs(u - udiag) / np.abs(udiag)) <= tol
    assert np.max(np.abs(l - lsub) / np.maximum(np.abs(lsub), 1e-300)) <= tol
    assert np.all(sup == c)


def pin_invariants(n: int, seed: int, s: float = 0.5):
    A = inputs.dense(n, s, seed)
    LU, info = oracle.lu_factor(A)
    assert info == 0
    L, U = oracle.split_lu(LU)
    rel = np.linalg.norm(L @ U - A) / np.linalg.norm(A)
    assert rel <= 1e-14, rel
    sign, logdet = np.linalg.slogdet(A)
    assert sign == np.prod(np.sign(np.diag(U)))
    assert abs(np.sum(np.log(np.abs(np.diag(U)))) - logdet) <= 1e-12 * max(1.0, abs(logdet))


def pin_lapack(n: int, seed: int, s: float = 0.5):
    """LAPACK getrf (partial pivoting) picks the identity permutation on these
    matrices (column dominance of the first column is not guaranteed, so it
    is checked), in which case its L and U are the Doolittle factors."""
    import scipy.linalg as sl
    A = inputs.dense(n, s, seed)
    lu_l, piv = sl.lu_factor(A)
    if not np.array_equal(piv, np.arange(n)):
        return False
    LU, info = oracle.lu_factor(A)
    assert info == 0
    err = np.max(np.abs(LU - lu_l))
    assert err <= 32 * n * EPS, err
    return True


def pin_solve_numpy(n: int, seed: int, nrhs: int = 3, s: float = 0.5):
    A = inputs.dense(n, s, seed)
    B = inputs.rhs(n, nrhs, seed + 7)
    X, _, _ = oracle.solve(A, B)
    Xr = np.linalg.solve(A, B)
    err = np.max(np.abs(X - Xr)) / np.max(np.abs(Xr))
    assert err <= 1e-13, err


def pin_band_tridiag(n: int):
    pin_tridiag(n, use_band=True)


def pin_band_vs_numpy(n: int, kl: int, ku: int, seed: int, nrhs: int = 2):
    AB = inputs.band(n, kl, ku, 0.5, seed)
    A = inputs.band_to_dense(AB, kl, ku)
    LUB, info = oracle.lu_factor_band(AB, kl, ku)
    assert info == 0
    # expand the band factors and check L U = A, with both factors inside the band
    LUd = inputs.band_to_dense(LUB, kl, ku)
    L, U = oracle.split_lu(LUd)
    assert np.linalg.norm(L @ U - A) / np.linalg.norm(A) <= 1e-14
    B = inputs.rhs(n, nrhs, seed + 3)
    X = oracle.lu_solve_band(LUB, kl, ku, B)
    Xr = np.linalg.solve(A, B)
    assert np.max(np.abs(X - Xr)) / np.max(np.abs(Xr)) <= 1e-13


def pin_adjoint(n: int, seed: int, nrhs: int = 2):
    """bbar = A^{-T} xbar against an independent solve of the transposed system;
    Euler identities <bbar, B> = <xbar, X> and <Abar, A> = -<xbar, X>."""
    A = inputs.dense(n, 0.5, seed)
    B = inputs.rhs(n, nrhs, seed + 1)
    W = inputs.rhs(n, nrhs, seed + 2)
    X, LU, _ = oracle.solve(A, B)
    bbar, abar = oracle.lu_solve_adjoint(LU, X, W)
    ref = np.linalg.solve(A.T, W)
    assert np.max(np.abs(bbar - ref)) / np.max(np.abs(ref)) <= 1e-13
    loss = float(np.sum(W * X))
    assert abs(float(np.sum(bbar * B)) - loss) <= 1e-12 * max(1.0, np.abs(W * X).sum())
    assert abs(float(np.sum(abar * A)) + loss) <= 1e-12 * max(1.0, np.abs(W * X).sum())
    # Abar = -bbar x^T elementwise against an outer product
    assert np.max(np.abs(abar + bbar @ X.T)) <= 1e-14 * max(1.0, np.abs(bbar @ X.T).max())


def pin_adjoint_fd(n: int, seed: int, h: float = 1e-6, samples: int = 24):
    """Central finite differences of L = sum(w * x) on the oracle's own solve."""
    A = inputs.dense(n, 0.5, seed)
    b = inputs.rhs(n, 1, seed + 1)
    w = inputs.rhs(n, 1, seed + 2)
    X, LU, _ = oracle.solve(A, b)
    bbar, abar = oracle.lu_solve_adjoint(LU, X, w)
    rng = np.random.Generator(np.random.PCG64(seed))
    fd, an = [], []
    for _ in range(samples):
        i, j = rng.integers(0, n, 2)
        Ap, Am = A.copy(), A.copy()
        Ap[i, j] += h
        Am[i, j] -= h
        lp = float(np.sum(w * oracle.solve(Ap, b)[0]))
        lm = float(np.sum(w * oracle.solve(Am, b)[0]))
        fd.append((lp - lm) / (2 * h))
        an.append(abar[i, j])
        bp, bm = b.copy(), b.copy()
        bp[i, 0] += h
        bm[i, 0] -= h
        lp = float(np.sum(w * oracle.solve(A, bp)[0]))
        lm = float(np.sum(w * oracle.solve(A, bm)[0]))
        fd.append((lp - lm) / (2 * h))
        an.append(bbar[i, 0])
    fd, an = np.array(fd), np.array(an)
    err = np.linalg.norm(fd - an) / np.linalg.norm(an)
    return err


# ------------------------------------------------------- explicit inverse ---
def gauss_jordan_inverse(F):
    """Exact inverse of a Fraction matrix by Gauss-Jordan elimination (no
    pivoting needed for these strictly dominant matrices)."""
    n = len(F)
    M = [list(r) + [Fraction(int(i == j)) for j in range(n)] for i, r in enumerate(F)]
    for k in range(n):
        p = M[k][k]
        M[k] = [v / p for v in M[k]]
        for i in range(n):
            if i != k and M[i][k] != 0:
                f = M[i][k]
                M[i] = [a - f * b for a, b in zip(M[i], M[k])]
    return [r[n:] for r in M]


def pin_inverse_exact(n: int, seed: int, s: float = 0.5):
    """oracle.inverse against the exact rational inverse, rounded once."""
    A = inputs.dense(n, s, seed)
    X, _ = oracle.inverse(A)
    Xe = np.array([[float(v) for v in r] for r in gauss_jordan_inverse(to_frac(A))])
    scale = np.abs(Xe).max()
    assert np.max(np.abs(X - Xe)) <= 8 * n * EPS * scale, np.max(np.abs(X - Xe))


def elementary_product_inverse(LU):
    """A^{-1} as the ordered product of elementary factors (Eq. 4-c), formed
    matrix by matrix from Doolittle factors: with L = prod_r (I + l_r e_r^T)
    and U = D (E_{n-2} ... E_0), E_r = I + e_r w_r^T (row r of U / U_rr right
    of the diagonal), A^{-1} = E_0^{-1} ... E_{n-2}^{-1} D^{-1}
    (I - l_{n-2} e_{n-2}^T) ... (I - l_0 e_0^T)."""
    n = LU.shape[0]
    I = np.eye(n)
    M = I.copy()
    for r in range(n - 1):  # upper elementary factors, left to right
        E = I.copy()
        E[r, r + 1:] = -LU[r, r + 1:] / LU[r, r]
        M = M @ E
    M = M @ np.diag(1.0 / np.diag(LU))
    for r in range(n - 2, -1, -1):  # lower elementary factors
        E = I.copy()
        E[r + 1:, r] = -LU[r + 1:, r]
        M = M @ E
    return M


def pin_inverse_product_form(n: int, seed: int, s: float = 0.5):
    """oracle.inverse equals the Eq. 4-c product of elementary factors built
    from the oracle's own factors, and A X = X A = I."""
    A = inputs.dense(n, s, seed)
    X, LU = oracle.inverse(A)
    P = elementary_product_inverse(LU)
    assert np.max(np.abs(X - P)) <= 16 * n * EPS * np.abs(P).max()
    I = np.eye(n)
    assert np.max(np.abs(A @ X - I)) <= 16 * n * EPS
    assert np.max(np.abs(X @ A - I)) <= 16 * n * EPS


# ----------------------------------------------------------------- skyline ---
def pin_skyline_vs_dense(n: int, seed: int, wshort: int = 8, wlong: int = 100, plong: float = 0.1):
    """The skyline oracle performs the dense oracle's nonzero operations in
    the same order, so on the densified matrix the two agree bitwise; and the
    dense factors vanish outside the envelope (no fill without pivoting)."""
    f, rp, AL, g, cp, AU = inputs.skyline(n, wshort, wlong, plong, 0.5, seed)
    A = inputs.skyline_to_dense(f, rp, AL, g, cp, AU)
    LL, UU, info = oracle.lu_factor_skyline(f, rp, AL, g, cp, AU)
    LU, info_d = oracle.lu_factor(A)
    assert info == info_d == 0
    D = inputs.skyline_to_dense(f, rp, LL, g, cp, UU)
    assert np.array_equal(D, LU)
    i, j = np.indices(A.shape)
    outside = ((j < i) & (j < np.asarray(f)[:, None])) | ((j >= i) & (i < np.asarray(g)[None, :]))
    assert np.all(LU[outside] == 0.0)
    B = inputs.rhs(n, 2, seed)
    assert np.array_equal(oracle.lu_solve_skyline(f, rp, LL, g, cp, UU, B), oracle.lu_solve(LU, B))


def pin_skyline_tridiag(n: int, a: float = 1.0, b: float = 0.25, c: float = 0.25):
    """Tridiagonal matrix in skyline storage (f_i = i - 1, g_j = j - 1):
    factors against the closed form of the D_i recurrence."""
    idx = np.arange(n)
    f = np.maximum(0, idx - 1).astype(np.int32)
    g = f.copy()
    rp = np.zeros(n + 1, np.int64)
    cp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum(idx - f)
    cp[1:] = np.cumsum(idx - g + 1)
    AL = np.full(int(rp[-1]), b)
    AU = np.full(int(cp[-1]), c)
    AU[cp[1:] - 1] = a
    LL, UU, info = oracle.lu_factor_skyline(f, rp, AL, g, cp, AU)
    assert info == 0
    udiag, lsub, _ = tridiag_closed_form(n, a, b, c)
    assert np.max(np.abs(UU[cp[1:] - 1] - udiag)) <= 64 * EPS
    assert np.max(np.abs(LL - lsub)) <= 64 * EPS
    assert np.all(UU[np.setdiff1d(np.arange(len(UU)), cp[1:] - 1)] == c)  # U_(i,i+1) = c exactly
