"""CPU tests: pin the FP64 oracle to the mathematics (not to itself)."""
from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1907_05767_amd import inputs
from tests import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------- generator -------
def test_generator_dominance_and_determinism():
    for n in (1, 2, 17, 300):
        A = inputs.dense(n, 0.5, 11)
        assert np.array_equal(A, inputs.dense(n, 0.5, 11))
        assert np.all(np.diag(A) == 1.0)
        off = np.abs(A).sum(axis=1) - 1.0
        if n > 1:
            assert np.max(np.abs(off - 0.5)) <= 4 * n * pins.EPS
    AB = inputs.band(200, 64, 64, 0.5, 3)
    A = inputs.band_to_dense(AB, 64, 64)
    assert np.all(np.diag(A) == 1.0)
    assert np.max(np.abs(np.abs(A).sum(axis=1) - 1.5)) <= 1e-13
    i, j = np.indices(A.shape)
    assert np.all(A[np.abs(i - j) > 64] == 0.0)


def test_generator_ragged_layout():
    ns, offA, A, offB, B = inputs.ragged(9, 16, 40, 0.5, 4)
    assert ns.min() >= 16 and ns.max() <= 40
    assert offA[-1] + int(ns[-1]) ** 2 == A.size
    assert offB[-1] + int(ns[-1]) == B.size
    k = 5
    n = int(ns[k])
    Ak = A[offA[k]:offA[k] + n * n].reshape(n, n)
    assert np.all(np.diag(Ak) == 1.0)


# ------------------------------------------------------------ golden -------
def test_golden_3x3_hand_derivation():
    g = json.load(open(os.path.join(GOLDEN, "doolittle_3x3.json")))
    F = lambda m: np.array([[float(Fraction(v)) for v in r] for r in m])
    A = F(g["A"])
    LU, info = oracle.lu_factor(A)
    assert info == 0
    L, U = oracle.split_lu(LU)
    assert np.max(np.abs(L - F(g["L"]))) <= 2 * pins.EPS
    assert np.max(np.abs(U - F(g["U"]))) <= 2 * pins.EPS
    assert abs(np.prod(np.diag(U)) - float(Fraction(g["det"]))) <= 4 * pins.EPS
    b = np.array([float(Fraction(v)) for v in g["b"]])
    y = oracle.forward(LU, b)
    assert np.max(np.abs(y - np.array([float(Fraction(v)) for v in g["y"]]))) <= 4 * pins.EPS
    x = oracle.lu_solve(LU, b)
    assert np.max(np.abs(x - np.array([float(Fraction(v)) for v in g["x"]]))) <= 8 * pins.EPS


# ------------------------------------------------------- exact identities ---
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_minor_identities(n):
    for seed in range(3):
        pins.pin_minors(n, 100 + seed)


def test_minor_identities_nonsymmetric_margin():
    # row sum 0.9: smaller dominance margin, larger multipliers
    pins.pin_minors(5, 7, s=0.9)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_cramer(n):
    for seed in range(4):
        pins.pin_cramer(n, 200 + seed)


# ------------------------------------------------------------ closed form ---
@pytest.mark.parametrize("n", [2, 3, 10, 257, 4000])
def test_tridiagonal_closed_form(n):
    pins.pin_tridiag(n)
    pins.pin_tridiag(n, a=1.0, b=0.3, c=-0.2)


# ------------------------------------------------------------- invariants ---
@pytest.mark.parametrize("n,s", [(64, 0.5), (300, 0.5), (300, 0.9), (513, 0.5)])
def test_invariants(n, s):
    pins.pin_invariants(n, 31 + n, s)


@pytest.mark.parametrize("n", [50, 200])
def test_against_lapack_getrf(n):
    hit = 0
    for seed in range(4):
        hit += bool(pins.pin_lapack(n, 40 + seed))
    assert hit >= 1  # identity permutation must occur for this matrix class


@pytest.mark.parametrize("n,s", [(1, 0.5), (7, 0.5), (100, 0.5), (100, 0.9)])
def test_solve_vs_numpy(n, s):
    pins.pin_solve_numpy(n, 300 + n, s=s)


# --------------------------------------------------------- special cases ---
def test_special_cases():
    n = 9
    rng = np.random.Generator(np.random.PCG64(5))
    # identity: L = U = I, x = b exactly
    LU, info = oracle.lu_factor(np.eye(n))
    assert info == 0 and np.array_equal(LU, np.eye(n))
    b = rng.standard_normal(n)
    assert np.array_equal(oracle.lu_solve(LU, b), b)
    # upper triangular: L = I, U = A exactly
    Ut = np.triu(rng.uniform(-1, 1, (n, n))) + 2 * np.eye(n)
    LU, info = oracle.lu_factor(Ut)
    assert info == 0 and np.array_equal(LU, Ut)
    # unit lower triangular: L = A, U = I exactly (Doolittle)
    Lt = np.tril(rng.uniform(-1, 1, (n, n)), -1) + np.eye(n)
    LU, info = oracle.lu_factor(Lt)
    assert info == 0 and np.array_equal(LU, Lt)
    # diagonal: x_i = b_i / a_ii correctly rounded
    d = rng.uniform(0.5, 2.0, n)
    LU, info = oracle.lu_factor(np.diag(d))
    assert np.array_equal(oracle.lu_solve(LU, b), b / d)
    # 1x1 and the 2x2 closed form
    LU, info = oracle.lu_factor(np.array([[3.0]]))
    assert LU[0, 0] == 3.0 and info == 0
    A2 = np.array([[2.0, 0.5], [0.75, 1.5]])
    LU, info = oracle.lu_factor(A2)
    l21 = 0.75 / 2.0
    assert LU[1, 0] == l21 and LU[0, 1] == 0.5 and LU[1, 1] == 1.5 - l21 * 0.5


def test_zero_pivot_info():
    LU, info = oracle.lu_factor(np.array([[0.0, 1.0], [1.0, 1.0]]))
    assert info == 1
    A = np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    LU, info = oracle.lu_factor(A)
    assert info == 2
    AB = np.array([[0.0, 0.0, 1.0], [1.0, 1.0, 0.0]])  # kl=ku=1, a11 = 0
    _, info = oracle.lu_factor_band(AB, 1, 1)
    assert info == 1


def test_nan_propagates():
    A = inputs.dense(6, 0.5, 1)
    A[3, 2] = np.nan
    LU, info = oracle.lu_factor(A)
    x = oracle.lu_solve(LU, np.ones(6))
    assert np.isnan(x).any()


# ------------------------------------------------------------------- band ---
@pytest.mark.parametrize("n", [2, 5, 300, 5000])
def test_band_tridiagonal_closed_form(n):
    pins.pin_band_tridiag(n)


@pytest.mark.parametrize("n,kl,ku", [(1, 0, 0), (10, 3, 2), (129, 64, 64), (300, 64, 64), (200, 5, 17)])
def test_band_vs_numpy(n, kl, ku):
    pins.pin_band_vs_numpy(n, kl, ku, 60 + n)


def test_band_equals_dense_oracle_on_band_entries():
    n, kl, ku = 150, 7, 4
    AB = inputs.band(n, kl, ku, 0.5, 9)
    LUB, _ = oracle.lu_factor_band(AB, kl, ku)
    LUd, _ = oracle.lu_factor(inputs.band_to_dense(AB, kl, ku))
    # the dense elimination only ever subtracts exact zeros outside the band,
    # so the band entries coincide bit for bit
    assert np.array_equal(inputs.band_to_dense(LUB, kl, ku), LUd)


# ---------------------------------------------------------------- adjoint ---
@pytest.mark.parametrize("n", [1, 3, 40, 257])
def test_adjoint_identities(n):
    pins.pin_adjoint(n, 500 + n)


def test_adjoint_finite_differences():
    err = pins.pin_adjoint_fd(24, 8)
    # central differences at h = 1e-6: truncation O(h^2) plus rounding eps*|L|/h
    assert err <= 1e-8, err


# -------------------------------------------------------- mixed precision ---
@pytest.mark.parametrize("n,s", [(50, 0.5), (200, 0.9)])
def test_refine_mixed(n, s):
    A = inputs.dense(n, s, 70)
    B = inputs.rhs(n, 3, 71)
    X, iters, relres, st = oracle.refine_mixed(A, B, 10, 1e-12)
    assert st == 0
    assert np.all(relres <= 1e-12) and np.all(iters <= 5) and np.all(iters >= 1)
    Xr = np.linalg.solve(A, B)
    assert np.max(np.abs(X - Xr)) / np.max(np.abs(Xr)) <= 1e-12


def test_refine_mixed_not_converged_flag():
    A = inputs.dense(40, 0.9, 3)
    B = inputs.rhs(40, 1, 4)
    _, iters, _, st = oracle.refine_mixed(A, B, 0, 1e-14)
    assert st == 1 and iters[0] == 0


# ---------------------------------------------------------------- batched ---
def test_batched_matches_single():
    ns, offA, A, offB, B = inputs.ragged(12, 1, 30, 0.5, 4)
    LUp, Xp, info = oracle.factor_solve_batched(ns, offA, A, offB, B)
    assert np.all(info == 0)
    for k in range(len(ns)):
        n = int(ns[k])
        Ak = A[offA[k]:offA[k] + n * n].reshape(n, n)
        bk = B[offB[k]:offB[k] + n]
        xk, luk, _ = oracle.solve(Ak, bk)
        assert np.array_equal(Xp[offB[k]:offB[k] + n], xk)
        assert np.array_equal(LUp[offA[k]:offA[k] + n * n].reshape(n, n), luk)
        Xr = np.linalg.solve(Ak, bk)
        assert np.max(np.abs(xk - Xr)) <= 1e-13 * max(1.0, np.abs(Xr).max())


# ------------------------------------------- explicit inverse (Eq. 4-c) -----
@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_inverse_exact_rationals(n):
    pins.pin_inverse_exact(n, 300 + n)


@pytest.mark.parametrize("n,s", [(4, 0.5), (17, 0.5), (40, 0.9)])
def test_inverse_equals_elementary_product(n, s):
    pins.pin_inverse_product_form(n, 310 + n, s)


def test_inverse_special_cases_and_lapack():
    # diagonal: correctly rounded reciprocals; 2 x 2 closed form; LAPACK
    d = np.array([2.0, 3.0, -7.0, 0.5])
    X, _ = oracle.inverse(np.diag(d))
    assert np.array_equal(X, np.diag(1.0 / d))
    a, b, c, e = 1.0, 0.25, -0.3, 1.0
    X, _ = oracle.inverse(np.array([[a, b], [c, e]]))
    det = a * e - b * c
    assert np.max(np.abs(X - np.array([[e, -b], [-c, a]]) / det)) <= 4 * pins.EPS
    for n in (64, 129):
        A = inputs.dense(n, 0.5, 320 + n)
        X, _ = oracle.inverse(A)
        assert np.max(np.abs(X - np.linalg.inv(A))) <= 64 * n * pins.EPS


# ---------------------------------------------------- skyline (profile) -----
@pytest.mark.parametrize("n,ws,wl,pl", [(1, 1, 1, 0.0), (2, 1, 2, 0.5), (40, 3, 30, 0.2), (300, 8, 100, 0.1),
                                        (129, 64, 128, 0.5)])
def test_skyline_matches_dense_oracle_bitwise(n, ws, wl, pl):
    pins.pin_skyline_vs_dense(n, 800 + n, ws, wl, pl)


@pytest.mark.parametrize("n", [2, 50, 1000])
def test_skyline_tridiagonal_closed_form(n):
    pins.pin_skyline_tridiag(n)


def test_skyline_generator_profile_and_dominance():
    f, rp, AL, g, cp, AU = inputs.skyline(500, 16, 200, 0.1, 0.5, 5)
    A = inputs.skyline_to_dense(f, rp, AL, g, cp, AU)
    assert np.all(np.diag(A) == 1.0)
    assert np.max(np.abs(np.abs(A).sum(axis=1) - 1.5)) <= 1e-13
    i, j = np.indices(A.shape)
    assert np.all(A[(j < i) & (j < f[:, None])] == 0.0)
    assert np.all(A[(j > i) & (i < g[None, :])] == 0.0)
    assert f.min() >= 0 and np.all(f <= np.arange(500)) and np.all(g <= np.arange(500))
