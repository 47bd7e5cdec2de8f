"""CPU tests: the pins reject plausible mistakes planted in copies of the oracle.

Each case copies ``oracle/ebv_oracle.c``, changes one expression (a dropped
term, a wrong sign, a transposed operand, an off-by-one bound), builds the copy
into a temporary library and runs the pins against it.  At least one pin must
fail for every mutant; the default oracle build is restored afterwards.
"""
from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest

import oracle
from tests import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "ebv_oracle.c")

MUTANTS = {
    # Eq. 6-c with the wrong sign
    "update_sign": ("ri[j] = ri[j] - l * rk[j];", "ri[j] = ri[j] + l * rk[j];"),
    # Eq. 6-a without the division by the pivot
    "no_pivot_division": ("A[i * lda + k] = A[i * lda + k] / p;", "A[i * lda + k] = A[i * lda + k];"),
    # transposed operand in the rank-1 update (column k instead of row k)
    "transposed_u": ("ri[j] = ri[j] - l * rk[j];", "ri[j] = ri[j] - l * A[j * lda + k];"),
    # update starts one column early (overwrites the multipliers)
    "update_bound": ("for (int64_t j = k + 1; j < n; ++j)\n                ri[j]", "for (int64_t j = k; j < n; ++j)\n                ri[j]"),
    # forward substitution includes the diagonal term
    "forward_bound": ("for (int64_t j = 0; j < i; ++j)\n                s = s - LU[i * lda + j] * B[j * ldb + c];",
                      "for (int64_t j = 0; j <= i; ++j)\n                s = s - LU[i * lda + j] * B[j * ldb + c];"),
    # backward substitution forgets the pivot
    "backward_no_div": ("B[i * ldb + c] = s / LU[i * lda + i];\n        }\n    }\n}\n\n/* Eq. 1",
                        "B[i * ldb + c] = s;\n        }\n    }\n}\n\n/* Eq. 1"),
    # band: the update stops one column short of the upper band edge
    "band_jlast": ("const int64_t jlast = (k + ku < n - 1) ? k + ku : n - 1;",
                   "const int64_t jlast = (k + ku - 1 < n - 1) ? k + ku - 1 : n - 1;"),
    # adjoint: U instead of U^T in the first triangular solve
    "adjoint_transpose": ("s = s - LU[j * lda + i] * Bbar[j * ldb + c];\n            Bbar[i * ldb + c] = s / LU[i * lda + i];",
                          "s = s - LU[i * lda + j] * Bbar[j * ldb + c];\n            Bbar[i * ldb + c] = s / LU[i * lda + i];"),
    # skyline: the envelope test of the columns off by one (skips the edge column)
    "skyline_cols": ("            if (g[j] <= k)\n                cols[nc++] = j;", "            if (g[j] < k)\n                cols[nc++] = j;"),
    # skyline: backward substitution misses the upper envelope's edge
    "skyline_backward": ("                if (g[j] <= i)\n                    s = s - SKY_U(i, j)", "                if (g[j] < i)\n                    s = s - SKY_U(i, j)"),
    # adjoint: Abar without the minus sign
    "adjoint_sign": ("Abar[i * ldabar + j] = -s;", "Abar[i * ldabar + j] = s;"),
}


def _all_pins():
    """Every pin, each reporting pass/fail; returns the list of failures."""
    fails = []
    checks = [
        lambda: pins.pin_minors(4, 101),
        lambda: pins.pin_cramer(3, 201),
        lambda: pins.pin_tridiag(50),
        lambda: pins.pin_invariants(64, 95),
        lambda: pins.pin_solve_numpy(30, 330),
        lambda: pins.pin_band_tridiag(40),
        lambda: pins.pin_band_vs_numpy(60, 5, 7, 61),
        lambda: pins.pin_adjoint(20, 520),
        lambda: pins.pin_skyline_vs_dense(60, 861, 4, 30, 0.2),
        lambda: pins.pin_skyline_tridiag(40),
    ]
    for k, chk in enumerate(checks):
        try:
            chk()
        except (AssertionError, ZeroDivisionError, FloatingPointError):
            fails.append(k)
    return fails


@pytest.fixture(scope="module")
def tmpdir_mod(tmp_path_factory):
    return tmp_path_factory.mktemp("mutants")


def test_pins_pass_on_default_build():
    oracle.use_library(None)
    assert _all_pins() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmpdir_mod):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new, 1)
    c_path = os.path.join(str(tmpdir_mod), f"{name}.c")
    so_path = os.path.join(str(tmpdir_mod), f"lib{name}.so")
    open(c_path, "w").write(mutated)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           c_path, "-o", so_path, "-lm"])
    oracle.use_library(so_path)
    try:
        fails = _all_pins()
    finally:
        oracle.use_library(None)
    assert fails, f"no pin caught mutant {name}"


# ---- the explicit inverse (Eq. 4-c), planted mistakes in its assembly ----
def _inv_forward_only(A):
    lu, _ = oracle.lu_factor(A)
    return oracle.forward(lu, np.eye(len(A))), lu


def _inv_transposed(A):
    X, lu = _ORIG_INVERSE(A)
    return X.T.copy(), lu


def _inv_swapped_order(A):
    # backward substitution first, then forward: U^{-1} applied before L^{-1}
    lu, _ = oracle.lu_factor(A)
    return oracle.forward(lu, oracle.backward(lu, np.eye(len(A)))), lu


_ORIG_INVERSE = oracle.inverse
INVERSE_MUTANTS = {"forward_only": _inv_forward_only, "transposed": _inv_transposed,
                   "swapped_order": _inv_swapped_order}


@pytest.mark.parametrize("name", sorted(INVERSE_MUTANTS))
def test_inverse_pins_reject_mutant(name, monkeypatch):
    monkeypatch.setattr(oracle, "inverse", INVERSE_MUTANTS[name])
    fails = 0
    for chk in (lambda: pins.pin_inverse_exact(4, 304), lambda: pins.pin_inverse_product_form(12, 322)):
        try:
            chk()
        except AssertionError:
            fails += 1
    assert fails, f"no pin caught inverse mutant {name}"
