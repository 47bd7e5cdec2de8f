"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

`oracle/ebv_oracle.c` is rebuilt with -fsanitize=address,undefined (gcc, no
recovery: the first finding aborts) into a temporary directory, and a child
Python process with the ASan runtime preloaded points the oracle module at
that build and runs every routine on small systems: dense factor, forward
and backward substitution, solve, inverse, band, skyline, adjoint, ragged
batch and the mixed-precision refinement, with sizes around the 64-row
blocks.  The test passes when the child exits cleanly and the sanitizers report nothing.
"""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CHILD = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[2])
import oracle
from paper_1907_05767_amd import inputs

oracle.use_library(sys.argv[1])
for n in (1, 2, 63, 64, 65, 130):
    A = inputs.dense(n, 0.5, n)
    B = inputs.rhs(n, 3, n + 1)
    LU, info = oracle.lu_factor(A)
    assert info == 0
    Y = oracle.forward(LU, B)
    X = oracle.backward(LU, Y)
    X2 = oracle.lu_solve(LU, B)
    X3, LU3, _ = oracle.solve(A, B)
    Ai = oracle.inverse(A)
    W = inputs.rhs(n, 3, n + 2)
    bbar, abar = oracle.lu_solve_adjoint(LU, X, W)
    assert np.allclose(X, X2) and np.allclose(X, X3)
for n, kl, ku in ((1, 0, 0), (70, 3, 5), (130, 64, 64)):
    AB = inputs.band(n, kl, ku, 0.5, n)
    LUB, info = oracle.lu_factor_band(AB, kl, ku)
    assert info == 0
    oracle.lu_solve_band(LUB, kl, ku, inputs.rhs(n, 2, n))
for n in (1, 65, 300):
    f, rp, AL, g, cp, AU = inputs.skyline(n, 8, 100, 0.2, 0.5, n)
    LL, UU, info = oracle.lu_factor_skyline(f, rp, AL, g, cp, AU)
    assert info == 0
    oracle.lu_solve_skyline(f, rp, LL, g, cp, UU, inputs.rhs(n, 2, n))
ns, offA, Ab, offB, Bb = inputs.ragged(12, 1, 140, 0.5, 7)
oracle.factor_solve_batched(ns, offA, Ab, offB, Bb)
A = inputs.dense(100, 0.9, 3)
oracle.refine_mixed(A, inputs.rhs(100, 2, 4))
print("sanitized oracle: all routines ran")
"""


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no AddressSanitizer runtime for gcc")
    so = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp", "-fPIC",
                           "-shared", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           os.path.join(ROOT, "oracle", "ebv_oracle.c"), "-o", so, "-lm"])
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=24"
    env["OMP_NUM_THREADS"] = "2"
    res = subprocess.run([sys.executable, "-c", CHILD, so, ROOT], env=env, capture_output=True, text=True,
                         timeout=600)
    report = res.stdout + res.stderr
    assert res.returncode == 0, report[-4000:]
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert "all routines ran" in res.stdout
