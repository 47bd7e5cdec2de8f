"""CPU tests of the C ABI (no GPU needed): the library loads, exports every
symbol the header declares, rejects invalid arguments before touching a
device, and its host-side helpers (workspace sizes, EbV batch order, the
ownership map) behave as specified."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_1907_05767_amd import ebv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ebv.LIB_PATH):
        from paper_1907_05767_amd import build
        build.build()
    return ebv.lib()


def test_exports_every_header_symbol(lib):
    names = ebv.header_symbols()
    assert "ebv_lu_factor" in names and "ebv_lu_solve_adjoint" in names
    out = subprocess.check_output(["nm", "-D", "--defined-only", ebv.LIB_PATH], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(lib, n)


def test_status_strings(lib):
    assert lib.ebv_status_string(0) == b"success"
    assert lib.ebv_status_string(-3) == b"invalid argument"
    assert lib.ebv_version() >= 100


def test_argument_validation_without_device(lib):
    # invalid arguments are rejected on the host, before any device query
    assert lib.ebv_lu_factor(7, 4, None, 4, 1, 16, None, None, 0, None) == -1
    assert lib.ebv_lu_factor(0, -1, None, 4, 1, 16, None, None, 0, None) == -2
    assert lib.ebv_lu_factor(0, 4, None, 4, 1, 16, None, None, 0, None) == -3
    assert lib.ebv_lu_factor(0, 4, ctypes.c_void_p(16), 3, 1, 16, None, None, 0, None) == -4
    assert lib.ebv_lu_factor(0, 4, ctypes.c_void_p(16), 4, 2, 15, None, None, 0, None) == -6
    assert lib.ebv_lu_factor(0, 0, None, 1, 1, 0, None, None, 0, None) == 0  # quick return
    assert lib.ebv_lu_solve(0, 4, 2, ctypes.c_void_p(16), 4, ctypes.c_void_p(16), 1, 1, 0, 0, None, 0, None) == -7
    assert lib.ebv_lu_factor_band(10, 3, 2, ctypes.c_void_p(16), 5, None, None) == -5
    assert lib.ebv_lu_factor_band(10, 65, 2, ctypes.c_void_p(16), 80, None, None) == 3  # unsupported
    assert lib.ebv_lu_solve_mixed(4, 1, None, 4, None, 1, None, 1, 3, 1e-12, None, None, None, None, 0, None) == -3
    assert lib.ebv_lu_solve_mixed(4, 1, ctypes.c_void_p(16), 4, ctypes.c_void_p(16), 1, ctypes.c_void_p(16), 1,
                                  -1, 1e-12, None, None, None, None, 0, None) == -9
    # mixed batched requires float64 storage
    assert lib.ebv_lu_factor_batched(1, 1, ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16), 16,
                                     ctypes.c_void_p(16), ctypes.c_void_p(16), 4, None, None, 1, 3, 1e-12, None,
                                     0, None, 0, None) == -1


def test_workspace_sizes(lib):
    # single system: control words (status, two solve-chain words, two per
    # 64-wide block step) rounded up to 256 bytes, then one 64 x 64 tile
    assert lib.ebv_workspace_size(ebv.OP_FACTOR, 0, 4096, 8, 1) == 64 * 64 * 8 + 768
    assert lib.ebv_workspace_size(ebv.OP_FACTOR, 1, 4096, 8, 1) == 64 * 64 * 4 + 768
    assert lib.ebv_workspace_size(ebv.OP_FACTOR, 0, 4096, 8, 3) == 0
    assert lib.ebv_workspace_size(ebv.OP_FACTOR, 0, 64 * 30, 8, 1) == 64 * 64 * 8 + 256  # 4 * 63 bytes
    assert lib.ebv_workspace_size(ebv.OP_FACTOR, 0, 64 * 31, 8, 1) == 64 * 64 * 8 + 512  # 4 * 65 bytes
    # factor_solve: the factor's workspace, then the backward substitution's
    # exchange rows and its two helper workgroups' partial sums per block
    assert lib.ebv_workspace_size(ebv.OP_FACTOR_SOLVE, 0, 4096, 8, 1) == 64 * 64 * 8 + 768 + 3 * 4096 * 16 * 8
    assert lib.ebv_workspace_size(ebv.OP_SOLVE, 0, 100, 8, 1) == 256 + 3 * 128 * 16 * 8
    s = lib.ebv_workspace_size(ebv.OP_SOLVE, 0, 4096, 8, 1)
    assert s >= 4 * 3 and s % 256 == 0
    assert lib.ebv_workspace_size(ebv.OP_SOLVE, 0, 4096, 8, 4) == 0
    m = lib.ebv_workspace_size(ebv.OP_MIXED, 0, 1000, 4, 1)
    assert m >= 4 * 1000 * 1000 + 12 * 1000 * 4
    b = lib.ebv_workspace_size(ebv.OP_BATCHED_MIXED, 0, 10 ** 6, 2000, 7)
    assert b >= 4 * 10 ** 6 + 12 * 2000


def test_batched_order_pairs_largest_with_smallest(lib):
    rng = np.random.default_rng(0)
    ns = rng.integers(16, 513, 101).astype(np.int32)
    order = ebv.batched_order(ns)
    assert sorted(order.tolist()) == list(range(101))  # a permutation
    cost = ns[order].astype(np.int64) ** 3
    srt = np.sort(ns.astype(np.int64) ** 3)[::-1]
    # slots 0, 2, 4, ... walk down from the largest; 1, 3, 5, ... up from the smallest
    assert np.array_equal(cost[0::2], srt[: len(cost[0::2])])
    assert np.array_equal(cost[1::2], srt[::-1][: len(cost[1::2])])
    # every adjacent (largest, smallest) pair sums close to twice the mean cost
    pair = cost[0:100:2] + cost[1:100:2]
    assert pair.max() <= 2 * srt.max() and pair.min() >= srt.min()


PAIRING_TEST = r"""
#include <cstdio>
#include <vector>
#include "ebv_pairing.h"
int main() {
    int bad = 0;
    /* joined vectors have equal length: column v of L below the diagonal has
       n-1-v entries; v and its partner together always have n-1 */
    for (int n = 1; n <= 300; ++n)
        for (int v = 0; v < n; ++v) {
            int p = ebv_partner(v, n);
            if (p < 0 || p >= n || ebv_partner(p, n) != v) bad++;
            if ((n - 1 - v) + (n - 1 - p) != n - 1) bad++;
        }
    /* ebv_batch_slot is a permutation alternating largest / smallest */
    for (int c = 1; c <= 50; ++c) {
        std::vector<int> s(c, 0);
        for (int r = 0; r < c; ++r) s[ebv_batch_slot(r, c)]++;
        for (int i = 0; i < c; ++i) if (s[i] != 1) bad++;
    }
    std::printf("%d\n", bad);
    return bad != 0;
}
"""


def test_pairing_map_invariants(tmp_path):
    src = tmp_path / "pairing_test.cpp"
    src.write_text(PAIRING_TEST)
    exe = tmp_path / "pairing_test"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "paper_1907_05767_amd", "csrc"),
                           str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout


def test_contiguous_ownership_is_worse_than_ebv():
    """Ablation of the ownership map: contiguous row blocks miss the optimal
    per-step maximum on many steps where the EbV fold does not."""
    n, U = 64, 16
    Q = n // U
    miss = 0
    for k in range(n):
        live_total = n - 1 - k
        opt = -(-live_total // U)
        mx = max(sum(1 for q in range(Q) if u * Q + q > k) for u in range(U))
        miss += mx != opt
    assert miss > n // 4
