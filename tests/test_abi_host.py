"""CPU tests of the C ABI (no GPU needed): the library loads, exports every
symbol the header declares, rejects invalid arguments before touching a
device, and its host-side helpers (workspace sizes, EbV batch order, the
ownership map) behave as specified."""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys

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


@pytest.fixture(scope="module")
def h(lib):
    hd = ctypes.c_void_p()
    assert lib.ebv_create(ctypes.byref(hd)) == 0 and hd.value
    yield hd
    assert lib.ebv_destroy(hd) == 0


def test_argument_validation_without_device(lib, h):
    # invalid arguments are rejected on the host, before any device query;
    # the handle is argument 1
    P = ctypes.c_void_p(256)
    assert lib.ebv_lu_factor(None, 0, 4, P, 4, 1, 16, None, None, 0, None) == -1
    assert lib.ebv_lu_factor(h, 7, 4, None, 4, 1, 16, None, None, 0, None) == -2
    assert lib.ebv_lu_factor(h, 0, -1, None, 4, 1, 16, None, None, 0, None) == -3
    assert lib.ebv_lu_factor(h, 0, 4, None, 4, 1, 16, None, None, 0, None) == -4
    assert lib.ebv_lu_factor(h, 0, 4, P, 3, 1, 16, None, None, 0, None) == -5
    assert lib.ebv_lu_factor(h, 0, 4, P, 4, 2, 15, None, None, 0, None) == -7
    assert lib.ebv_lu_factor(h, 0, 0, None, 1, 1, 0, None, None, 0, None) == 0  # quick return
    assert lib.ebv_lu_solve(h, 0, 4, 2, P, 4, P, 1, 1, 0, 0, None, None, 0, None) == -8
    assert lib.ebv_lu_factor_solve(h, 0, 4, 2, P, 4, P, 1, None, None, 0, None) == -8
    assert lib.ebv_lu_factor_band(h, 10, 3, 2, P, 5, None, None, 0, None) == -6
    assert lib.ebv_lu_factor_band(h, 10, 65, 2, P, 80, None, None, 0, None) == 3  # unsupported
    assert lib.ebv_lu_solve_band(h, 10, 3, 2, 1, P, 6, P, 0, None, None, 0, None) == -9
    assert lib.ebv_lu_solve_mixed(h, 4, 1, None, 4, None, 1, None, 1, 3, 1e-12, None, None, None, None, 0,
                                  None) == -4
    assert lib.ebv_lu_solve_mixed(h, 4, 1, P, 4, P, 1, P, 1, -1, 1e-12, None, None, None, None, 0, None) == -10
    assert lib.ebv_lu_solve_mixed(h, 4, 65, P, 4, P, 65, P, 65, 3, 1e-12, None, None, None, None, 0, None) == -3
    # mixed batched requires float64 storage
    assert lib.ebv_lu_factor_batched(h, 1, 1, P, P, P, 16, P, P, 4, None, None, 1, 3, 1e-12, None, 0, None, 0,
                                     None) == -2
    assert lib.ebv_lu_factor_batched(h, 0, 1, P, P, P, 16, P, P, 4, None, None, 0, 3, 1e-12, None, 9, None, 0,
                                     None) == -17
    assert lib.ebv_lu_solve_adjoint(h, 0, 4, 1, P, 4, None, 1, P, 1, P, 4, 1, 0, 0, 0, 0, None, None, 0,
                                    None) == -7
    # skyline: a profile entry past the diagonal is rejected before any device query
    import numpy as np
    fbad = np.array([0, 2, 1], dtype=np.int32)
    fok = np.array([0, 0, 1], dtype=np.int32)
    hp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert lib.ebv_lu_factor_skyline(h, 3, hp(fbad), hp(fok), P, P, P, P, P, P, None, None, 0, None) == -3
    assert lib.ebv_lu_factor_skyline(h, 3, hp(fok), hp(fbad), P, P, P, P, P, P, None, None, 0, None) == -3
    # one envelope tile, one inverse pack per block row, then 256 bytes of control words
    assert lib.ebv_skyline_workspace_size(3, hp(fok), hp(fok)) == 2 * 64 * 64 * 8 + 256
    # two block rows reaching back to column 0: tiles (0,0), (1,0), (1,1), (0,1), two packs
    z = np.zeros(65, dtype=np.int32)
    assert lib.ebv_skyline_workspace_size(65, hp(z), hp(z)) == (4 + 2) * 64 * 64 * 8 + 256
    big = np.zeros(16385, dtype=np.int32)
    assert lib.ebv_lu_factor_skyline(h, 16385, hp(big), hp(big), P, P, P, P, P, P, None, None, 0, None) == 3
    # explicit inverse: the result may not overlap the factors
    assert lib.ebv_lu_inverse(h, 0, 4, P, 4, P, 4, None, 0, None) == -6
    assert lib.ebv_lu_inverse(h, 0, 4, P, 3, ctypes.c_void_p(1 << 20), 4, None, 0, None) == -5
    assert lib.ebv_lu_inverse(h, 0, 0, None, 1, None, 1, None, 0, None) == 0
    assert lib.ebv_workspace_size(9, 0, 65, 0, 1) == 2 * 64 * 64 * 8
    # allocation-free factor + solve: oversize n rejected before any device query
    big = lib.ebv_noalloc_max_n() + 1
    assert lib.ebv_lu_factor_solve_noalloc(h, 0, big, 1, P, big, P, 1, None, None) == 8
    assert lib.ebv_lu_factor_solve_noalloc(None, 0, 4, 1, P, 4, P, 1, None, None) == -1
    assert lib.ebv_lu_factor_solve_noalloc(h, 0, 4, 2, P, 3, P, 2, None, None) == -6
    assert lib.ebv_lu_factor_solve_noalloc(h, 0, 0, 1, None, 1, None, 1, None, None) == 0  # quick return
    assert lib.ebv_noalloc_scratch_bytes() == lib.ebv_workspace_size(7, 0, lib.ebv_noalloc_max_n(), 1, 1)
    assert lib.ebv_set_dense_tuning(h, 0, 1, 5, 0) == -4
    assert lib.ebv_set_dense_tuning(None, 0, 1, 3, 0) == -1
    assert lib.ebv_profile_update_enable(h, -1) == -2


def test_handle_lifecycle(lib):
    hd = ctypes.c_void_p()
    assert lib.ebv_create(None) == -1
    assert lib.ebv_create(ctypes.byref(hd)) == 0
    w, o = ctypes.c_int(), ctypes.c_int()
    assert lib.ebv_get_batched_tuning(hd, 0, 0, ctypes.byref(w), ctypes.byref(o)) == 0
    assert (w.value, o.value) == (2, ebv.ORDER_EBV)  # defaults
    assert lib.ebv_set_batched_tuning(hd, 0, 1, 3, ebv.ORDER_LONGEST_FIRST) == 0
    assert lib.ebv_get_batched_tuning(hd, 0, 1, ctypes.byref(w), ctypes.byref(o)) == 0
    assert (w.value, o.value) == (3, ebv.ORDER_LONGEST_FIRST)
    # the forms are independent
    assert lib.ebv_get_batched_tuning(hd, 0, 0, ctypes.byref(w), ctypes.byref(o)) == 0
    assert (w.value, o.value) == (2, ebv.ORDER_EBV)
    assert lib.ebv_set_batched_tuning(hd, 0, 0, 9, 0) == -4
    assert lib.ebv_set_batched_tuning(hd, 0, 0, 2, 3) == -5
    assert lib.ebv_destroy(hd) == 0
    assert lib.ebv_destroy(None) == 0


def test_tuning_table_parsing(lib, tmp_path):
    hd = ctypes.c_void_p()
    assert lib.ebv_create(ctypes.byref(hd)) == 0
    good = tmp_path / "t.txt"
    good.write_text("# comment\n\nbatched.f64.wg_per_cu 4   # trailing comment\n"
                    "batched.mixed.order longest\ndense.defer_group 2\n")
    assert lib.ebv_load_tuning(hd, str(good).encode()) == 0
    w, o = ctypes.c_int(), ctypes.c_int()
    lib.ebv_get_batched_tuning(hd, 0, 0, ctypes.byref(w), ctypes.byref(o))
    assert (w.value, o.value) == (4, ebv.ORDER_EBV)
    lib.ebv_get_batched_tuning(hd, 0, 1, ctypes.byref(w), ctypes.byref(o))
    assert (w.value, o.value) == (2, ebv.ORDER_LONGEST_FIRST)
    # all or nothing: a bad line leaves the previous tuning in place
    for text in ("batched.f64.wg_per_cu 0\n", "batched.f64.wg_per_cu 3 extra\n", "no.such.key 1\n",
                 "batched.f64.order random\n", "batched.f64.wg_per_cu\n"):
        bad = tmp_path / "bad.txt"
        bad.write_text("batched.f64.wg_per_cu 1\n" + text)
        assert lib.ebv_load_tuning(hd, str(bad).encode()) == 6, text
        lib.ebv_get_batched_tuning(hd, 0, 0, ctypes.byref(w), ctypes.byref(o))
        assert w.value == 4, text
    assert lib.ebv_load_tuning(hd, str(tmp_path / "missing.txt").encode()) == 6
    assert lib.ebv_destroy(hd) == 0


def test_committed_tuning_table_loads(lib):
    if not os.path.exists(ebv.TUNING_PATH):
        pytest.skip("no tuning table committed")
    hd = ctypes.c_void_p()
    assert lib.ebv_create(ctypes.byref(hd)) == 0
    assert lib.ebv_load_tuning(hd, ebv.TUNING_PATH.encode()) == 0
    assert lib.ebv_destroy(hd) == 0


def test_tuning_file_from_environment(tmp_path):
    # ebv_create reads EBV_TUNING_FILE; a malformed table makes it fail
    code = ("import ctypes, sys; sys.path.insert(0, %r)\n"
            "from paper_1907_05767_amd import ebv\n"
            "h = ctypes.c_void_p(); rc = ebv.lib().ebv_create(ctypes.byref(h))\n"
            "w, o = ctypes.c_int(), ctypes.c_int()\n"
            "if rc == 0: ebv.lib().ebv_get_batched_tuning(h, 1, 0, ctypes.byref(w), ctypes.byref(o))\n"
            "print(rc, w.value)\n") % ROOT
    good = tmp_path / "g.txt"
    good.write_text("batched.f32.wg_per_cu 5\n")
    bad = tmp_path / "b.txt"
    bad.write_text("batched.f32.wg_per_cu 50\n")
    for path, want in ((good, "0 5"), (bad, "6 0")):
        env = dict(os.environ, EBV_TUNING_FILE=str(path))
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
        assert out.stdout.strip() == want, out.stderr


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
    # band: the factor needs none; the solve one 64 x 64 inverse pack per diagonal tile
    assert lib.ebv_workspace_size(ebv.OP_BAND, 0, 16384, 0, 1) == 0
    assert lib.ebv_workspace_size(ebv.OP_BAND_SOLVE, 0, 16384, 8, 1) == 256 * 4 * 64 * 64 * 8
    assert lib.ebv_workspace_size(ebv.OP_BAND_SOLVE, 0, 65, 1, 1) == 2 * 4 * 64 * 64 * 8


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
    # the other policies
    assert np.array_equal(ebv.batched_order(ns, ebv.ORDER_INDEX), np.arange(101))
    lf = ebv.batched_order(ns, ebv.ORDER_LONGEST_FIRST)
    assert np.all(np.diff(ns[lf].astype(np.int64)) <= 0)
    assert lib.ebv_batched_order(3, 1, ns.ctypes.data_as(ctypes.c_void_p), None) == -1


def _greedy_makespan(cost, order, workers):
    """The persistent kernel's queue: each of `workers` workgroups takes the
    next system in `order` as soon as it is free."""
    import heapq
    free = [0.0] * workers
    for s in order:
        t = heapq.heappop(free)
        heapq.heappush(free, t + cost[s])
    return max(free)


def test_ebv_order_balances_the_persistent_queue(lib):
    """The batch order the library computes, run through a model of the
    persistent kernel's ticket queue on the ragged workload's drawn sizes
    (4096 systems, n ~ U{16..512}, 512 workgroups): the EbV order finishes
    within a few percent of the lower bound max(total / workers, largest
    system) and well ahead of index order.  (Longest-first, the classic LPT
    rule, does as well or better in this model; the autotuner measures both
    on the GPU.)"""
    from paper_1907_05767_amd import inputs
    ns = inputs.ragged_sizes(4096, 16, 512, 4)
    cost = ns.astype(np.float64) ** 3
    W = 512
    bound = max(cost.sum() / W, cost.max())
    m_ebv = _greedy_makespan(cost, ebv.batched_order(ns, ebv.ORDER_EBV), W)
    m_idx = _greedy_makespan(cost, ebv.batched_order(ns, ebv.ORDER_INDEX), W)
    m_lpt = _greedy_makespan(cost, ebv.batched_order(ns, ebv.ORDER_LONGEST_FIRST), W)
    assert m_ebv <= 1.06 * bound
    assert m_idx >= 1.2 * m_ebv
    assert m_lpt <= m_ebv * 1.01


PAIRING_TEST = r"""
#include <cstdio>
#include <vector>
#include "ebv_pairing.h"
int main() {
    int bad = 0;
    /* ebv_batch_slot is a permutation alternating largest / smallest:
       slot r takes sorted index r/2 (even r) or count-1-r/2 (odd r) */
    for (int c = 1; c <= 300; ++c) {
        std::vector<int> s(c, 0);
        for (int r = 0; r < c; ++r) {
            const int k = ebv_batch_slot(r, c);
            if (k < 0 || k >= c) { bad++; continue; }
            s[k]++;
            if (r % 2 == 0 && k != r / 2) bad++;
            if (r % 2 == 1 && k != c - 1 - r / 2) bad++;
        }
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
