"""Benchmark of the EbV LU hot path on one MI355X.

Headline workload: dense FP64 system, n = 4096, 8 right-hand sides, unit
diagonal with off-diagonal row |sum| 0.5 (the paper's Eq. 2 problem class),
factor + forward/backward substitution.  A step is one factor + solve of one
such system; every step works on its own pristine copy of A and B already
resident in HBM, so no restore happens inside the timed region.

Secondary lines (reported inside the same JSON object): the band variant
(n = 16384, kl = ku = 64, 8 RHS), the ragged batch (4096 systems,
n ~ U{16..512}) plain FP64 vs mixed precision, the mixed-precision dense
solve (n = 16384, row sum 0.9, 4 RHS) and the adjoint (512 x n = 1024).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "LU factor+solve GFLOP/s n=4096; batched solves/s at rel err≤1e-12, plain vs MP"
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
COPY_CAL_BYTES = 256 << 20  # plain device copy used to calibrate the HBM byte counters
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_dense_n4096_hbm_traffic.json")
KERNEL_SOURCES = ["paper_1907_05767_amd/csrc/ebv_kernels.hip", "paper_1907_05767_amd/csrc/ebv_device.hpp"]


def kernel_source_hash() -> str:
    """Digest of the kernel sources: stored counter readings apply only to the
    code they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic():
    """HBM bytes per k_step launch from the committed counter summary, or
    None when it is missing or was taken on different kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def summarize_counters(fetch_dir: str, write_dir: str):
    """Build the traffic summary from two rocprofv3 --pmc runs of
    `bench.py --steps 1 --warmup 0 --no-secondary --no-cpu-baseline
    --copy-calibration` (FETCH_SIZE, then WRITE_SIZE): per-dispatch KiB of the
    k_step launches, scaled by what the same counter reads for the plain
    copy of COPY_CAL_BYTES."""
    import csv
    import glob

    def read(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not f:
            raise SystemExit(f"no counter_collection.csv under {d}")
        rows = [r for r in csv.DictReader(open(f[0])) if r.get("Counter_Name") == counter]
        step = [float(r["Counter_Value"]) for r in rows if "k_step<double" in r["Kernel_Name"]]
        copy = [float(r["Counter_Value"]) for r in rows
                if "copyBuffer" in r["Kernel_Name"] or "copy" in r["Kernel_Name"].lower()]
        if not step or not copy:
            raise SystemExit(f"{counter}: no k_step or copy dispatches in {f[0]}")
        cal = max(copy) * 1024.0 / COPY_CAL_BYTES  # counter bytes per true byte
        return sum(step) * 1024.0 / cal, len(step), cal

    rd, nl, cal_r = read(fetch_dir, "FETCH_SIZE")
    wr, nl2, cal_w = read(write_dir, "WRITE_SIZE")
    rec = {
        "kernel": "k_step (dense factor block step, FP64)", "workload": "dense FP64 n=4096, 8 RHS",
        "launches": nl, "read_bytes_per_launch": rd / nl, "write_bytes_per_launch": wr / nl2,
        "bytes_per_launch": rd / nl + wr / nl2,
        "copy_calibration": {"bytes": COPY_CAL_BYTES, "fetch_counter_bytes_per_byte": cal_r,
                             "write_counter_bytes_per_byte": cal_w},
        "kernel_source_sha256": kernel_source_hash(),
    }
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def lu_flops(n: int, nrhs: int) -> float:
    """Factor (2/3 n^3 - n^2/2 - n/6) + solve (2 n^2 per right-hand side)."""
    return (2.0 / 3.0) * n ** 3 - 0.5 * n ** 2 - n / 6.0 + 2.0 * n * n * nrhs


def factor_flops(n: int) -> float:
    return (2.0 / 3.0) * n ** 3 - 0.5 * n ** 2 - n / 6.0


def inverse_flops(n: int) -> float:
    """Factor (2/3 n^3) plus the explicit inverse from the factors (4/3 n^3:
    L^{-1} applied to the identity, n^3 / 3 with its zeros skipped, then U^{-1}
    to the dense result, n^3): 2 n^3 in all, to leading order."""
    return 2.0 * n ** 3


def skyline_flops(f, g, nrhs: int) -> float:
    """Exact flops of the envelope-restricted factor + solve: at step k, one
    division per active row and 2 per (active row, active column) pair; the
    substitutions 2 per envelope entry per right-hand side (plus the
    divisions by the pivots)."""
    f = np.asarray(f, dtype=np.int64)
    g = np.asarray(g, dtype=np.int64)
    n = len(f)
    # active rows at step k: i > k with f_i <= k (a difference array over k)
    ar = np.zeros(n + 1, dtype=np.int64)
    np.add.at(ar, f, 1)
    np.add.at(ar, np.arange(n), -1)
    rows = np.cumsum(ar)[:n]
    ac = np.zeros(n + 1, dtype=np.int64)
    np.add.at(ac, g, 1)
    np.add.at(ac, np.arange(n), -1)
    cols = np.cumsum(ac)[:n]
    factor = float((rows + 2 * rows * cols).sum())
    env = float((np.arange(n) - f).sum() + (np.arange(n) - g).sum())
    return factor + nrhs * (2.0 * env + n)


def band_flops(n: int, kl: int, ku: int, nrhs: int) -> float:
    f = 0.0
    for k in range(n):
        m = n - 1 - k
        a, b = min(kl, m), min(ku, m)
        f += a + 2.0 * a * b
    return f + 2.0 * n * (kl + ku) * nrhs + n * nrhs


def fwd_err(x, ref) -> float:
    x = np.asarray(x, dtype=np.float64).reshape(len(ref), -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(len(ref), -1)
    return float((np.abs(x - ref).max(axis=0) / np.maximum(np.abs(ref).max(axis=0), 1e-300)).max())


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def rep_times(fn, reps: int, torch, prepare=None):
    """Per-rep ms of fn(r) from HIP events on the current stream; prepare(r)
    (a restore of in-place inputs) runs before each rep outside the events.
    Returns {median, p10, p90, mean, reps}."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    torch.cuda.synchronize()
    for r in range(reps):
        if prepare is not None:
            prepare(r)
        ev[r][0].record()
        fn(r)
        ev[r][1].record()
    torch.cuda.synchronize()
    t = np.array([s.elapsed_time(e) for s, e in ev])
    return {"median": float(np.median(t)), "p10": float(np.percentile(t, 10)), "p90": float(np.percentile(t, 90)),
            "mean": float(t.mean()), "reps": reps}


def flops_ms(flops: float, tflops: float) -> float:
    """Milliseconds `flops` take at `tflops` TFLOP/s."""
    return flops / (tflops * 1e12) * 1e3


def bytes_ms(nbytes: float) -> float:
    """Milliseconds `nbytes` take at the HBM peak."""
    return nbytes / (PEAK_HBM_GBS * 1e9) * 1e3


def roofline(bound: str, t_bound_ms: float, ms: float, detail: str, **extra):
    """Fraction of a bound: the bound's time for this workload over the measured time."""
    d = {"bound": bound, "bound_ms": t_bound_ms, "measured_ms": ms, "frac": t_bound_ms / ms if ms else None,
         "basis": detail}
    d.update(extra)
    return d


# ------------------------------------------------------- CPU baselines ---
# Each sample is run in a child process (the oracle's OpenMP thread count is
# fixed at its start): once with every host core and once with one.
CPU_SAMPLES = {
    "dense_n4096": "one factor+solve of a dense n=2048, 8-RHS system of the same generator (seed 2)",
    "dense_n256": "20 factor+solves of the dense n=256, 1-RHS system (seed 1)",
    "band": "one band factor+solve of the whole n=16384, kl=ku=64, 8-RHS system (seed 3)",
    "batched": "factor+solve of the first 256 systems of the ragged batch (seed 4)",
    "mixed": "one FP64 factor+solve of a dense n=2048, row-sum-0.9, 4-RHS system (seed 5)",
    "adjoint": "factor+solve+adjoint of 4 systems of the n=1024 adjoint batch (seed 6)",
    "inverse": "factor + explicit inverse of a dense n=1024 system of the same generator (seed 2)",
    "skyline": "skyline factor+solve of the whole n=16384 profile system, 8 RHS (seed 7)",
}


def cpu_sample(name: str) -> dict:
    """Run one sample on the oracle in this process; returns seconds and work."""
    import oracle
    from paper_1907_05767_amd import inputs
    if name == "dense_n4096":
        A, B = inputs.dense(2048, 0.5, 2), inputs.rhs(2048, 8, 2)
        t = time.perf_counter()
        oracle.solve(A, B)
        return {"seconds": time.perf_counter() - t, "flops": lu_flops(2048, 8)}
    if name == "dense_n256":
        A, B = inputs.dense(256, 0.5, 1), inputs.rhs(256, 1, 1)
        t = time.perf_counter()
        for _ in range(20):
            oracle.solve(A, B)
        return {"seconds": (time.perf_counter() - t) / 20, "flops": lu_flops(256, 1)}
    if name == "band":
        AB, B = inputs.band(16384, 64, 64, 0.5, 3), inputs.rhs(16384, 8, 3)
        t = time.perf_counter()
        lub, _ = oracle.lu_factor_band(AB, 64, 64)
        oracle.lu_solve_band(lub, 64, 64, B)
        return {"seconds": time.perf_counter() - t, "flops": band_flops(16384, 64, 64, 8)}
    if name == "batched":
        ns, offA, A, offB, B = inputs.ragged(4096, 16, 512, 0.5, 4)
        k = 256
        na, nb = int(offA[k]), int(offB[k])
        t = time.perf_counter()
        oracle.factor_solve_batched(ns[:k], offA[:k], A[:na], offB[:k], B[:nb])
        return {"seconds": time.perf_counter() - t, "systems": k,
                "flops": float(sum(lu_flops(int(m), 1) for m in ns[:k]))}
    if name == "mixed":
        A, B = inputs.dense(2048, 0.9, 5), inputs.rhs(2048, 4, 5)
        t = time.perf_counter()
        oracle.solve(A, B)
        return {"seconds": time.perf_counter() - t, "flops": lu_flops(2048, 4)}
    if name == "adjoint":
        A, B = inputs.uniform_batch(4, 1024, 0.5, 6)
        W = np.random.default_rng(6).standard_normal((4, 1024, 1))
        t = time.perf_counter()
        for s in range(4):
            x, lu, _ = oracle.solve(A[s], B[s])
            oracle.lu_solve_adjoint(lu, x, W[s])
        return {"seconds": time.perf_counter() - t, "systems": 4, "flops": 4 * (lu_flops(1024, 1) + 4.0 * 1024 ** 2)}
    if name == "skyline":
        f, rp, AL, g, cp, AU = inputs.skyline(16384, 64, 1024, 0.1, 0.5, 7)
        B = inputs.rhs(16384, 8, 7)
        t = time.perf_counter()
        LL, UU, _ = oracle.lu_factor_skyline(f, rp, AL, g, cp, AU)
        oracle.lu_solve_skyline(f, rp, LL, g, cp, UU, B)
        return {"seconds": time.perf_counter() - t, "flops": skyline_flops(f, g, 8)}
    if name == "inverse":
        A = inputs.dense(1024, 0.5, 2)
        t = time.perf_counter()
        oracle.inverse(A)
        return {"seconds": time.perf_counter() - t, "flops": inverse_flops(1024)}
    raise SystemExit(f"unknown CPU sample {name}")


CPU_BASELINES = True  # --no-cpu-baseline turns every CPU baseline off (profiling runs)


def cpu_baseline(name: str, unit: str):
    """The oracle as it stands, on all host cores and on one core, for one
    bounded sample of a workload; value in `unit` (GFLOP/s or solves/s)."""
    if not CPU_BASELINES:
        return None
    import subprocess
    out = {"kind": "oracle", "unit": unit, "sample": CPU_SAMPLES[name], "cpu": cpu_model(),
           "host_cores": os.cpu_count()}
    for tag, threads in (("all", None), ("one", "1")):
        env = dict(os.environ)
        if threads:
            env["OMP_NUM_THREADS"] = threads
        code = ("import json, sys; sys.path.insert(0, %r); import bench, oracle; r = bench.cpu_sample(%r); "
                "r['threads'] = oracle.num_threads(); print(json.dumps(r))") % (ROOT, name)
        res = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
        if res.returncode != 0:
            raise RuntimeError(f"CPU sample {name} failed: {res.stderr[-400:]}")
        r = json.loads(res.stdout.strip().splitlines()[-1])
        val = (r["systems"] / r["seconds"]) if unit == "solves/s" else r["flops"] / r["seconds"] / 1e9
        if tag == "all":
            out.update({"value": val, "cores": r["threads"], "seconds": r["seconds"]})
        else:
            out.update({"value_one_core": val, "seconds_one_core": r["seconds"]})
    return out


# -------------------------------------------------------- secondary lines ---
def line_dense_n256(torch, ebv, inputs, oracle, reps):
    n, nrhs = 256, 1
    log("dense n=256 nrhs=1")
    A, B = inputs.dense(n, 0.5, 1), inputs.rhs(n, nrhs, 1)
    a0, b0 = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    As = a0.unsqueeze(0).repeat(reps + 3, 1, 1).contiguous()
    Bs = b0.unsqueeze(0).repeat(reps + 3, 1, 1).contiguous()
    ws = ebv.workspace(ebv.OP_FACTOR_SOLVE, ebv.F64, n, nrhs, 1)
    info = torch.zeros(reps + 3, dtype=torch.int32, device="cuda")
    for i in range(3):
        ebv.lu_factor_solve_(As[i], Bs[i], info[i:i + 1], ws)
    t = rep_times(lambda r: ebv.lu_factor_solve_(As[r + 3], Bs[r + 3], info[r + 3:r + 4], ws), reps, torch)
    assert int(info.abs().max().item()) == 0
    X_ref, _, _ = oracle.solve(A, B)
    fl = lu_flops(n, nrhs)
    us = t["median"] * 1e3
    cu_gf = PEAK_FP64_TFLOPS * 1e3 / 256  # one compute unit's FP64 rate, GFLOP/s
    return {"us": us, "us_p10": t["p10"] * 1e3, "us_p90": t["p90"] * 1e3, "reps": reps,
            "gflops": fl / (t["median"] * 1e-3) / 1e9,
            "rel_err_vs_oracle": fwd_err(Bs[-1].cpu().numpy(), X_ref),
            "roofline": roofline("one-CU FP64 (serial chain)", fl / (cu_gf * 1e9) * 1e3, t["median"],
                                 f"{fl:.3e} flop at one compute unit's {cu_gf:.0f} GFLOP/s"),
            "cpu_baseline": cpu_baseline("dense_n256", "GFLOP/s")}


def line_band(torch, ebv, inputs, oracle, reps):
    n, kl, ku, nrhs = 16384, 64, 64, 8
    log("band n=16384 kl=ku=64 nrhs=8")
    AB, B = inputs.band(n, kl, ku, 0.5, 3), inputs.rhs(n, nrhs, 3)
    ab0, b0 = torch.from_numpy(AB).cuda(), torch.from_numpy(B).cuda()
    tab, tb = ab0.clone(), b0.clone()
    wsf = ebv.workspace(ebv.OP_BAND, ebv.F64, n, 0, 1)
    wss = ebv.workspace(ebv.OP_BAND_SOLVE, ebv.F64, n, nrhs, 1)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    sinfo = torch.zeros(1, dtype=torch.int32, device="cuda")

    def restore(r):
        tab.copy_(ab0)
        tb.copy_(b0)

    def step(r):
        ebv.lu_factor_band_(tab, kl, ku, info, wsf)
        ebv.lu_solve_band_(tab, kl, ku, tb, sinfo, wss)

    restore(0)
    step(0)
    t = rep_times(step, reps, torch, prepare=restore)
    assert int(info.item()) == 0 and int(sinfo.item()) == 0
    lub, _ = oracle.lu_factor_band(AB, kl, ku)
    xb = oracle.lu_solve_band(lub, kl, ku, B)
    fl = band_flops(n, kl, ku, nrhs)
    cu_gf = PEAK_FP64_TFLOPS * 1e3 / 256
    byts = 2.0 * AB.nbytes + 2.0 * B.nbytes
    return {"ms": t["median"], "ms_p10": t["p10"], "ms_p90": t["p90"], "reps": reps,
            "gflops": fl / (t["median"] * 1e-3) / 1e9, "rel_err_vs_oracle": fwd_err(tb.cpu().numpy(), xb),
            "roofline": roofline("one-CU FP64 (serial block chain)", fl / (cu_gf * 1e9) * 1e3, t["median"],
                                 f"{fl:.3e} flop at one compute unit's {cu_gf:.0f} GFLOP/s",
                                 hbm_bound_ms=bytes_ms(byts)),
            "cpu_baseline": cpu_baseline("band", "GFLOP/s")}


def line_batched(torch, ebv, inputs, oracle, reps):
    """Plain FP64 and FP32-factor + FP64-refinement forms of the ragged batch,
    each captured once in a HIP graph and timed over `reps` replays (inputs
    restored before each replay, outside the events)."""
    log("ragged batch 4096 x U{16..512}: inputs")
    ns, offA, A, offB, Bv = inputs.ragged(4096, 16, 512, 0.5, 4)
    a0, b0 = torch.from_numpy(A).cuda(), torch.from_numpy(Bv).cuda()
    log("ragged batch: oracle reference of every system")
    _, X_ref, _ = oracle.factor_solve_batched(ns, offA, A, offB, Bv)
    flops = float(sum(lu_flops(int(m), 1) for m in ns))
    ffac = float(sum(factor_flops(int(m)) for m in ns))
    n2 = float((ns.astype(np.float64) ** 2).sum())
    out = {}
    for mixed in (False, True):
        tag = "mixed_fp32_ir_fp64" if mixed else "plain_fp64"
        wpc, pol = ebv.get_batched_tuning(ebv.F64, mixed)
        rb = ebv.RaggedBatch(ns, offA, offB, policy=pol)
        ws = ebv.workspace(ebv.OP_BATCHED_MIXED if mixed else ebv.OP_BATCHED, ebv.F64, rb.totA, rb.totB, rb.count)
        tA, tB = a0.clone(), b0.clone()
        info = torch.zeros(rb.count, dtype=torch.int32, device="cuda")
        iters = torch.zeros(rb.count, dtype=torch.int32, device="cuda")
        call = lambda: ebv.factor_solve_batched_(rb, tA, tB, mixed=mixed, info=info, iters=iters, ws=ws)
        call()
        torch.cuda.synchronize()
        log(f"ragged batch {tag}: graph capture, {reps} replays")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            call()

        def restore(r):
            if not mixed:
                tA.copy_(a0)
            tB.copy_(b0)

        t = rep_times(lambda r: g.replay(), reps, torch, prepare=restore)
        assert int(info.abs().max().item()) == 0
        Xh = tB.cpu().numpy()
        errs = [fwd_err(Xh[offB[k]:offB[k] + ns[k]], X_ref[offB[k]:offB[k] + ns[k]]) for k in range(len(ns))]
        ms = t["median"]
        if mixed:
            it = iters.cpu().numpy()
            # FP32 factor on the FP32 peak, refinement residuals in FP64; bytes:
            # A64 read for the copy and per residual, the float copy written once
            bound_flops = flops_ms(ffac, PEAK_FP32_TFLOPS) + flops_ms((flops - ffac) * (1 + it.mean()), PEAK_FP64_TFLOPS)
            bound_bytes = bytes_ms(8.0 * n2 * (1 + it.mean()) + 4.0 * n2)
            extra = {"iters_min": int(it.min()), "iters_max": int(it.max()), "iters_mean": float(it.mean())}
        else:
            bound_flops = flops_ms(flops, PEAK_FP64_TFLOPS)
            bound_bytes = bytes_ms(16.0 * n2 + 16.0 * float(ns.sum()))
            extra = {}
        tb_ms = max(bound_flops, bound_bytes)
        out[tag] = dict(ms=ms, ms_p10=t["p10"], ms_p90=t["p90"], reps=reps, solves_per_s=4096 / (ms * 1e-3),
                        gflops_fp64_equiv=flops / (ms * 1e-3) / 1e9, rel_err_vs_oracle_max_all_systems=max(errs),
                        wg_per_cu=wpc, order=[k for k, v in ebv.ORDER_NAMES.items() if v == pol][0],
                        roofline=roofline("FP64 MFMA" if not mixed else "FP32 MFMA factor + FP64 refinement",
                                          tb_ms, ms, "max(sum of flops / peak, algorithmic bytes / 8 TB/s) over "
                                          "the drawn sizes", flops_bound_ms=bound_flops,
                                          bytes_bound_ms=bound_bytes), **extra)
        if not mixed:
            # the paper's pairing at batch granularity against the other orders,
            # same grid, each captured and replayed like the tuned form
            abl = {}
            for name, pcode in ebv.ORDER_NAMES.items():
                rbo = ebv.RaggedBatch(ns, offA, offB, policy=pcode)
                go = torch.cuda.CUDAGraph()
                with torch.cuda.graph(go):
                    ebv.factor_solve_batched_(rbo, tA, tB, info=info, ws=ws, wg_per_cu=wpc)
                to = rep_times(lambda r: go.replay(), max(10, reps // 5), torch, prepare=restore)
                assert int(info.abs().max().item()) == 0
                abl[name] = {"ms": to["median"], "solves_per_s": 4096 / (to["median"] * 1e-3)}
                del go
            log("ragged batch order ablation: " + ", ".join(f"{k} {v['ms']:.3f} ms" for k, v in abl.items()))
            out[tag]["order_ablation"] = abl
        del g, tA, tB, ws
        torch.cuda.empty_cache()
    out["cpu_baseline"] = cpu_baseline("batched", "solves/s")
    return out


GOLDEN_MIXED = os.path.join(ROOT, "tests", "golden", "mixed_n16384_s0.9_seed5_X.npy")


def line_mixed(torch, ebv, inputs, oracle, reps):
    n, nrhs = 16384, 4
    log("mixed precision n=16384 s=0.9 nrhs=4")
    A, B = inputs.dense(n, 0.9, 5), inputs.rhs(n, nrhs, 5)
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    del A
    wsm = ebv.workspace(ebv.OP_MIXED, ebv.F64, n, nrhs, 1)
    res = {}

    def mp(r):
        res["out"] = ebv.solve_mixed(tA, tB, tol=1e-12, max_iter=10, ws=wsm)

    mp(0)
    t = rep_times(mp, reps, torch)
    X, iters, ferr, info = res["out"]
    assert int(info.item()) == 0
    Xh = X.cpu().numpy()
    lu64, x64 = tA.clone(), tB.clone()
    ws64 = ebv.workspace(ebv.OP_FACTOR_SOLVE, ebv.F64, n, nrhs, 1)
    info64 = torch.zeros(1, dtype=torch.int32, device="cuda")

    def restore(r):
        lu64.copy_(tA)
        x64.copy_(tB)

    t64 = rep_times(lambda r: ebv.lu_factor_solve_(lu64, x64, info64, ws64), max(2, reps // 2), torch,
                    prepare=restore)
    assert int(info64.item()) == 0
    X64 = x64.cpu().numpy()
    X_ref = np.load(GOLDEN_MIXED) if os.path.exists(GOLDEN_MIXED) else None
    it = iters.cpu().numpy()
    fl = lu_flops(n, nrhs)
    # float factor at the FP32 peak; per correction the float solves read the
    # float factor (4 n^2 bytes) and the residual the double A (8 n^2); the
    # copy reads A once and writes the float factor
    b_ms = (flops_ms(factor_flops(n), PEAK_FP32_TFLOPS)
            + bytes_ms(12.0 * n * n + (1 + it.max()) * 12.0 * n * n))
    return {"ms": t["median"], "ms_p10": t["p10"], "ms_p90": t["p90"], "reps": reps,
            "gflops_fp64_equiv": fl / (t["median"] * 1e-3) / 1e9,
            "fp64_ebv_factor_solve_ms": t64["median"], "speedup_vs_fp64_ebv": t64["median"] / t["median"],
            "iters": it.tolist(), "ferr_bound": ferr.cpu().tolist(),
            "rel_err_vs_oracle": fwd_err(Xh, X_ref) if X_ref is not None else None,
            "rel_err_fp64_ebv_vs_oracle": fwd_err(X64, X_ref) if X_ref is not None else None,
            "rel_err_vs_fp64_ebv": fwd_err(Xh, X64),
            "roofline": roofline("FP32 MFMA factor + HBM refinement", b_ms, t["median"],
                                 "float factor flops / 157.3 TFLOP/s + (copy + per-correction A64 and LU32 "
                                 "reads) / 8 TB/s"),
            "cpu_baseline": cpu_baseline("mixed", "GFLOP/s")}


def line_adjoint(torch, ebv, inputs, oracle, reps):
    batch, n = 512, 1024
    log("adjoint 512 x 1024")
    A, B = inputs.uniform_batch(batch, n, 0.5, 6)
    W = np.random.default_rng(6).standard_normal((batch, n, 1))
    tA, tB, tW = (torch.from_numpy(v).cuda() for v in (A, B, W))
    LU, X = tA.clone(), tB.clone()
    info = torch.zeros(batch, dtype=torch.int32, device="cuda")

    def restore(r):
        LU.copy_(tA)
        X.copy_(tB)

    # factor + both substitutions of every system in one persistent launch
    # (the forward substitution fused into the factorization); LU keeps the
    # factors the backward pass reuses
    rb = ebv.uniform_ragged(batch, n)
    ws = ebv.workspace(ebv.OP_BATCHED, ebv.F64, rb.totA, rb.totB, rb.count)

    def fwd(r):
        ebv.factor_solve_batched_(rb, LU.view(-1), X.view(-1), info=info, ws=ws)

    restore(0)
    fwd(0)
    tf = rep_times(fwd, reps, torch, prepare=restore)
    keep = {}
    binfo = torch.zeros(1, dtype=torch.int32, device="cuda")

    def bwd(r):
        keep["g"] = ebv.lu_solve_adjoint(LU, X, tW, info=binfo)

    bwd(0)
    tb = rep_times(bwd, reps, torch)
    assert int(info.abs().max().item()) == 0 and int(binfo.item()) == 0
    bbar, abar = keep["g"]
    errs = []
    for s in (0, 255, 511):
        xr, lur, _ = oracle.solve(A[s], B[s])
        br, ar = oracle.lu_solve_adjoint(lur, xr, W[s])
        errs.append(max(fwd_err(X[s].cpu().numpy(), xr), fwd_err(bbar[s].cpu().numpy(), br),
                        float(np.linalg.norm(abar[s].cpu().numpy() - ar) / np.linalg.norm(ar))))
    ffl = batch * lu_flops(n, 1)
    bbytes = batch * (8.0 * n * n + 8.0 * n * n)  # read LU, write Abar
    return {"forward_ms": tf["median"], "forward_ms_p10": tf["p10"], "forward_ms_p90": tf["p90"],
            "backward_ms": tb["median"], "backward_ms_p10": tb["p10"], "backward_ms_p90": tb["p90"], "reps": reps,
            "backward_gbs": bbytes / (tb["median"] * 1e-3) / 1e9,
            "rel_err_vs_oracle_sampled3": max(errs),
            "roofline_forward": roofline("FP64 MFMA", flops_ms(ffl, PEAK_FP64_TFLOPS), tf["median"],
                                         "factor+solve flops / 78.6 TFLOP/s"),
            "roofline_backward": roofline("HBM", bytes_ms(bbytes), tb["median"],
                                          "read LU + write Abar (16 n^2 bytes per system) / 8 TB/s"),
            "cpu_baseline": cpu_baseline("adjoint", "solves/s")}


def line_inverse(torch, ebv, inputs, oracle, reps):
    """Factor + explicit inverse (Eq. 4-c's product form) of the n = 4096
    headline matrix; parity on sampled columns against the oracle."""
    n = 4096
    log("explicit inverse n=4096")
    A = inputs.dense(n, 0.5, 2)
    a0 = torch.from_numpy(A).cuda()
    tA = a0.clone()
    X = torch.empty_like(a0)
    wsf = ebv.workspace(ebv.OP_FACTOR, ebv.F64, n, 0, 1)
    wsi = ebv.workspace(ebv.OP_INVERSE, ebv.F64, n, 0, 1)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")

    def restore(r):
        tA.copy_(a0)

    def fi(r):
        ebv.lu_factor_(tA, info, wsf)
        ebv.lu_inverse(tA, X, wsi)

    def inv_only(r):
        ebv.lu_inverse(tA, X, wsi)

    t = rep_times(fi, reps, torch, prepare=restore)
    ti = rep_times(inv_only, reps, torch)
    assert int(info.item()) == 0
    Xh = X.cpu().numpy()
    LU_ref, _ = oracle.lu_factor(A)
    cols = np.array([0, 1, 777, 2048, 4095])
    E = np.zeros((n, len(cols)))
    E[cols, np.arange(len(cols))] = 1.0
    err = float(np.max(np.abs(Xh[:, cols] - oracle.lu_solve(LU_ref, E))) / np.max(np.abs(Xh[:, cols])))
    fl = inverse_flops(n)
    return {"ms": t["median"], "ms_p10": t["p10"], "ms_p90": t["p90"], "reps": reps,
            "inverse_only_ms": ti["median"], "gflops": fl / (t["median"] * 1e-3) / 1e9,
            "rel_err_vs_oracle_sampled_columns": err,
            "roofline": roofline("FP64 MFMA", flops_ms(fl, PEAK_FP64_TFLOPS), t["median"],
                                 "2 n^3 flop (factor 2/3 n^3 + inverse 4/3 n^3) / 78.6 TFLOP/s"),
            "cpu_baseline": cpu_baseline("inverse", "GFLOP/s")}


def line_transfer(torch, ebv, inputs, oracle, reps):
    """Host<->device transfers measured the way the paper's Table 3 reports
    them (to the GPU: the system A and b; from the GPU: x), over pinned host
    memory, and the transfer pipeline's overlap on 8 host-resident
    n = 4096, 8-RHS systems: the same work run serially (upload, factor +
    solve, download, one system after the other) against the pipeline."""
    table = []
    for n in (500, 1000, 2000, 4000, 8000, 16000):
        log(f"transfers n={n}")
        ha = torch.empty((n, n), dtype=torch.float64).pin_memory()
        hb = torch.empty((n, 1), dtype=torch.float64).pin_memory()
        hx = torch.empty((n, 1), dtype=torch.float64).pin_memory()
        da = torch.empty((n, n), dtype=torch.float64, device="cuda")
        db = torch.empty((n, 1), dtype=torch.float64, device="cuda")
        tin = rep_times(lambda r: (da.copy_(ha, non_blocking=True), db.copy_(hb, non_blocking=True)), 5, torch)
        tout = rep_times(lambda r: hx.copy_(db, non_blocking=True), 5, torch)
        table.append({"n": n, "to_gpu_s": tin["median"] * 1e-3, "from_gpu_s": tout["median"] * 1e-3,
                      "to_gpu_gbs": (n * n + n) * 8 / (tin["median"] * 1e-3) / 1e9})
        del ha, hb, hx, da, db
    torch.cuda.empty_cache()
    n, nrhs, count = 4096, 8, 8
    log(f"transfer pipeline: {count} systems n={n} nrhs={nrhs}")
    A, B = inputs.dense(n, 0.5, 2), inputs.rhs(n, nrhs, 2)
    ah = [torch.from_numpy(A).pin_memory() for _ in range(count)]
    bh = [torch.from_numpy(B).pin_memory() for _ in range(count)]
    a_pristine, b_pristine = torch.from_numpy(A), torch.from_numpy(B)

    def restore():
        for s in range(count):
            ah[s].copy_(a_pristine)
            bh[s].copy_(b_pristine)

    info = torch.zeros(count, dtype=torch.int32, device="cuda")
    da = torch.empty((n, n), dtype=torch.float64, device="cuda")
    db = torch.empty((n, nrhs), dtype=torch.float64, device="cuda")
    ws = ebv.workspace(ebv.OP_FACTOR_SOLVE, ebv.F64, n, nrhs, 1)

    def serial(r):
        for s in range(count):
            da.copy_(ah[s], non_blocking=True)
            db.copy_(bh[s], non_blocking=True)
            ebv.lu_factor_solve_(da, db, info[s:s + 1], ws)
            bh[s].copy_(db, non_blocking=True)

    pipe = ebv.Pipeline(n, nrhs)
    ts, tp = [], []
    for r in range(6):  # the first pair warms up (streams, events, first copies)
        restore()
        a = rep_times(serial, 1, torch)["median"]
        restore()
        b = rep_times(lambda r: pipe.run(ah, bh, info), 1, torch)["median"]
        if r:
            ts.append(a)
            tp.append(b)
    assert int(info.abs().max().item()) == 0
    X_ref, _, _ = oracle.solve(A, B)
    err = max(fwd_err(bh[0].numpy(), X_ref), fwd_err(bh[-1].numpy(), X_ref))
    ms_s, ms_p = float(np.median(ts)), float(np.median(tp))
    return {"table3": table,
            "pipeline": {"systems": count, "n": n, "nrhs": nrhs, "reps": len(tp), "serial_ms": ms_s,
                         "pipelined_ms": ms_p, "serial_ms_min": float(min(ts)), "pipelined_ms_min": float(min(tp)),
                         "overlap_speedup": ms_s / ms_p, "per_system_ms": ms_p / count,
                         "gflops_pcie_inclusive": count * lu_flops(n, nrhs) / (ms_p * 1e-3) / 1e9,
                         "rel_err_vs_oracle": err}}


def line_skyline(torch, ebv, inputs, oracle, reps):
    """Skyline (profile) factor + solve, the stand-in for the paper's sparse
    systems (Table 1): n = 16384, widths U{1..64} with U{64..1024} for one
    row / column in ten, 8 RHS; parity on the whole result."""
    n, nrhs = 16384, 8
    log("skyline n=16384 nrhs=8")
    f, rp, AL, g, cp, AU = inputs.skyline(n, 64, 1024, 0.1, 0.5, 7)
    B = inputs.rhs(n, nrhs, 7)
    sk = ebv.Skyline(f, rp, AL, g, cp, AU)
    al0, au0 = sk.AL.clone(), sk.AU.clone()
    b0 = torch.from_numpy(B).cuda()
    tb = b0.clone()
    info = torch.zeros(1, dtype=torch.int32, device="cuda")

    def restore(r):
        sk.AL.copy_(al0)
        sk.AU.copy_(au0)
        tb.copy_(b0)

    def step(r):
        sk.factor_(info)
        sk.solve_(tb)

    t = rep_times(step, reps, torch, prepare=restore)
    assert int(info.item()) == 0
    LL, UU, _ = oracle.lu_factor_skyline(f, rp, AL, g, cp, AU)
    X_ref = oracle.lu_solve_skyline(f, rp, LL, g, cp, UU, B)
    fl = skyline_flops(f, g, nrhs)
    cu_gf = PEAK_FP64_TFLOPS * 1e3 / 256
    env = int(rp[-1] + cp[-1])
    return {"ms": t["median"], "ms_p10": t["p10"], "ms_p90": t["p90"], "reps": reps,
            "gflops": fl / (t["median"] * 1e-3) / 1e9, "envelope_entries": env,
            "envelope_tiles_mb": sk.ws.numel() / 1e6,
            "rel_err_vs_oracle": fwd_err(tb.cpu().numpy(), X_ref),
            "roofline": roofline("one-CU FP64 (serial block chain)", fl / (cu_gf * 1e9) * 1e3, t["median"],
                                 f"{fl:.3e} flop (exact, envelope-restricted) at one compute unit's {cu_gf:.0f} GFLOP/s"),
            "cpu_baseline": cpu_baseline("skyline", "GFLOP/s")}


def summarize_trace(trace_dir: str, workload: str, command: str, out_path: str):
    """Write a kernel-trace summary (markdown) from a rocprofv3
    --kernel-trace --stats --output-format csv run: per kernel, calls and
    average / min / max / total duration."""
    import csv
    import glob
    f = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not f:
        raise SystemExit(f"no kernel_stats.csv under {trace_dir}")
    rows = list(csv.DictReader(open(f[0])))
    lines = [f"# Kernel trace: {workload}", "",
             "Command (from the repository root, on the MI355X):", "", "```", command, "```", "",
             "| kernel | calls | avg us | min us | max us | total ms | % |", "|---|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"]
        short = name.split("(")[0].replace("void ", "")
        lines.append(f"| `{short}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.1f} |")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {out_path}")


def secondary(torch, ebv, inputs, oracle, reps: int, only=None):
    out = {}
    # the transfer pipeline first: its three streams overlap only on distinct
    # hardware queues, which HIP assigns to streams round-robin (four per
    # process by default), and the graph captures of the batched line create
    # streams of their own
    for name, fn, r in (("transfers_table3", line_transfer, reps),
                        ("dense_n256_nrhs1", line_dense_n256, max(reps, 100)),
                        ("band_n16384_kl64_ku64_nrhs8", line_band, reps),
                        ("batched_4096_n16_512", line_batched, max(reps, 100)),
                        ("mixed_dense_n16384_s0.9_nrhs4", line_mixed, max(5, reps // 4)),
                        ("adjoint_512_n1024", line_adjoint, max(5, reps // 4)),
                        ("inverse_n4096", line_inverse, max(5, reps // 4)),
                        ("skyline_n16384_nrhs8", line_skyline, max(5, reps // 4))):
        if only is not None and name != only:
            continue
        out[name] = fn(torch, ebv, inputs, oracle, r)
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--secondary-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run a plain device copy of 256 MiB (HBM counter calibration)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the k_step HBM traffic summary from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--summarize-trace", nargs=4, metavar=("TRACE_DIR", "WORKLOAD", "COMMAND", "OUT"),
                    help="write a kernel-trace summary (markdown) from a rocprofv3 --stats csv run and exit")
    ap.add_argument("--line", default=None,
                    help="run only this secondary line (no headline) and print its JSON; for profiling")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the EbV LU path in this repository runs on a single "
              "MI355X and has no multi-GPU code (how it would shard is described in DESIGN.md). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    import oracle
    from paper_1907_05767_amd import ebv, inputs

    global CPU_BASELINES
    CPU_BASELINES = not args.no_cpu_baseline
    if args.line:
        res = secondary(torch, ebv, inputs, oracle, args.secondary_reps, only=args.line)
        if not res:
            raise SystemExit(f"unknown line {args.line}")
        print(json.dumps(res))
        return

    n, nrhs = 4096, 8
    K, W = args.steps, args.warmup
    log(f"dense n={n} nrhs={nrhs} steps={K} warmup={W}")
    A = inputs.dense(n, 0.5, 2)
    B = inputs.rhs(n, nrhs, 2)
    dev = torch.device("cuda:0")
    a0 = torch.from_numpy(A).to(dev)
    b0 = torch.from_numpy(B).to(dev)
    # pristine copies: W warm-up steps, K timed steps, K instrumented steps
    As = a0.unsqueeze(0).repeat(2 * K + W, 1, 1).contiguous()
    Bs = b0.unsqueeze(0).repeat(2 * K + W, 1, 1).contiguous()
    ws = ebv.workspace(ebv.OP_FACTOR_SOLVE, ebv.F64, n, nrhs, 1)
    # one info word per step: each reports a zero pivot or a bounded wait
    # that gave up (-status) in that step
    info = torch.zeros(2 * K + W, dtype=torch.int32, device=dev)

    def step(i):
        ebv.lu_factor_solve_(As[i], Bs[i], info[i:i + 1], ws)

    for i in range(W):
        step(i)
    torch.cuda.synchronize()
    # timed pass: nothing but the steps between the two synchronizations
    t0 = time.perf_counter()
    for i in range(W, W + K):
        step(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # instrumented pass over K more pristine copies: every block-step launch
    # bracketed by HIP events on its stream (the events add a few microseconds
    # per launch, so they stay out of the timed pass)
    nupd = (n + 63) // 64
    ebv.profile_update_enable(K * nupd)
    torch.cuda.synchronize()
    for i in range(W + K, W + 2 * K):
        step(i)
    torch.cuda.synchronize()
    upd_ms, upd_launches, upd_flops = ebv.profile_update_read()
    ebv.profile_update_enable(0)
    ms_step = wall * 1e3 / K
    flops = lu_flops(n, nrhs)
    value = flops / (ms_step / 1e3) / 1e9
    bad = int((info != 0).sum().item())
    assert bad == 0, f"{bad} steps reported a nonzero info"
    assert ebv.workspace_status(ws) == 0
    X = Bs[W + K - 1].cpu().numpy()

    if args.copy_calibration:
        src = torch.empty(COPY_CAL_BYTES // 8, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    achieved = upd_flops / (upd_ms / 1e3) / 1e12 if upd_ms > 0 else None
    roof = {"kernel": "k_step (block step: rank-64 trailing update on FP64 MFMA 16x16x4 + diagonal tile + panel)",
            "bound": "mfma",
            "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": (achieved / PEAK_FP64_TFLOPS) if achieved else None, "traffic": stored_traffic(),
            "launches_per_step": upd_launches / K if K else None,
            "avg_launch_us": upd_ms * 1e3 / upd_launches if upd_launches else None,
            "flops_per_launch_avg": upd_flops / upd_launches if upd_launches else None}

    cpu = None
    log("oracle factor+solve of the same n=4096 x 8 system (parity of the timed step)")
    t = time.perf_counter()
    X_ref, _, _ = oracle.solve(A, B)
    cs = time.perf_counter() - t
    err = fwd_err(X, X_ref)
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on all host cores and on one core")
        cpu = cpu_baseline("dense_n4096", "GFLOP/s")
        cpu["full_step_seconds_all_cores"] = cs
        cpu["full_step_value_all_cores"] = flops / cs / 1e9
    sec = None
    if not args.no_secondary:
        del As, Bs
        torch.cuda.empty_cache()
        sec = secondary(torch, ebv, inputs, oracle, reps=args.secondary_reps)

    rec = {
        "metric": METRIC, "value": value, "unit": "GFLOP/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "dense FP64 n=4096, 8 RHS, unit diagonal, off-diagonal row |sum| 0.5, seed 2; "
                               "EbV factor + forward/backward substitution (ebv_lu_factor_solve)",
                   "n": n, "nrhs": nrhs, "flops_per_step": flops, "parallelism": "single GPU"},
        "rel_err_vs_oracle": err,
        "fraction_of_fp64_peak_whole_step": value / 1e3 / PEAK_FP64_TFLOPS,
        "roofline": roof,
        "cpu_baseline": cpu,
        "secondary": sec,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
