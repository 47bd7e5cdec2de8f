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


def timed(fn, reps: int, torch):
    """Mean ms of fn() over reps, with HIP events on the current stream."""
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for r in range(reps):
        fn(r)
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def secondary(torch, ebv, inputs, oracle, reps: int):
    out = {}
    dev = "cuda"

    # ---- band: n = 16384, kl = ku = 64, 8 RHS
    n, kl, ku, nrhs = 16384, 64, 64, 8
    log("band n=16384 kl=ku=64 nrhs=8")
    AB = inputs.band(n, kl, ku, 0.5, 3)
    B = inputs.rhs(n, nrhs, 3)
    ab0 = torch.from_numpy(AB).to(dev)
    b0 = torch.from_numpy(B).to(dev)
    abs_ = [ab0.clone() for _ in range(reps + 1)]
    bs = [b0.clone() for _ in range(reps + 1)]
    ebv.lu_factor_band_(abs_[0], kl, ku)
    ebv.lu_solve_band_(abs_[0], kl, ku, bs[0])

    def band_step(r):
        ebv.lu_factor_band_(abs_[r + 1], kl, ku)
        ebv.lu_solve_band_(abs_[r + 1], kl, ku, bs[r + 1])

    ms = timed(band_step, reps, torch)
    lub, _ = oracle.lu_factor_band(AB, kl, ku)
    xb = oracle.lu_solve_band(lub, kl, ku, B)
    out["band_n16384_kl64_ku64_nrhs8"] = {
        "ms": ms, "gflops": band_flops(n, kl, ku, nrhs) / ms / 1e6,
        "rel_err_vs_oracle": fwd_err(bs[1].cpu().numpy(), xb)}
    del abs_, bs

    # ---- ragged batch: 4096 systems, n ~ U{16..512}, plain FP64 vs mixed
    log("ragged batch 4096 x U{16..512}")
    ns, offA, A, offB, Bv = inputs.ragged(4096, 16, 512, 0.5, 4)
    rb = ebv.RaggedBatch(ns, offA, offB, device=dev)
    a0 = torch.from_numpy(A).to(dev)
    bb0 = torch.from_numpy(Bv).to(dev)
    flops = float(sum(lu_flops(int(m), 1) for m in ns))
    ws = ebv.workspace(ebv.OP_BATCHED, ebv.F64, rb.totA, rb.totB, rb.count)
    a_cp = [a0.clone() for _ in range(2)]
    b_cp = [bb0.clone() for _ in range(2)]
    ebv.factor_solve_batched_(rb, a_cp[0], b_cp[0], ws=ws)

    def bat_step(r):
        ebv.factor_solve_batched_(rb, a_cp[1], b_cp[1], ws=ws)

    ms_plain = timed(bat_step, 1, torch)
    Xp = b_cp[1].cpu().numpy()
    del a_cp, b_cp
    wsm = ebv.workspace(ebv.OP_BATCHED_MIXED, ebv.F64, rb.totA, rb.totB, rb.count)
    bm = [bb0.clone() for _ in range(reps + 1)]
    ebv.factor_solve_batched_(rb, a0, bm[0], mixed=True, ws=wsm)

    def mix_step(r):
        ebv.factor_solve_batched_(rb, a0, bm[r + 1], mixed=True, ws=wsm)

    ms_mixed = timed(mix_step, reps, torch)
    Xm = bm[1].cpu().numpy()
    rng = np.random.default_rng(0)
    ep = em = 0.0
    for k in rng.choice(len(ns), 16, replace=False):
        m = int(ns[k])
        xk, _, _ = oracle.solve(A[offA[k]:offA[k] + m * m].reshape(m, m), Bv[offB[k]:offB[k] + m])
        ep = max(ep, fwd_err(Xp[offB[k]:offB[k] + m], xk))
        em = max(em, fwd_err(Xm[offB[k]:offB[k] + m], xk))
    bytes_alg = float(sum(16.0 * int(m) * int(m) + 16.0 * int(m) for m in ns))
    out["batched_4096_n16_512"] = {
        "plain_fp64": {"ms": ms_plain, "solves_per_s": 4096 / (ms_plain / 1e3), "gflops": flops / ms_plain / 1e6,
                       "rel_err_vs_oracle_sampled16": ep},
        "mixed_fp32_ir_fp64": {"ms": ms_mixed, "solves_per_s": 4096 / (ms_mixed / 1e3),
                               "gflops_fp64_equiv": flops / ms_mixed / 1e6, "rel_err_vs_oracle_sampled16": em},
        "roofline_ms": max(flops / (PEAK_FP64_TFLOPS * 1e9), bytes_alg / (PEAK_HBM_GBS * 1e6)),
    }
    del a0, bb0, bm, ws, wsm

    # ---- mixed precision dense: n = 16384, row sum 0.9, 4 RHS
    n, nrhs = 16384, 4
    log("mixed precision n=16384 s=0.9 nrhs=4")
    A = inputs.dense(n, 0.9, 5)
    B = inputs.rhs(n, nrhs, 5)
    tA, tB = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    del A
    wsm = ebv.workspace(ebv.OP_MIXED, ebv.F64, n, nrhs, 1)
    res = {}

    def mp_step(r):
        res["out"] = ebv.solve_mixed(tA, tB, tol=1e-12, max_iter=10, ws=wsm)

    mp_step(0)
    ms_mp = timed(mp_step, 2, torch)
    X, iters, relres, _ = res["out"]
    lu64 = tA.clone()

    def fp64_step(r):
        lu64.copy_(tA)
        ebv.lu_factor_(lu64)
        res["x64"] = ebv.lu_solve(lu64, tB)

    ms_64 = timed(fp64_step, 1, torch)
    out["mixed_dense_n16384_s0.9_nrhs4"] = {
        "ms": ms_mp, "fp64_ebv_ms_incl_copy": ms_64, "gflops_fp64_equiv": lu_flops(n, nrhs) / ms_mp / 1e6,
        "iters": iters.cpu().tolist(), "relres": relres.cpu().tolist(),
        "rel_err_vs_fp64_ebv": fwd_err(X.cpu().numpy(), res["x64"].cpu().numpy())}
    del tA, tB, lu64, wsm, res

    # ---- adjoint: 512 systems, n = 1024
    batch, n = 512, 1024
    log("adjoint 512 x 1024")
    A, B = inputs.uniform_batch(batch, n, 0.5, 6)
    W = np.random.default_rng(6).standard_normal((batch, n, 1))
    tA, tB, tW = (torch.from_numpy(v).to(dev) for v in (A, B, W))
    LU = tA.clone()
    X = tB.clone()

    def fwd(r):
        LU.copy_(tA)
        ebv.lu_factor_(LU)
        X.copy_(tB)
        ebv.lu_solve_(LU, X)

    fwd(0)
    ms_f = timed(fwd, 1, torch)
    keep = {}

    def bwd(r):
        keep["g"] = ebv.lu_solve_adjoint(LU, X, tW)

    bwd(0)
    ms_b = timed(bwd, 2, torch)
    bbar, abar = keep["g"]
    xr, lur, _ = oracle.solve(A[0], B[0])
    br, ar = oracle.lu_solve_adjoint(lur, xr, W[0])
    out["adjoint_512_n1024"] = {
        "forward_ms_incl_copies": ms_f, "backward_ms": ms_b,
        "backward_gbs": (batch * (n * n * 8 * 2.0)) / ms_b / 1e6,
        "rel_err_bbar_vs_oracle_sys0": fwd_err(bbar[0].cpu().numpy(), br),
        "rel_err_abar_vs_oracle_sys0": float(np.abs(abar[0].cpu().numpy() - ar).max() / np.abs(ar).max())}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run a plain device copy of 256 MiB (HBM counter calibration)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the k_step HBM traffic summary from two rocprofv3 --pmc runs and exit")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
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
    info = torch.zeros(1, dtype=torch.int32, device=dev)

    def step(i):
        ebv.lu_factor_solve_(As[i], Bs[i], info, ws)

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
    assert int(info.item()) == 0
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
    err = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle factor+solve of the same n=4096 x 8 system")
        t = time.perf_counter()
        X_ref, _, _ = oracle.solve(A, B)
        cs = time.perf_counter() - t
        err = fwd_err(X, X_ref)
        cpu = {"value": flops / cs / 1e9, "unit": "GFLOP/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": "one full factor+solve of the n=4096, 8-RHS system (the whole step), "
                         f"{cs:.1f} s on {cpu_model()}", "seconds": cs}
    sec = None
    if not args.no_secondary:
        del As, Bs
        torch.cuda.empty_cache()
        sec = secondary(torch, ebv, inputs, oracle, reps=3)

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
