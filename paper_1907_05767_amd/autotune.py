"""Autotuner of the library's schedule knobs on the GPU it runs on.

Sweeps, on the benchmark workloads themselves (seeded synthetic inputs):

* the ragged batch (4096 systems, n ~ U{16..512}, one right-hand side), for
  each form -- FP64, FP32, FP32 factor + FP64 refinement -- over workgroups
  per compute unit of the persistent grid and the order in which workgroups
  take the systems (EbV pairing of the costliest with the cheapest remaining
  system, index order, longest first);
* the single dense factor + solve (n = 4096, 8 right-hand sides) over the
  column-class group size G and the trailing-block size above which column
  classes are used;
* the group size G of the FP32 factor, on the mixed-precision dense solve
  (n = 16384, s = 0.9, 4 right-hand sides), set through a one-key table.

Every point is timed with HIP events over repeated calls (inputs restored
outside the timed region) and the fastest setting per form is written as a
tuning table (the key/value format `ebv_load_tuning` reads), with the
measured sweep kept beside it as JSON.  The binding loads the table into its
default handle when present.

Usage (on the GPU):  python -m paper_1907_05767_amd.autotune [--reps R] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TABLE = os.path.join(HERE, "tuning", "mi355x.txt")
SWEEP = os.path.join(HERE, "tuning", "mi355x_sweep.json")


def log(msg: str):
    print(f"[autotune] {msg}", file=sys.stderr, flush=True)


def time_calls(torch, call, restore, reps: int) -> float:
    """Median milliseconds of `call` over `reps` runs, `restore` outside the events."""
    ts = []
    for r in range(reps + 1):
        restore()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        call()
        e1.record()
        torch.cuda.synchronize()
        if r:
            ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def sweep_batched(torch, ebv, inputs, reps: int, wpcs, policies):
    log("ragged batch 4096 x U{16..512}: inputs")
    ns, offA, A, offB, Bv = inputs.ragged(4096, 16, 512, 0.5, 4)
    a64, b64 = torch.from_numpy(A).cuda(), torch.from_numpy(Bv).cuda()
    a32, b32 = a64.float(), b64.float()
    forms = [("f64", ebv.F64, False, a64, b64), ("f32", ebv.F32, False, a32, b32), ("mixed", ebv.F64, True, a64, b64)]
    results, best = {}, {}
    for name, dt, mixed, a0, b0 in forms:
        tA, tB = a0.clone(), b0.clone()
        info = torch.zeros(len(ns), dtype=torch.int32, device="cuda")
        iters = torch.zeros(len(ns), dtype=torch.int32, device="cuda")
        op = ebv.OP_BATCHED_MIXED if mixed else ebv.OP_BATCHED
        ws = None
        results[name] = []
        for pol_name in policies:
            rb = ebv.RaggedBatch(ns, offA, offB, policy=ebv.ORDER_NAMES[pol_name])
            if ws is None:
                ws = ebv.workspace(op, dt, rb.totA, rb.totB, rb.count)
            for wpc in wpcs:
                def call():
                    ebv.factor_solve_batched_(rb, tA, tB, mixed=mixed, info=info, iters=iters, ws=ws,
                                              wg_per_cu=wpc)

                def restore():
                    tA.copy_(a0)
                    tB.copy_(b0)

                ms = time_calls(torch, call, restore, reps)
                if int(info.abs().max().item()) != 0:
                    raise SystemExit(f"batched {name}: nonzero info at wg_per_cu={wpc} order={pol_name}")
                log(f"batched {name}: wg_per_cu={wpc} order={pol_name}: {ms:.3f} ms")
                results[name].append({"wg_per_cu": wpc, "order": pol_name, "ms": ms,
                                      "solves_per_s": len(ns) / (ms * 1e-3)})
        best[name] = min(results[name], key=lambda r: r["ms"])
        del tA, tB, ws
        torch.cuda.empty_cache()
    return results, best


def sweep_dense(torch, ebv, inputs, reps: int, groups, aboves):
    n, nrhs = 4096, 8
    log(f"dense n={n} nrhs={nrhs}: inputs")
    a0 = torch.from_numpy(inputs.dense(n, 0.5, 2)).cuda()
    b0 = torch.from_numpy(inputs.rhs(n, nrhs, 2)).cuda()
    tA, tB = a0.clone(), b0.clone()
    ws = ebv.workspace(ebv.OP_FACTOR_SOLVE, ebv.F64, n, nrhs, 1)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    results = []
    try:
        for g in groups:
            for above in aboves:
                if g == 1 and above != aboves[0]:
                    continue  # G = 1 updates everything every launch: the threshold is moot
                ebv.set_dense_tuning(0, True, g, above)

                def call():
                    ebv.lu_factor_solve_(tA, tB, info=info, ws=ws)

                def restore():
                    tA.copy_(a0)
                    tB.copy_(b0)

                ms = time_calls(torch, call, restore, reps)
                if int(info.item()) != 0:
                    raise SystemExit(f"dense: info {int(info.item())} at G={g} above={above}")
                log(f"dense: defer_group={g} defer_above={above}: {ms:.3f} ms")
                results.append({"defer_group": g, "defer_above": above, "ms": ms})
    finally:
        ebv.set_dense_tuning()
    return results, min(results, key=lambda r: r["ms"])


def sweep_f32_group(torch, ebv, inputs, reps: int, groups):
    n, nrhs = 16384, 4
    log(f"mixed dense n={n} s=0.9 nrhs={nrhs}: inputs")
    A = torch.from_numpy(inputs.dense(n, 0.9, 5)).cuda()
    B = torch.from_numpy(inputs.rhs(n, nrhs, 5)).cuda()
    ws = ebv.workspace(ebv.OP_MIXED, ebv.F64, n, nrhs, 1)
    tmpdir = tempfile.mkdtemp()
    path = os.path.join(tmpdir, "f32_group.txt")

    def set_group(g):
        with open(path, "w") as fh:
            fh.write(f"dense.f32.defer_group {g}\n")
        if ebv.lib().ebv_load_tuning(ebv.handle(), path.encode()) != 0:
            raise SystemExit(f"could not set the FP32 group to {g}")

    results = []
    try:
        for g in groups:
            set_group(g)
            info = []

            def call():
                info.append(ebv.solve_mixed(A, B, ws=ws)[3])

            ms = time_calls(torch, call, lambda: None, reps)
            if any(int(i.item()) != 0 for i in info):
                raise SystemExit(f"mixed dense: nonzero info at FP32 group {g}")
            log(f"mixed dense: f32 defer_group={g}: {ms:.3f} ms")
            results.append({"f32_defer_group": g, "ms": ms})
    finally:
        set_group(4)
        os.remove(path)
        os.rmdir(tmpdir)
    return results, min(results, key=lambda r: r["ms"])


def write_table(best_b, best_d, path: str, best_f32=None):
    lines = ["# Tuning table for MI355X (gfx950), written by paper_1907_05767_amd/autotune.py.",
             "# Fastest measured setting per form; the full sweep is in mi355x_sweep.json.",
             f"dense.small_update_below 0",
             f"dense.lookahead 1",
             f"dense.defer_group {best_d['defer_group']}",
             f"dense.defer_above {best_d['defer_above']}"]
    if best_f32 is not None:
        lines.append(f"dense.f32.defer_group {best_f32['f32_defer_group']}")
    for name in ("f64", "f32", "mixed"):
        b = best_b[name]
        lines.append(f"batched.{name}.wg_per_cu {b['wg_per_cu']}")
        lines.append(f"batched.{name}.order {b['order']}")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--quick", action="store_true", help="fewer points (a smoke run of the tuner)")
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args()

    import torch

    from paper_1907_05767_amd import ebv, inputs

    if not torch.cuda.is_available():
        raise SystemExit("the autotuner needs a GPU")
    t0 = time.time()
    wpcs = (1, 2) if args.quick else (1, 2, 3, 4)
    policies = ("ebv", "index") if args.quick else ("ebv", "index", "longest")
    groups = (3,) if args.quick else (1, 2, 3, 4)
    aboves = (1024,) if args.quick else (512, 1024, 2048)
    bres, bbest = sweep_batched(torch, ebv, inputs, args.reps, wpcs, policies)
    dres, dbest = sweep_dense(torch, ebv, inputs, args.reps, groups, aboves)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    fres, fbest = sweep_f32_group(torch, ebv, inputs, max(3, args.reps // 3), (3, 4) if args.quick else (2, 3, 4))
    write_table(bbest, dbest, args.out, fbest)
    sweep_path = os.path.splitext(args.out)[0] + "_sweep.json"
    with open(sweep_path, "w") as fh:
        json.dump({"device": torch.cuda.get_device_name(0), "reps": args.reps, "seconds": time.time() - t0,
                   "batched": bres, "batched_best": bbest, "dense": dres, "dense_best": dbest,
                   "f32_group": fres, "f32_group_best": fbest}, fh, indent=1)
    log(f"wrote {args.out} and {sweep_path}")
    print(json.dumps({"batched_best": bbest, "dense_best": dbest, "f32_group_best": fbest}))


if __name__ == "__main__":
    main()
