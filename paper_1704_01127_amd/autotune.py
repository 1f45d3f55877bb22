"""Autotuner: measure, on the GPU, which kernel variant and which cluster size
to use, and write them to a tune table the library loads.

1. Kernel variant of the matrix-core cluster kernels for each (dtype, k,
   number of targets on qubits 0..5): both variants are timed on seeded
   target sets of that class at the benchmark size; the faster one wins.
2. Cost table of the analytic scheduler: microseconds per op by k (k = 0:
   diagonal pass) on an n_ref-qubit state with the chosen variants.
3. Best (scheduler, k_max) per (dtype, size bucket): the supremacy circuit of
   that size is timed with every k_max and both the greedy and the analytic
   scheduler.
4. Cluster size and launch shape of the batched persistent kernel (k_max,
   tiles per work item, padding qubits), timed on the 512-circuit workload.

    python -m paper_1704_01127_amd.autotune --out paper_1704_01127_amd/tune_table.json
    python -m paper_1704_01127_amd.autotune --only-batch --out paper_1704_01127_amd/tune_table.json
"""
from __future__ import annotations

import argparse
import json
import statistics
import sys
import time

import numpy as np

from . import qsim
from .tune import haar

def targets_for(n, k, cls, rng):
    """k targets with exactly `cls` of them (at least 3 for class 3) on qubits 0..5."""
    n_low = cls if cls < 3 else int(rng.integers(3, min(k, 6) + 1))
    n_low = min(n_low, k)
    low = [int(q) for q in rng.choice(6, n_low, replace=False)]
    high = [int(q) for q in rng.choice(range(6, n), k - n_low, replace=False)]
    return sorted(low + high)


def op_ms(state, qubits, mat, reps):
    gates = [("U", tuple(qubits), mat)] * reps
    state.run_circuit(gates, scheduler="per_gate", record_timings=True)
    return statistics.median(r["ms"] for r in state.op_timings() if r["kind"] == "cluster")


def op7_ms(state, qubits, reps, seed):
    """Median time of one 7-qubit cluster: a single gate has at most 6 qubits,
    so two dense gates over the 7 qubits, which a k_max = 7 schedule fuses
    into one cluster (one run per repetition)."""
    g = [("U", tuple(qubits[:6]), haar(6, seed)), ("U", (qubits[5], qubits[6]), haar(2, seed + 1))]
    ts = []
    for _ in range(reps):
        state.run_circuit(g, scheduler="greedy", kmax=7, record_timings=True)
        ts += [r["ms"] for r in state.op_timings() if r["kind"] == "cluster" and r["k"] == 7]
    return statistics.median(ts)


def diag_ms(state, n, reps):
    gates = [("CZ", (2 * i, 2 * i + 1)) for i in range(n // 2)] + [("T", (q,)) for q in range(0, n, 3)]
    ts = []
    for _ in range(reps):
        state.run_circuit(gates, kmax=2, record_timings=True)
        ts += [r["ms"] for r in state.op_timings() if r["kind"] == "diag"]
    return statistics.median(ts)


def tune_variants(n, dt, reps, seed, log, trials=8):
    rng = np.random.default_rng(seed)
    state = qsim.State(n, dt, init="uniform", kmax=6)
    table = {}
    kmin, kmax = (4, 6) if dt == "c64" else (3, 5)  # complex64 k = 6: the fp16-halves kernel's variants
    for k in range(kmin, kmax + 1):
        mat = haar(k, k)
        row = []
        for cls in range(4):
            t = {0: [], 1: []}
            for trial in range(trials):
                qs = targets_for(n, k, cls, rng)
                for v in (0, 1):
                    qsim.set_option(qsim.OPT_CLUSTER_VARIANT, v)
                    t[v].append(op_ms(state, qs, mat, reps))
            qsim.set_option(qsim.OPT_CLUSTER_VARIANT, -1)
            best = 0 if sum(t[0]) <= sum(t[1]) else 1
            row.append(best)
            log("variant %s k=%d class=%d: direct %.3f ms, staged %.3f ms -> %d" %
                (dt, k, cls, statistics.mean(t[0]), statistics.mean(t[1]), best))
        table[str(k)] = row
    del state
    return table


def apply_variants(table_by_dtype):
    L = qsim.lib()
    for dt, rows in table_by_dtype.items():
        code = qsim.C64 if dt == "c64" else qsim.C128
        for k, row in rows.items():
            for cls, v in enumerate(row):
                qsim._check(L.qsim_set_tune_entry(code, int(k), cls, int(v)))


def tune_costs(n, dt, reps, seed, log):
    """us_by_k for k = 0..7 (k = 7: complex64 only; a complex128 table repeats
    its k = 6 entry, which its runs never exceed)."""
    rng = np.random.default_rng(seed + 1)
    state = qsim.State(n, dt, init="uniform", kmax=7)
    us = [diag_ms(state, n, reps) * 1e3]
    for k in range(1, 8):
        if k == 7 and dt != "c64":
            us.append(us[-1])
            break
        ts = []
        for _ in range(3):
            qs = sorted(int(q) for q in rng.choice(n, k, replace=False))
            ts.append(op7_ms(state, qs, reps, k) if k == 7 else op_ms(state, qs, haar(k, k), reps))
        us.append(statistics.mean(ts) * 1e3)
        log("cost %s k=%d: %.1f us" % (dt, k, us[-1]))
    del state
    return us


def tune_kmax(dt, buckets, seed, log):
    from supremacy_inputs import supremacy_circuit
    res = {}
    for n, (R, C) in buckets.items():
        circ = supremacy_circuit(R, C, 25, seed)
        state = qsim.State(circ.n, dt, kmax=7)
        best = None
        for sched in ("greedy", "analytic"):
            for kmax in ((3, 4, 5, 6, 7) if dt == "c64" else (3, 4, 5, 6)):
                opts = dict(kmax=kmax, scheduler=sched, fuse_diag=True, skip_trailing_diag=True,
                            skip_initial_h=True)
                state.init("zero")
                state.run_circuit(circ.gates, **opts)
                state.sync()
                ts = []
                for _ in range(2):
                    state.init("zero")
                    state.sync()
                    t0 = time.perf_counter()
                    st = state.run_circuit(circ.gates, **opts)
                    state.sync()
                    ts.append(time.perf_counter() - t0)
                t = min(ts)
                log("kmax %s n=%d %s kmax=%d: %.2f ms, %d ops" % (dt, circ.n, sched, kmax, t * 1e3, st["n_ops"]))
                if best is None or t < best[0]:
                    best = (t, sched, kmax)
        res[str(circ.n)] = {"scheduler": best[1], "kmax": best[2], "ms": best[0] * 1e3}
        del state
    return res


BATCH_OPTIONS = ("item_tiles", "grid", "pad")


def tune_batch(n_circuits, reps, log):
    """Cluster size and launch shape of the batched persistent kernel, timed
    on the batch workload (n_circuits circuits of 14-24 qubits, depth 10-40):
    k_max (5: every cluster padded to 5 qubits; 6: 6-qubit clusters on the
    fp16 kernel), tiles per work item, and the identity qubits that pad
    clusters to 5 targets (0 lowest, 1 highest). The grid is the kernel's
    occupancy (one work-group per compute unit)."""
    import torch
    from supremacy_inputs import batch_circuit
    circs = [batch_circuit(i) for i in range(n_circuits)]
    opt = {"item_tiles": qsim.OPT_BATCH_ITEM_TILES, "grid": qsim.OPT_BATCH_GRID, "pad": qsim.OPT_BATCH_PAD}
    old = {k: qsim.get_option(v) for k, v in opt.items()}
    best = None
    try:
        for kmax in (5, 6):
            for pad in (0, 1):
                for tiles in (32, 64, 128, 256, 512):
                    cfg = {"item_tiles": tiles, "grid": 0, "pad": pad}
                    for k, v in cfg.items():
                        qsim.set_option(opt[k], v)
                    b = qsim.Batch(circs, kmax=kmax)
                    b.run()
                    t = min(b.run()["run_ms"] for _ in range(reps))
                    log("batch kmax=%d pad=%d item_tiles=%d: %.2f ms" % (kmax, pad, tiles, t))
                    if best is None or t < best[0]:
                        best = (t, dict(cfg, kmax=kmax))
                    del b
                    torch.cuda.empty_cache()
    finally:
        for k, v in old.items():
            qsim.set_option(opt[k], v)
    return dict(best[1], ms=best[0], circuits=n_circuits)


def apply_batch(cfg):
    qsim.set_option(qsim.OPT_BATCH_ITEM_TILES, int(cfg["item_tiles"]))
    qsim.set_option(qsim.OPT_BATCH_GRID, int(cfg["grid"]))
    qsim.set_option(qsim.OPT_BATCH_PAD, int(cfg["pad"]))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--n", type=int, default=28, help="state size of the cost-table measurements")
    ap.add_argument("--n-variant", type=int, default=30, help="state size of the variant measurements")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--dtypes", default="c64,c128")
    ap.add_argument("--no-kmax", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-circuits", type=int, default=512)
    ap.add_argument("--only-batch", action="store_true", help="re-tune the batch launch shape in an existing table")
    ap.add_argument("--only-variants", action="store_true",
                    help="re-tune the cluster kernel variants in an existing table")
    ap.add_argument("--variant-trials", type=int, default=8,
                    help="random target sets per (k, low class) in the variant search")
    ap.add_argument("--buckets", default="20,24,28,30",
                    help="size buckets (qubits) of the (scheduler, k_max) search, from 20, 24, 28, 30")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    import torch

    def log(msg):
        print(msg, flush=True)

    if args.only_batch:
        qsim.load_tuning(args.out)
        with open(args.out) as f:
            out = json.load(f)
        out["batch"] = tune_batch(args.batch_circuits, args.reps, log)
        log("batch best: %s" % json.dumps(out["batch"]))
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
        return out
    if args.only_variants:
        qsim.load_tuning(args.out)
        with open(args.out) as f:
            out = json.load(f)
        for dt in args.dtypes.split(","):
            out["variants"][dt] = tune_variants(args.n_variant if dt == "c64" else args.n_variant - 1, dt,
                                                args.reps, args.seed, log, args.variant_trials)
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
        return out
    out = {"device": torch.cuda.get_device_name(0), "n_ref": args.n, "variants": {}, "cost_us": {},
           "best": {}, "created": time.strftime("%Y-%m-%d %H:%M:%S")}
    dts = args.dtypes.split(",")
    for dt in dts:
        out["variants"][dt] = tune_variants(args.n_variant if dt == "c64" else args.n_variant - 1, dt, args.reps,
                                            args.seed, log, args.variant_trials)
    apply_variants(out["variants"])
    for dt in dts:
        out["cost_us"][dt] = tune_costs(args.n, dt, args.reps, args.seed, log)
        qsim.set_cost_table(qsim.C64 if dt == "c64" else qsim.C128, out["cost_us"][dt], args.n)
    if not args.no_kmax:
        grids = {20: (4, 5), 24: (4, 6), 28: (4, 7), 30: (5, 6)}
        buckets = {int(b): grids[int(b)] for b in args.buckets.split(",")}
        for dt in dts:
            out["best"][dt] = tune_kmax(dt, buckets if dt == "c64" else {k: v for k, v in buckets.items() if k <= 28},
                                        args.seed, log)
    if not args.no_batch:
        out["batch"] = tune_batch(args.batch_circuits, args.reps, log)
        log("batch best: %s" % json.dumps(out["batch"]))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
    return out


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
