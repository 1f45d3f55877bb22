"""Kernel microbenchmarks on the GPU (the measurements the autotuner uses).

For every cluster size k and target-qubit pattern, one dense k-qubit gate is
applied to an n-qubit state through qsim_run_circuit with per-launch HIP
event timing; the cluster kernel's time gives its HBM bandwidth (one read and
one write of the state, the algorithmic traffic of an in-place cluster) and
its FLOP rate (2^n (8 2^k - 2) per launch). A device-to-device copy of the
same size is timed as the achievable-bandwidth reference, and the diagonal
pass and per-gate kernels are timed alongside.

    python -m paper_1704_01127_amd.tune --n 30 --dtype c64 --out tune.json
"""
from __future__ import annotations

import argparse
import json
import statistics
import sys
import time

import numpy as np

from . import qsim


def patterns(n: int, k: int, rng) -> dict:
    """Target sets: low bits, high bits, spread, and clusters as the scheduler
    forms them on a 2D grid circuit (a mix of low and high qubits)."""
    out = {"low": list(range(k)), "high": list(range(n - k, n)),
           "spread": sorted(set(int(round(i * (n - 1) / max(1, k - 1))) for i in range(k)))}
    if len(out["spread"]) < k:
        out["spread"] = list(range(0, 2 * k, 2))
    out["mid"] = list(range(n // 2 - k // 2, n // 2 - k // 2 + k))
    out["random"] = sorted(int(q) for q in rng.choice(n, k, replace=False))
    out["nolow"] = sorted(int(q) for q in rng.choice(range(3, n), k, replace=False))
    return out


def haar(k: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    d = 2 ** k
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]


def time_cluster(state, qubits, mat, reps):
    gates = [("U", tuple(qubits), mat)] * reps
    state.run_circuit(gates, kmax=len(qubits), scheduler="per_gate", record_timings=True)
    recs = [r for r in state.op_timings() if r["kind"] == "cluster"]
    return [r["ms"] for r in recs]


def time_gates(state, gate, reps):
    state.run_circuit([gate] * reps, scheduler="per_gate", record_timings=True)
    return [r["ms"] for r in state.op_timings() if r["kind"] != "build"]


def copy_bandwidth(state, reps):
    import torch
    a = state.amps
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
    for i in range(reps):
        ev[2 * i].record()
        b.copy_(a)
        ev[2 * i + 1].record()
    torch.cuda.synchronize()
    ms = [ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(reps)]
    del b
    return ms


def circuit_ops(args):
    """Per-op times of one supremacy circuit run (the ops the scheduler forms)."""
    from supremacy_inputs import supremacy_circuit
    R, C, depth = (int(x) for x in args.circuit.split("x"))
    circ = supremacy_circuit(R, C, depth, args.seed)
    n = circ.n
    amp = 8 if args.dtype == "c64" else 16
    state = qsim.State(n, args.dtype, kmax=6)
    opts = dict(kmax=args.kmax, fuse_diag=bool(args.fuse_diag), skip_trailing_diag=True, skip_initial_h=True)
    state.run_circuit(circ.gates, **opts)
    state.run_circuit(circ.gates, record_timings=True, **opts)
    recs = state.op_timings()
    total = sum(r["ms"] for r in recs)
    for r in recs:
        gbs = 2 * 2 ** n * amp / r["ms"] / 1e6 if r["kind"] != "build" else 0.0
        print("%-8s k=%d epi=%d %-24s %8.3f ms %7.0f GB/s" % (r["kind"], r["k"], r["epi"], r["qubits"], r["ms"], gbs),
              flush=True)
    print("total GPU time %.3f ms over %d launches" % (total, len(recs)), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"circuit": args.circuit, "n": n, "dtype": args.dtype, "opts": opts, "ops": recs}, f, indent=1)
    return recs


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--dtype", default="c64", choices=["c64", "c128"])
    ap.add_argument("--ks", default="1,2,3,4,5,6")
    ap.add_argument("--patterns", default="low,high,spread,mid,random,nolow")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None)
    ap.add_argument("--no-other", action="store_true", help="skip copy / diagonal / per-gate timings")
    ap.add_argument("--circuit", default=None,
                    help="RxCxDEPTH: time every op of that supremacy circuit instead (e.g. 5x6x25)")
    ap.add_argument("--kmax", type=int, default=5)
    ap.add_argument("--fuse-diag", type=int, default=1)
    ap.add_argument("--variant", type=int, default=None, help="matrix-core cluster kernel variant (0 or 1)")
    ap.add_argument("--k6-kernel", type=int, default=None,
                    help="6-qubit complex64 kernel: 0 fp32 real-split, 1 fp32 three-product, 2 fp16 halves")
    args = ap.parse_args(argv)
    if args.variant is not None:
        qsim.set_option(qsim.OPT_CLUSTER_VARIANT, args.variant)
    if args.k6_kernel is not None:
        qsim.set_option(qsim.OPT_K6_KERNEL, args.k6_kernel)

    import torch  # noqa: F401

    if args.circuit:
        return circuit_ops(args)

    n = args.n
    amp = 8 if args.dtype == "c64" else 16
    nbytes = 2 * 2 ** n * amp
    state = qsim.State(n, args.dtype, init="uniform", kmax=6)
    rng = np.random.default_rng(args.seed)
    res = {"n": n, "dtype": args.dtype, "bytes_per_pass": nbytes, "clusters": [], "other": {}}
    if not args.no_other:
        ms = copy_bandwidth(state, args.reps)
        res["other"]["device_copy"] = {"ms": statistics.median(ms), "GBs": nbytes / statistics.median(ms) / 1e6}
        for name, gate in (("gate1q_H_q0", ("H", (0,))), ("gate1q_H_q%d" % (n - 1), ("H", (n - 1,))),
                           ("gate1q_H_q7", ("H", (7,))), ("phase_T_q3", ("T", (3,))), ("cz_2_9", ("CZ", (2, 9)))):
            ms = time_gates(state, gate, args.reps)
            res["other"][name] = {"ms": statistics.median(ms), "GBs_full_pass": nbytes / statistics.median(ms) / 1e6}
        # diagonal pass with a CZ layer and phases
        pairs = [(2 * i, 2 * i + 1) for i in range(n // 2)]
        t0 = time.perf_counter()
        state.run_circuit([("CZ", p) for p in pairs] + [("T", (q,)) for q in range(0, n, 3)],
                          kmax=2, record_timings=True)
        ms = [r["ms"] for r in state.op_timings() if r["kind"] == "diag"]
        if ms:
            res["other"]["diag_pass"] = {"ms": statistics.median(ms), "GBs": nbytes / statistics.median(ms) / 1e6}
    for k in [int(x) for x in args.ks.split(",")]:
        pats = patterns(n, k, rng)
        mat = haar(k, k)
        for pname in args.patterns.split(","):
            qs = pats[pname]
            ms = time_cluster(state, qs, mat, args.reps)
            med = statistics.median(ms)
            flops = 2 ** n * (8 * 2 ** k - 2)
            row = {"k": k, "pattern": pname, "qubits": qs, "ms": med, "ms_min": min(ms),
                   "GBs": nbytes / med / 1e6, "TFLOPs": flops / med / 1e9}
            res["clusters"].append(row)
            print("k=%d %-7s %-28s %8.3f ms %7.0f GB/s %6.1f TF/s" % (k, pname, qs, med, row["GBs"],
                                                                       row["TFLOPs"]), flush=True)
    for name, v in res["other"].items():
        print("%-20s %8.3f ms %7.0f GB/s" % (name, v["ms"], v.get("GBs", v.get("GBs_full_pass"))), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
    return res


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
