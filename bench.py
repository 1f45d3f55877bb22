#!/usr/bin/env python3
"""Time-to-solution of a 30-qubit depth-25 random supremacy circuit on one
MI355X: float32 fused clusters versus float64 one gate at a time.

One step = initialise |0...0>, run the whole circuit through the library
(scheduling, float64 cluster-matrix build on the GPU, cluster / diagonal
kernels), then the float64 reductions (norm, sum p^2, entropy) that give the
output distribution's statistics. Inputs are resident in HBM; the timed
region is bracketed by device synchronisation.

Prints one JSON line. `value` is the float32 fused time-to-solution in
seconds. `roofline` is measured live from HIP events around every launch of
the timed steps; `cpu_baseline` times the CPU oracle on a bounded sample of
the same circuit and scales it to the whole circuit.
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "30q depth-25 time-to-solution + % HBM peak, FP32-fused vs FP64 per-gate"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3   # dense FP32 matrix cores
FP64_PEAK_TFLOPS = 78.6


def kernel_source_hash() -> str:
    with open(os.path.join(ROOT, "paper_1704_01127_amd", "csrc", "qsim_kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def kernel_name(rec, k6_kernel=2, pair_tile=11) -> str:
    """Name (as rocprofv3 reports it) of the float cluster kernel a launch used."""
    k, lowt = rec["k"], rec["qubits"][0] == 0
    if rec["kind"] == "pair":
        q = set(rec["qubits"])
        ten = pair_tile == 10 and (0 in q or len(q) < 10)  # the 10-qubit tile holds qubit 0
        return "k_cluster_f32_pair10<12>" if ten else "k_cluster_f32_multi<2, 8>"
    if not rec.get("mfma"):
        return "k_cluster_valu<float, %d>" % k
    b = lambda x: "true" if x else "false"  # noqa: E731
    if k == 6 and k6_kernel in (1, 2):
        if k6_kernel == 2 and rec.get("staged"):
            return "k_cluster_f32_split6s<%s>" % b(lowt)
        if k6_kernel == 2:  # the direct kernel: its second flag sums the reductions (a run's last op)
            return "k_cluster_f32_split6<%s, %s>" % (b(lowt), b(rec.get("stats")))
        return "k_cluster_f32_gauss6<%s>" % b(lowt)
    if rec.get("staged"):
        return "k_cluster_f32_stage<%d, 6, %s>" % (k, b(lowt))
    return "k_cluster_f32_mfma<%d, %d, %s, %s>" % (k, 1 if k == 6 else 2, b(lowt), b(rec.get("stats")))


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--rows", type=int, default=5)
    ap.add_argument("--cols", type=int, default=6)
    ap.add_argument("--depth", type=int, default=25)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--drop-corner", action="store_true",
                    help="leave out the grid's last site (34 qubits: 5x7 minus site (4, 6))")
    ap.add_argument("--kmax", type=int, default=6)
    ap.add_argument("--scheduler", default="learned")
    ap.add_argument("--no-fuse-diag", action="store_true")
    ap.add_argument("--pair-tile", type=int, default=None, choices=[10, 11],
                    help="qubits of the tile the pair kernel holds in LDS")
    ap.add_argument("--pair", type=int, default=None,
                    help="pairing of small clusters: 0 off, 1 pairs, 2 every cluster alone in the pair kernel")
    ap.add_argument("--fp64-steps", type=int, default=None, help="steps of the float64 per-gate form")
    ap.add_argument("--fp64-kmax", type=int, default=5, help="largest cluster of the float64 fused form")
    ap.add_argument("--no-fp64-fused", action="store_true", help="skip the float64 fused form")
    ap.add_argument("--only", choices=["fused", "pergate", "batch"], default=None,
                    help="run one form only (for profiling); batch: the 512-circuit launch alone")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-gates", type=int, default=24)
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-circuit batched launch")
    ap.add_argument("--batch-kmax", type=int, default=None,
                    help="largest cluster of the batched circuits (default: the binding's, from the tune table)")
    return ap.parse_args()


def batch_bench(qsim, torch, kmax, runs=3, n_check=8):
    """512 circuits (n ~ U[14, 24], depth ~ U[10, 40], seeds 1000 + i) in one
    persistent launch: circuits per second of qsim_batch_run (initialisation
    and every op of every circuit, matrices built on the GPU) and of plan + run,
    and a sample of circuits compared with the float64 per-gate path."""
    from supremacy_inputs import batch_circuit
    circs = [batch_circuit(i) for i in range(512)]
    t0 = time.perf_counter()
    b = qsim.Batch(circs, kmax=kmax)
    plan_s = time.perf_counter() - t0
    kmax = b.kmax
    b.run()
    runs_ms = [b.run()["run_ms"] for _ in range(runs)]
    st = b.run()
    run_s = min(runs_ms + [st["run_ms"]]) / 1e3
    # algorithmic bytes: every cluster op reads and writes its whole state, the
    # initialisation writes it; with the folded start the first cluster starts
    # from the uniform state in registers and only writes
    fold = qsim.get_option(qsim.OPT_FOLD_INIT) != 0
    alg = 0
    for i, c in enumerate(circs):
        sc = qsim.schedule(c.n, c.gates, kmax=kmax, scheduler="greedy", fuse_diag=True, skip_initial_h=True)
        m = len(sc["op_kind"])
        if fold and m and sc["op_kind"][0] == 0:
            alg += ((m - 1) * 16 + 8) * 2 ** c.n
        else:
            alg += (m * 16 + 8) * 2 ** c.n
    worst = 1.0
    idx = [int(i) for i in range(0, 512, 512 // n_check)][:n_check]
    for i in idx:
        c = circs[i]
        s = qsim.State(c.n, "c128")
        s.run_circuit(c.gates, scheduler="per_gate")
        f, _ = s.compare(b.states[i].to(torch.complex128))
        worst = min(worst, f)
        del s
    res = {"circuits": 512, "qubits": "14-24", "depths": "10-40", "dtype": "c64", "kmax": kmax,
           "circuits_per_s": round(512 / run_s, 1), "run_ms": round(run_s * 1e3, 2),
           "circuits_per_s_with_plan": round(512 / (run_s + st["plan_ms"] / 1e3), 1),
           "plan_ms": round(st["plan_ms"], 2), "ops": st["n_ops"], "work_items": st["n_items"],
           "grid": st["grid"], "algorithmic_GB": round(alg / 1e9, 1),
           "hbm_GBs": round(alg / run_s / 1e9, 1), "hbm_frac": round(alg / run_s / 1e9 / HBM_PEAK_GBS, 4),
           "min_fidelity_vs_fp64_per_gate": worst, "fidelity_sample": "%d circuits" % len(idx),
           "python_plan_s": round(plan_s, 3)}
    del b
    torch.cuda.empty_cache()
    return res


def cpu_baseline(circ, n_sample):
    """Time the oracle on a stratified sample of the circuit's gates at full
    size and scale to all gates (the oracle applies every gate, one at a time)."""
    import ctypes

    import numpy as np

    import oracle
    from supremacy_inputs import Circuit, to_text

    L = oracle.lib()
    n = circ.n
    step = max(1, len(circ.gates) // n_sample)
    sample = circ.gates[::step][:n_sample]
    psi = np.empty(2 ** n, np.complex128)
    ptr = psi.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    t0 = time.perf_counter()
    L.oracle_run_text(ptr, n, ("n %d\n" % n).encode())  # |0...0>
    t1 = time.perf_counter()
    rc = L.oracle_apply_text(ptr, n, to_text(Circuit(n, sample)).encode())
    t2 = time.perf_counter()
    assert rc == len(sample)
    per_gate = (t2 - t1) / len(sample)
    est = (t1 - t0) + per_gate * len(circ.gates)
    del psi
    return {"value": round(est, 2), "unit": "s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "%d of %d gates (every %d-th) applied to the full 2^%d complex128 state in %.1f s, "
                      "plus |0> initialisation %.1f s; scaled to all %d gates"
                      % (len(sample), len(circ.gates), step, n, t2 - t1, t1 - t0, len(circ.gates))}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the whole state vector lives in one MI355X's HBM and "
              "this build has no multi-GPU path (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1704_01127_amd import qsim
    from supremacy_inputs import supremacy_circuit

    if args.pair is not None:
        qsim.set_option(qsim.OPT_PAIR, args.pair)
    if args.pair_tile is not None:
        qsim.set_option(qsim.OPT_PAIR_TILE, args.pair_tile)
    drop = ((args.rows - 1, args.cols - 1),) if args.drop_corner else ()
    circ = supremacy_circuit(args.rows, args.cols, args.depth, args.seed, drop=drop)
    n = circ.n
    gates = circ.gates
    # fused_stats: the last cluster pass also sums the reductions the step reports
    fused_opts = dict(kmax=args.kmax, scheduler=args.scheduler, fuse_diag=not args.no_fuse_diag,
                      skip_trailing_diag=True, skip_initial_h=True, fused_stats=True)
    pergate_opts = dict(scheduler="per_gate", skip_trailing_diag=True, skip_initial_h=True)

    def writes_whole_state(opts):
        """True when the run replaces the leading H layer by writing the uniform
        state (every qubit's first gate is an H the schedule skips): the run then
        starts from |0...0> without reading the state, and a |0...0> pass before
        it would be overwritten unread."""
        sc = qsim.schedule(n, gates, qsim.C64 if opts is fused_opts else qsim.C128, **opts)
        first = {}
        for i, g in enumerate(gates):
            for q in g.qubits:
                first.setdefault(q, i)
        return len(first) == n and all(gates[i].name == "H" and sc["gate_op"][i] == -1 for i in first.values())

    def timed(state, opts, steps, warmup, record):
        fresh = writes_whole_state(opts)

        def step():
            if not fresh:
                state.init("zero")
            st = state.run_circuit(gates, record_timings=record, **opts)
            return st, state.probs()
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        recs, per = [], []
        for _ in range(steps):
            # a step ends with the reductions' device-to-host copy (synchronous)
            t0 = time.perf_counter()
            st, res = step()
            torch.cuda.synchronize()
            per.append(time.perf_counter() - t0)
            if record:  # reading the step's HIP events is measurement, outside the step
                recs.extend(state.op_timings())
        return sum(per) / steps, per, st, res, recs

    out = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "data": "synthetic"}
    if args.only == "batch":
        print(json.dumps({"batch": batch_bench(qsim, torch, args.batch_kmax)}), flush=True)
        return

    fused = pergate = None
    if args.only in (None, "fused"):
        s32 = qsim.State(n, "c64", kmax=max(args.kmax, 5))
        fused = timed(s32, fused_opts, args.steps, args.warmup, record=True)
    if args.only in (None, "pergate"):
        s64 = qsim.State(n, "c128", kmax=max(args.kmax, 5))
        k64 = args.fp64_steps if args.fp64_steps is not None else args.steps
        pergate = timed(s64, pergate_opts, k64, min(args.warmup, 1), record=False)

    ref = fused if fused is not None else pergate
    tts, per, st, res, recs = ref
    out["value"] = round(tts, 5)
    out["unit"] = "s"
    out["ms_per_step"] = round(tts * 1e3, 3)
    out["dtype"] = "f32" if fused is not None else "f64"
    out["config"] = {"workload": "%d-qubit %dx%d-grid%s depth-%d random supremacy circuit (%d gates, seed %d)"
                                 % (n, args.rows, args.cols, " minus corner site" if args.drop_corner else "",
                                    args.depth, len(gates), args.seed),
                     "form": "float32 state, fused clusters k<=%d, scheduler %s, diagonal fusion %s"
                             % (args.kmax, args.scheduler, "on" if not args.no_fuse_diag else "off")
                             if fused is not None else "float64 state, one launch per gate",
                     "skips": "leading H layer -> uniform init; trailing diagonal gates dropped (Sec. 3.6)"}
    out["stats"] = {"norm": res[0], "sum_p2_times_N": res[1] * 2 ** n, "entropy_nats": res[2],
                    "ops": st["n_ops"], "clusters_by_k": st["n_clusters_by_k"], "diag_ops": st["n_diag_ops"],
                    "gates_applied": st["n_gates_applied"], "schedule_ms": round(st["schedule_ms"], 3),
                    "step_s_median": round(statistics.median(per), 5),
                    "step_s": [round(x, 5) for x in per]}
    out["amplitude_updates_per_s"] = len(gates) * 2 ** n / tts

    if pergate is not None and fused is not None:
        out["fp64_per_gate"] = {"tts_s": round(pergate[0], 4), "steps": len(pergate[1]),
                                "launches": pergate[2]["n_ops"], "norm": pergate[3][0],
                                "entropy_nats": pergate[3][2]}
        out["speedup_vs_fp64_per_gate"] = round(pergate[0] / fused[0], 2)
        fid, maxd = s32.compare(s64.amps)
        out["fused_vs_fp64_per_gate"] = {"fidelity": fid, "max_abs_diff": maxd}
        if not args.no_fp64_fused:
            # float64 state, fused clusters: the float64 path's accuracy at full size
            f64_opts = dict(fused_opts, kmax=args.fp64_kmax)
            s64f = qsim.State(n, "c128", kmax=max(args.fp64_kmax, 5))
            f64 = timed(s64f, f64_opts, args.steps, min(args.warmup, 1), record=False)
            fid64, maxd64 = s64f.compare(s64.amps)
            out["fp64_fused"] = {"tts_s": round(f64[0], 5), "steps": len(f64[1]), "kmax": args.fp64_kmax,
                                 "scheduler": args.scheduler, "ops": f64[2]["n_ops"],
                                 "vs_fp64_per_gate": {"fidelity": fid64, "max_abs_diff": maxd64},
                                 "speedup_vs_fp64_per_gate": round(pergate[0] / f64[0], 2)}
            del s64f
            torch.cuda.empty_cache()

    if recs:
        k6k = qsim.get_option(qsim.OPT_K6_KERNEL)
        amp_bytes = 8
        # passes that apply clusters: single clusters and pairs (two clusters, one pass)
        clusters = [r for r in recs if r["kind"] in ("cluster", "pair")]
        total_ms = sum(r["ms"] for r in recs)
        groups = {}
        for r in clusters:
            groups.setdefault(kernel_name(r, k6k, qsim.get_option(qsim.OPT_PAIR_TILE)), []).append(r["ms"])
        kname, times = max(groups.items(), key=lambda kv: sum(kv[1]))
        bytes_per_launch = 2 * 2 ** n * amp_bytes
        avg_ms = sum(times) / len(times)
        ach = bytes_per_launch / (avg_ms * 1e-3) / 1e9
        traffic = None
        tpath = os.path.join(ROOT, "profiles", "traffic_cluster_f32_30q.json")
        if n == 30 and os.path.exists(tpath):  # the counters were taken on the 30-qubit workload
            with open(tpath) as f:
                t = json.load(f)
            if t.get("kernel_source_sha") == kernel_source_hash() and kname in t.get("kernels", {}):
                traffic = round(t["kernels"][kname]["bytes_per_launch"])
        out["roofline"] = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname,
                           "launches": len(times), "avg_ms": round(avg_ms, 4),
                           "algorithmic_bytes_per_launch": bytes_per_launch,
                           "kernel_groups": {k: {"launches": len(v), "avg_ms": round(sum(v) / len(v), 4)}
                                             for k, v in groups.items()}}
        csum = sum(r["ms"] for r in clusters)
        cbytes = len(clusters) * 2 * 2 ** n * amp_bytes
        cflops = sum(2 ** n * (8 * 2 ** r["k"] - 2) * (2 if r["kind"] == "pair" else 1) for r in clusters)
        out["cluster_kernels"] = {"launches_per_step": len(clusters) // max(1, args.steps),
                                  "hbm_GBs": round(cbytes / (csum * 1e-3) / 1e9, 1),
                                  "hbm_frac": round(cbytes / (csum * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                  "tflops": round(cflops / (csum * 1e-3) / 1e12, 2),
                                  "share_of_gpu_time": round(csum / total_ms, 4)}
        by_k = {}
        for r in clusters:
            d = by_k.setdefault("pair" if r["kind"] == "pair" else r["k"], [0, 0.0])
            d[0] += 1
            d[1] += r["ms"]
        out["cluster_kernels"]["by_k"] = {
            str(kk): {"launches": v[0], "avg_ms": round(v[1] / v[0], 4),
                      "GBs": round(2 * 2 ** n * amp_bytes / (v[1] / v[0] * 1e-3) / 1e9, 1)}
            for kk, v in sorted(by_k.items(), key=lambda kv: str(kv[0]))}
        others = {}
        for r in recs:
            if r["kind"] not in ("cluster", "pair"):
                d = others.setdefault(r["kind"], [0, 0.0])
                d[0] += 1
                d[1] += r["ms"]
        out["other_kernels"] = {kk: {"launches": v[0], "total_ms": round(v[1], 3)} for kk, v in others.items()}

    if not args.no_batch and args.only is None:
        del s32, s64
        torch.cuda.empty_cache()
        out["batch"] = batch_bench(qsim, torch, args.batch_kmax)

    if not args.no_cpu_baseline:
        # free the GPU states first: the oracle needs 16 GiB of host memory
        out["cpu_baseline"] = cpu_baseline(circ, args.cpu_sample_gates)
    out["paper_context"] = {"tts_s": 9.58, "hardware": "1 Cori II node (Xeon Phi 7250, 68 cores)",
                            "precision": "complex128", "gates": 369, "source": "Table 2"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
