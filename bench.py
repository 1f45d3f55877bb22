#!/usr/bin/env python3
"""Time-to-solution of a 30-qubit depth-25 random supremacy circuit on one
MI355X: float32 fused clusters versus float64 one gate at a time.

One step = initialise |0...0>, run the whole circuit through the library
(scheduling, float64 cluster-matrix build on the GPU, cluster / diagonal
kernels), then the float64 reductions (norm, sum p^2, entropy) that give the
output distribution's statistics. Inputs are resident in HBM; the timed
region is bracketed by device synchronisation.

Prints one JSON line. `value` is the time-to-solution in seconds of the
complex64 fused form (6-qubit clusters on fp16 matrix cores with hi/lo
operand halves and fp32 accumulation, smaller clusters on fp32 matrix
cores). Also timed: the same form with 6-qubit clusters on fp32 matrix
cores, float64 fused clusters and float64 one gate at a time. `roofline` is
measured live from HIP events around every launch of the timed steps.
`cpu_baseline` is the CPU oracle run once over the whole circuit (the same
gates the GPU forms apply); every GPU form is then compared with the
oracle's state, amplitude by amplitude, in float64 on the GPU.
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


def kernel_name(rec, k6_kernel=2, pair_tile=11, dbl=False, n=None) -> str:
    """Name (as rocprofv3 reports it) of the cluster kernel a launch used (n:
    the state's qubits, which decide the vector-ALU kernel's form)."""
    k, lowt = rec["k"], rec["qubits"][0] == 0
    staged_valu = n is not None and 2 <= k <= 3 and n - k >= 6 and not rec.get("mfma")
    if dbl:
        if not rec.get("mfma"):
            return ("k_cluster_valu_staged<double, %d, false>" if staged_valu else "k_cluster_valu<double, %d>") % k
        if rec.get("staged"):
            return "k_cluster_f64_stage<%d, 5, %d>" % (k, 512 if k == 5 else 256)
        return "k_cluster_f64_mfma<%d, %d, %d>" % (k, 1 if k == 6 else 2, 512 if k == 6 else 256)
    if rec["kind"] == "pair":
        q = set(rec["qubits"])
        ten = pair_tile == 10 and (0 in q or len(q) < 10)  # the 10-qubit tile holds qubit 0
        return "k_cluster_f32_pair10<12>" if ten else "k_cluster_f32_multi<2, 8>"
    b = lambda x: "true" if x else "false"  # noqa: E731
    if staged_valu:  # its second flag sums the reductions
        return "k_cluster_valu_staged<float, %d, %s>" % (k, b(rec.get("stats")))
    if not rec.get("mfma"):
        return "k_cluster_valu<float, %d>" % k
    if k == 7:  # the direct kernel only; its second flag sums the reductions
        return "k_cluster_f32_split7<%s, %s>" % (b(lowt), b(rec.get("stats")))
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
    ap.add_argument("--kmax", type=int, default=7)
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
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle (and with it every comparison against the oracle)")
    ap.add_argument("--no-fp32-k6", action="store_true",
                    help="skip the form with 6-qubit clusters on the fp32 matrix cores")
    ap.add_argument("--no-k6", action="store_true",
                    help="skip the form whose clusters have at most 6 qubits (with --kmax 7)")
    ap.add_argument("--no-mapped", action="store_true",
                    help="skip the fused forms with the qubit mapping (QSIM_OPT_MAP_QUBITS)")
    ap.add_argument("--batch-check-every", type=int, default=8,
                    help="compare every n-th circuit of the batch with the oracle (0: none)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-circuit batched launch")
    ap.add_argument("--batch-kmax", type=int, default=None,
                    help="largest cluster of the batched circuits (default: the binding's, from the tune table)")
    return ap.parse_args()


def host_info() -> dict:
    """CPU model, CPUs this process may run on, and RAM of the host."""
    info = {"cpu_model": "", "cpus_available": len(os.sched_getaffinity(0)), "ram_GiB": None}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    info["ram_GiB"] = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return info


def batch_bench(qsim, torch, kmax, runs=3, check_every=8):
    """512 circuits (n ~ U[14, 24], depth ~ U[10, 40], seeds 1000 + i) in one
    persistent launch: circuits per second of qsim_batch_run (initialisation
    and every op of every circuit, matrices built on the GPU) and of plan + run,
    and every `check_every`-th circuit compared with the CPU oracle."""
    import numpy as np

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
    res = {"circuits": 512, "qubits": "14-24", "depths": "10-40", "dtype": "c64", "kmax": kmax,
           "circuits_per_s": round(512 / run_s, 1), "run_ms": round(run_s * 1e3, 2),
           "circuits_per_s_with_plan": round(512 / (run_s + st["plan_ms"] / 1e3), 1),
           "plan_ms": round(st["plan_ms"], 2), "ops": st["n_ops"], "work_items": st["n_items"],
           "grid": st["grid"], "algorithmic_GB": round(alg / 1e9, 1),
           "hbm_GBs": round(alg / run_s / 1e9, 1), "hbm_frac": round(alg / run_s / 1e9 / HBM_PEAK_GBS, 4),
           "python_plan_s": round(plan_s, 3)}
    if check_every:
        import oracle
        worst_f, worst_d, worst_rel, t_or = 1.0, 0.0, 0.0, 0.0
        idx = list(range(0, 512, check_every))
        for i in idx:
            c = circs[i]
            t1 = time.perf_counter()
            psi = oracle.run(c)
            t_or += time.perf_counter() - t1
            mx = float(np.max(np.abs(psi)))
            ref = torch.from_numpy(psi).to(b.states[i].device)
            s = qsim.State(c.n, "c64", init="keep", amps=b.states[i])
            f, d = s.compare(ref)
            worst_f, worst_d, worst_rel = min(worst_f, f), max(worst_d, d), max(worst_rel, d / mx)
            del s, ref, psi
        res["vs_oracle"] = {"circuits": len(idx), "subset": "every %d-th circuit (indices 0, %d, ..., %d)"
                            % (check_every, check_every, idx[-1]), "min_fidelity": worst_f,
                            "max_abs_diff": worst_d, "max_abs_diff_over_max_amp": worst_rel,
                            "oracle_s": round(t_or, 2)}
    del b
    torch.cuda.empty_cache()
    return res


def cpu_baseline(circ):
    """The CPU oracle over the whole circuit, once, timed by the wall clock
    (float64, one gate at a time, OpenMP over the host's cores). Returns its
    record and the state it computed."""
    import oracle
    t0 = time.perf_counter()
    psi = oracle.run(circ)
    dt = time.perf_counter() - t0
    rec = {"value": round(dt, 2), "unit": "s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": "the whole circuit once, not a sample: %d gates (%s) applied one at a time to the "
                     "2^%d complex128 state (%.0f GiB) from |0...0>, allocation included"
                     % (len(circ.gates), ", ".join("%s %d" % kv for kv in sorted(circ.counts().items())),
                        circ.n, 2 ** circ.n * 16 / 2 ** 30),
           "gates_per_s": round(len(circ.gates) / dt, 2), "host": host_info()}
    return rec, psi


def cluster_roofline(recs, n, dbl, steps, k6_kernel, pair_tile):
    """Roofline of the dominant cluster kernel of a recorded run (its
    algorithmic bytes per launch over its average HIP-event duration), and
    the totals of all cluster passes."""
    amp_bytes = 16 if dbl else 8
    clusters = [r for r in recs if r["kind"] in ("cluster", "pair")]
    if not clusters:
        return None, None
    total_ms = sum(r["ms"] for r in recs)
    groups = {}
    for r in clusters:
        groups.setdefault(kernel_name(r, k6_kernel, pair_tile, dbl, n), []).append(r["ms"])
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
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": kname,
            "launches": len(times), "avg_ms": round(avg_ms, 4),
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "kernel_groups": {k: {"launches": len(v), "avg_ms": round(sum(v) / len(v), 4)}
                              for k, v in groups.items()}}
    csum = sum(r["ms"] for r in clusters)
    cbytes = len(clusters) * 2 * 2 ** n * amp_bytes
    cflops = sum(2 ** n * (8 * 2 ** r["k"] - 2) * (2 if r["kind"] == "pair" else 1) for r in clusters)
    ck = {"launches_per_step": len(clusters) // max(1, steps),
          "hbm_GBs": round(cbytes / (csum * 1e-3) / 1e9, 1),
          "hbm_frac": round(cbytes / (csum * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
          "tflops": round(cflops / (csum * 1e-3) / 1e12, 2),
          "share_of_gpu_time": round(csum / total_ms, 4)}
    by_k = {}
    for r in clusters:
        d = by_k.setdefault("pair" if r["kind"] == "pair" else r["k"], [0, 0.0])
        d[0] += 1
        d[1] += r["ms"]
    ck["by_k"] = {str(kk): {"launches": v[0], "avg_ms": round(v[1] / v[0], 4),
                            "GBs": round(2 * 2 ** n * amp_bytes / (v[1] / v[0] * 1e-3) / 1e9, 1)}
                  for kk, v in sorted(by_k.items(), key=lambda kv: str(kv[0]))}
    others = {}
    for r in recs:
        if r["kind"] not in ("cluster", "pair"):
            d = others.setdefault(r["kind"], [0, 0.0])
            d[0] += 1
            d[1] += r["ms"]
    ck["other_kernels"] = {kk: {"launches": v[0], "total_ms": round(v[1], 3)} for kk, v in others.items()}
    return roof, ck


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the whole state vector lives in one MI355X's HBM and "
              "the library runs on one GPU (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
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
    # the gate list in the library's C layout, built once like the resident
    # state: a step times the library call (validation, scheduling, matrix
    # builds, passes), not Python's marshalling of the list
    cgates = qsim.Gates(gates)
    # fused_stats: the last cluster pass also sums the reductions the step reports
    fused_opts = dict(kmax=args.kmax, scheduler=args.scheduler, fuse_diag=not args.no_fuse_diag,
                      skip_trailing_diag=True, skip_initial_h=True, fused_stats=True)
    pergate_opts = dict(scheduler="per_gate", skip_trailing_diag=True, skip_initial_h=True)
    k6_opts = dict(fused_opts, kmax=6)

    def timed(state, opts, steps, warmup, record):
        fresh = writes_whole_state(qsim, n, gates, opts, state.dt)

        def step():
            if not fresh:
                state.init("zero")
            st = state.run_circuit(cgates, record_timings=record, **opts)
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
        return dict(tts=sum(per) / steps, per=per, st=st, res=res, recs=recs)

    out = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "data": "synthetic"}
    if args.only == "batch":
        print(json.dumps({"batch": batch_bench(qsim, torch, args.batch_kmax, check_every=0)}), flush=True)
        return

    k6_default = qsim.get_option(qsim.OPT_K6_KERNEL)
    pair_tile = qsim.get_option(qsim.OPT_PAIR_TILE)
    states, forms = {}, {}
    if args.only in (None, "fused"):
        states["c64_fused"] = qsim.State(n, "c64", kmax=max(args.kmax, 5))
        forms["c64_fused"] = timed(states["c64_fused"], fused_opts, args.steps, args.warmup, record=True)
    if args.only is None and not args.no_k6 and args.kmax >= 7:
        # the same scheduler with clusters of at most 6 qubits (fp16-halves 6-qubit kernel)
        states["c64_fused_k6"] = qsim.State(n, "c64", kmax=6)
        forms["c64_fused_k6"] = timed(states["c64_fused_k6"], k6_opts, args.steps, min(args.warmup, 1), record=True)
    if args.only is None and not args.no_fp32_k6 and args.kmax >= 6:
        # 6-qubit clusters on the fp32 matrix cores (7-qubit clusters need the
        # fp16 kernel, so the cap is 6 there)
        qsim.set_option(qsim.OPT_K6_KERNEL, 0)
        try:
            states["c64_fused_fp32_k6"] = qsim.State(n, "c64", kmax=max(args.kmax, 5))
            forms["c64_fused_fp32_k6"] = timed(states["c64_fused_fp32_k6"], fused_opts, args.steps,
                                               min(args.warmup, 1), record=True)
        finally:
            qsim.set_option(qsim.OPT_K6_KERNEL, k6_default)
    if args.only is None and not args.no_mapped:
        # the same form with the qubit mapping: relabelled qubits, one permutation pass at the end
        qsim.set_option(qsim.OPT_MAP_QUBITS, 1)
        try:
            states["c64_fused_mapped"] = qsim.State(n, "c64", kmax=max(args.kmax, 5))
            forms["c64_fused_mapped"] = timed(states["c64_fused_mapped"], fused_opts, args.steps,
                                              min(args.warmup, 1), record=True)
        finally:
            qsim.set_option(qsim.OPT_MAP_QUBITS, 0)
    if args.only in (None, "pergate"):
        states["c128_per_gate"] = qsim.State(n, "c128", kmax=max(args.kmax, 5))
        k64 = args.fp64_steps if args.fp64_steps is not None else args.steps
        forms["c128_per_gate"] = timed(states["c128_per_gate"], pergate_opts, k64, min(args.warmup, 1),
                                       record=False)
    if args.only is None and not args.no_fp64_fused:
        # float64 state, fused clusters: the float64 path's accuracy at full size
        f64_opts = dict(fused_opts, kmax=args.fp64_kmax)
        states["c128_fused"] = qsim.State(n, "c128", kmax=max(args.fp64_kmax, 5))
        forms["c128_fused"] = timed(states["c128_fused"], f64_opts, args.steps, min(args.warmup, 1), record=True)
        if not args.no_mapped:
            qsim.set_option(qsim.OPT_MAP_QUBITS, 1)
            try:
                states["c128_fused_mapped"] = qsim.State(n, "c128", kmax=max(args.fp64_kmax, 5))
                forms["c128_fused_mapped"] = timed(states["c128_fused_mapped"], f64_opts, args.steps,
                                                   min(args.warmup, 1), record=True)
            finally:
                qsim.set_option(qsim.OPT_MAP_QUBITS, 0)

    main_key = "c64_fused" if "c64_fused" in forms else "c128_per_gate"
    ref = forms[main_key]
    tts, per, st, res = ref["tts"], ref["per"], ref["st"], ref["res"]
    out["value"] = round(tts, 5)
    out["unit"] = "s"
    out["ms_per_step"] = round(tts * 1e3, 3)
    if main_key == "c64_fused":
        out["dtype"] = "f32 (6- and 7-qubit clusters: f16 hi/lo operand halves, f32 accumulate)"
        form = ("complex64 state; clusters of <= %d qubits (scheduler %s, diagonal fusion %s) built in "
                "float64 on the GPU; 6- and 7-qubit clusters on fp16 matrix cores with hi/lo halves of both "
                "operands (three products, fp32 accumulation; 7-qubit ones on the real and imaginary parts "
                "of the matrix), smaller ones on fp32 matrix cores; float64 reductions"
                % (args.kmax, args.scheduler, "on" if not args.no_fuse_diag else "off"))
    else:
        out["dtype"] = "f64"
        form = "complex128 state, one launch per gate"
    out["config"] = {"workload": "%d-qubit %dx%d-grid%s depth-%d random supremacy circuit (%d gates, seed %d)"
                                 % (n, args.rows, args.cols, " minus corner site" if args.drop_corner else "",
                                    args.depth, len(gates), args.seed),
                     "form": form,
                     "skips": "leading H layer -> uniform init; trailing diagonal gates dropped (Sec. 3.6)"}
    out["stats"] = {"norm": res[0], "sum_p2_times_N": res[1] * 2 ** n, "entropy_nats": res[2],
                    "ops": st["n_ops"], "clusters_by_k": st["n_clusters_by_k"], "diag_ops": st["n_diag_ops"],
                    "gates_applied": st["n_gates_applied"], "schedule_ms": round(st["schedule_ms"], 3),
                    "step_s_median": round(statistics.median(per), 5),
                    "step_s": [round(x, 5) for x in per]}
    out["amplitude_updates_per_s"] = len(gates) * 2 ** n / tts

    if ref["recs"]:
        roof, ck = cluster_roofline(ref["recs"], n, False, args.steps, k6_default, pair_tile)
        out["roofline"] = roof
        out["cluster_kernels"] = ck
    desc = {"c64_fused_k6": "complex64 state, the same scheduler with clusters of <= 6 qubits (6-qubit ones "
                            "on fp16 matrix cores with operand halves)",
            "c64_fused_fp32_k6": "complex64 state, clusters of <= 6 qubits with the 6-qubit ones on fp32 matrix "
                                 "cores (real-split product)",
            "c128_fused": "complex128 state, fused clusters of <= %d qubits on fp64 matrix cores" % args.fp64_kmax,
            "c128_per_gate": "complex128 state, one launch per gate (the plain method)",
            "c64_fused_mapped": "the complex64 form with the qubit mapping (least used qubits on the slow bit "
                                "locations, one permutation pass at the end)",
            "c128_fused_mapped": "the complex128 fused form with the qubit mapping"}
    out["forms"] = {}
    for key, f in forms.items():
        if key == main_key:
            continue
        d = {"form": desc[key], "tts_s": round(f["tts"], 5), "steps": len(f["per"]), "ops": f["st"]["n_ops"],
             "norm": f["res"][0], "entropy_nats": f["res"][2]}
        if f["recs"]:
            perm = [r["ms"] for r in f["recs"] if r["kind"] == "permute"]
            if perm:
                d["permute_ms"] = round(sum(perm) / len(perm), 4)
        if f["recs"]:
            d["roofline"], _ = cluster_roofline(f["recs"], n, key.startswith("c128"), len(f["per"]),
                                                0 if key == "c64_fused_fp32_k6" else k6_default, pair_tile)
        out["forms"][key] = d
    if "c128_per_gate" in forms and main_key != "c128_per_gate":
        out["speedup_vs_fp64_per_gate"] = round(forms["c128_per_gate"]["tts"] / tts, 2)

    if not args.no_cpu_baseline:
        # the oracle applies the gates the GPU forms apply: the leading H layer
        # explicitly (the GPU writes the uniform state instead, the same state),
        # and not the trailing diagonal gates
        import oracle
        kept, dropped = oracle.drop_trailing_diagonal(circ)
        rec, psi = cpu_baseline(kept)
        rec["trailing_diagonal_gates_dropped"] = len(dropped)
        out["cpu_baseline"] = rec
        onorm, os2, oent = oracle.stats(psi)
        mx = float(np.max(np.abs(psi)))
        ref_dev = torch.from_numpy(psi).to(states[main_key].amps.device)
        del psi
        vs = {"oracle": "float64 CPU oracle, %d gates; compared in float64 on the GPU" % len(kept.gates),
              "max_abs_amp": mx}
        for key, f in forms.items():
            fid, md = states[key].compare(ref_dev)
            # every form applies the oracle's gates: those not skipped, plus the H layer it replaces
            opts = pergate_opts if key == "c128_per_gate" else (k6_opts if key == "c64_fused_k6" else fused_opts)
            fresh = writes_whole_state(qsim, n, gates, opts, states[key].dt)
            same = f["st"]["n_gates_applied"] + (n if fresh else 0) == len(kept.gates)
            vs[key] = {"fidelity": fid, "max_abs_diff": md, "max_abs_diff_over_max_amp": md / mx,
                       "same_gates": same, "norm_diff": f["res"][0] - onorm,
                       "entropy_diff_nats": f["res"][2] - oent,
                       "sum_p2_rel_diff": (f["res"][1] - os2) / os2}
        out["vs_oracle"] = vs
        del ref_dev
    for key in list(states):
        del states[key]
    torch.cuda.empty_cache()

    if not args.no_batch and args.only is None:
        out["batch"] = batch_bench(qsim, torch, args.batch_kmax, check_every=args.batch_check_every)

    out["paper_context"] = {"tts_s": 9.58, "hardware": "1 Cori II node (Xeon Phi 7250, 68 cores)",
                            "precision": "complex128", "gates": 369, "source": "Table 2"}
    print(json.dumps(out), flush=True)


def writes_whole_state(qsim, n, gates, opts, dtype) -> bool:
    """True when a run replaces the leading H layer by writing the uniform
    state (every qubit's first gate is an H the schedule skips): the run then
    starts from |0...0> without reading the state, and a |0...0> pass before
    it would be overwritten unread."""
    sc = qsim.schedule(n, gates, dtype, **opts)
    first = {}
    for i, g in enumerate(gates):
        for q in g.qubits:
            first.setdefault(q, i)
    return len(first) == n and all(gates[i].name == "H" and sc["gate_op"][i] == -1 for i in first.values())


if __name__ == "__main__":
    main()
