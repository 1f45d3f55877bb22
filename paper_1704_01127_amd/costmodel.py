"""Learned cost model of the clustering scheduler: record, train, compare.

record   runs seeded random circuits (supremacy circuits of depth 40 with a
         Haar-random 5-qubit gate after every 8th cycle) under many schedules
         with per-launch HIP-event timing and stores, per op, the library's
         feature vector and ln(us per 2^30 amplitudes).
train    fits the MLP (16 -> 64 -> 64 -> 1, float32) with the library's own
         GPU forward / backward / Adam kernels and writes cost_model.npz.
compare  times held-out circuits with the learned scheduler against the
         fixed-k greedy scheduler (and the analytic one) and checks that the
         results agree.

    python -m paper_1704_01127_amd.costmodel record --out records.npz
    python -m paper_1704_01127_amd.costmodel train --data records.npz --out paper_1704_01127_amd/cost_model.npz
    python -m paper_1704_01127_amd.costmodel compare
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import qsim

N_IN, N_HIDDEN = 16, 64


def workload(n: int, depth: int, seed: int):
    from supremacy_inputs import supremacy_circuit, with_haar_layers
    from supremacy_inputs.circuits import batch_grid
    R, C, drop = batch_grid(n)
    circ = supremacy_circuit(R, C, depth, seed, drop)
    return with_haar_layers(circ, 8, 5, seed + 77)


def op_record_rows(recs, n, dtype_code):
    feats, ys = [], []
    for r in recs:
        if r["kind"] not in ("cluster", "diag"):
            continue
        k = r["k"] if r["kind"] == "cluster" else 0
        qs = r["qubits"] if k else []
        f = qsim.cost_features(n, dtype_code, qs, n_epi=r["n_epi"])  # what the scheduler passes for the op
        feats.append(f)
        ys.append(math.log(r["ms"] * 1e3 / 2.0 ** (n - 30)))
    return feats, ys


def cmd_record(args):
    import torch  # noqa: F401
    feats, ys, meta = [], [], []
    if args.append:  # extend an earlier record file (its rows come first)
        old = np.load(args.append, allow_pickle=False)
        feats, ys, meta = list(old["x"]), list(old["y"]), [tuple(m) for m in old["meta"]]
    t_start = time.time()
    sizes = [int(x) for x in args.n.split(",")]
    kmaxes = [int(x) for x in args.kmax.split(",")]
    for dt in args.dtypes.split(","):
        code = qsim.C64 if dt == "c64" else qsim.C128
        # 7-qubit clusters exist on complex64 only (complex128 runs cap k_max at 6)
        configs = [dict(kmax=k, fuse_diag=fd) for k in kmaxes if dt == "c64" or k <= 6 for fd in (False, True)]
        for n in sizes:
            state = qsim.State(n, dt, kmax=7)
            for seed in range(args.seeds):
                circ = workload(n, args.depth, seed)
                for ci, cfg in enumerate(configs):
                    # both matrix-core kernel variants (direct gather, LDS-staged
                    # tiles) on every op, so the model learns which is faster
                    # for a given target set
                    for variant in (0, 1):
                        qsim.set_option(qsim.OPT_CLUSTER_VARIANT, variant)
                        try:
                            state.init("uniform")
                            state.run_circuit(circ.gates, record_timings=True, skip_trailing_diag=True, **cfg)
                            f, y = op_record_rows(state.op_timings(), n, code)
                        finally:
                            qsim.set_option(qsim.OPT_CLUSTER_VARIANT, -1)
                        feats += f
                        ys += y
                        meta += [(seed, n, code, ci)] * len(y)
                print("recorded %s n=%d seed=%d: %d records (%.0f s)" % (dt, n, seed, len(ys), time.time() - t_start),
                      flush=True)
            del state
    np.savez(args.out, x=np.array(feats, np.float32), y=np.array(ys, np.float64),
             meta=np.array(meta, np.int32))
    print("wrote %d records to %s" % (len(ys), args.out), flush=True)


def init_params(rng, n_in=N_IN, h=N_HIDDEN):
    """He-uniform weights, zero biases, in the library's flat layout."""
    def u(fan_in, shape):
        lim = math.sqrt(6.0 / fan_in)
        return rng.uniform(-lim, lim, shape)
    return np.concatenate([u(n_in, h * n_in), np.zeros(h), u(h, h * h), np.zeros(h), u(h, h) * 0.1,
                           np.zeros(1)]).astype(np.float32)


def train(x, y, steps=4000, batch=512, lr=2e-3, seed=0, val=None, log=print):
    """Train on the GPU with the library's kernels. x: [N, in] normalised
    float32, y: [N] normalised. Returns (params, history)."""
    import torch
    dev = torch.device("cuda")
    rng = np.random.default_rng(seed)
    p = torch.from_numpy(init_params(rng)).to(dev)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    xt = torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(dev)
    yt = torch.from_numpy(np.ascontiguousarray(y, np.float32)).to(dev)
    hist = []
    N = x.shape[0]
    for step in range(1, steps + 1):
        idx = torch.from_numpy(rng.integers(0, N, batch)).to(dev)
        xb = xt.index_select(0, idx).contiguous()
        yb = yt.index_select(0, idx).contiguous()
        grad, loss = qsim.mlp_backward(p, N_IN, N_HIDDEN, xb, yb)
        cur_lr = lr * (0.5 * (1 + math.cos(math.pi * step / steps)) * 0.9 + 0.1)
        qsim.mlp_adam(p, grad, m, v, step, cur_lr)
        if step % max(1, steps // 10) == 0 or step == 1:
            rec = {"step": step, "train_mse": float(loss.item())}
            if val is not None:
                pv = qsim.mlp_forward(p, N_IN, N_HIDDEN, torch.from_numpy(val[0]).to(dev))
                rec["val_mse"] = float(((pv.cpu().numpy() - val[1]) ** 2).mean())
            hist.append(rec)
            log(json.dumps(rec))
    return p.cpu().numpy(), hist


def cmd_train(args):
    d = np.load(args.data, allow_pickle=False)
    x, y, meta = d["x"], d["y"], d["meta"]
    held = meta[:, 0] % 5 == 4  # every fifth seed is validation
    mean = x[~held].mean(0)
    std = x[~held].std(0)
    std[std < 1e-6] = 1.0
    y_mean, y_std = float(y[~held].mean()), float(y[~held].std())
    xn = ((x - mean) / std).astype(np.float32)
    yn = ((y - y_mean) / y_std).astype(np.float32)
    params, hist = train(xn[~held], yn[~held], steps=args.steps, val=(xn[held], yn[held]))
    # validation error in log space -> typical relative error of a time prediction
    pred = qsim.mlp_predict_host(params, N_IN, N_HIDDEN, xn[held]) * y_std + y_mean
    rmse = float(np.sqrt(np.mean((pred - y[held]) ** 2)))
    mae_rel = float(np.mean(np.abs(np.exp(pred - y[held]) - 1)))
    print("validation: rmse(ln us) = %.4f, mean |relative error| = %.2f%% over %d ops" %
          (rmse, 100 * mae_rel, int(held.sum())), flush=True)
    np.savez(args.out, params=params, n_in=N_IN, n_hidden=N_HIDDEN, feat_mean=mean.astype(np.float32),
             feat_std=std.astype(np.float32), y_mean=y_mean, y_std=y_std, val_rmse_log=rmse,
             val_mean_rel_err=mae_rel, n_train=int((~held).sum()), n_val=int(held.sum()),
             history=json.dumps(hist))


def time_run(state, circ, opts, reps=3):
    best, st = None, None
    for _ in range(reps + 1):
        state.init("zero")
        state.sync()
        t0 = time.perf_counter()
        st = state.run_circuit(circ.gates, **opts)
        state.sync()
        t = time.perf_counter() - t0
        best = t if best is None or t < best else best
    return best, st


def compare(n_list=(28, 29, 30), seeds=range(100, 104), depth=40, dtype="c64", log=print):
    """Time held-out circuits with the learned scheduler (k <= 7; 6 on
    complex128 states) against the
    method without the model: the fixed-k greedy scheduler at the k_max the
    autotuner found best for this dtype and size (qsim.best_opts), and also
    greedy at k = 5 and k = 6 and the analytic model. The results of every
    schedule are checked to agree (fidelity against the tuned greedy run)."""
    import torch
    rows = []
    base = dict(fuse_diag=True, skip_trailing_diag=True, skip_initial_h=True)
    for n in n_list:
        tuned = qsim.best_opts(n, dtype)
        s1 = qsim.State(n, dtype, kmax=7)
        s2 = qsim.State(n, dtype, kmax=7)
        for seed in seeds:
            circ = workload(n, depth, seed)
            tg, stg = time_run(s1, circ, dict(base, scheduler="greedy", kmax=tuned["kmax"]))
            tl, stl = time_run(s2, circ, dict(base, scheduler="learned", kmax=7))
            fid, maxd = s1.compare(s2.amps)
            t5, st5 = time_run(s1, circ, dict(base, scheduler="greedy", kmax=5))
            t6, st6 = time_run(s1, circ, dict(base, scheduler="greedy", kmax=6))
            t7, st7 = time_run(s1, circ, dict(base, scheduler="greedy", kmax=7))
            ta, sta = time_run(s1, circ, dict(base, scheduler="analytic", kmax=7))
            row = dict(n=n, dtype=dtype, seed=seed, tuned_kmax=tuned["kmax"], tuned_greedy_ms=tg * 1e3,
                       tuned_schedule_ms=stg["schedule_ms"],
                       greedy_ms=t5 * 1e3, greedy6_ms=t6 * 1e3, greedy7_ms=t7 * 1e3, learned_ms=tl * 1e3,
                       analytic_ms=ta * 1e3,
                       tuned_greedy_ops=stg["n_ops"], greedy_ops=st5["n_ops"], greedy6_ops=st6["n_ops"],
                       greedy7_ops=st7["n_ops"],
                       learned_ops=stl["n_ops"], analytic_ops=sta["n_ops"],
                       tuned_clusters_by_k=stg["n_clusters_by_k"], learned_clusters_by_k=stl["n_clusters_by_k"],
                       learned_schedule_ms=stl["schedule_ms"], fidelity_learned_vs_greedy=fid, max_abs_diff=maxd)
            rows.append(row)
            log(json.dumps(row))
        del s1, s2
        torch.cuda.empty_cache()
    tg = sum(r["tuned_greedy_ms"] for r in rows)
    g5 = sum(r["greedy_ms"] for r in rows)
    g6 = sum(r["greedy6_ms"] for r in rows)
    g7 = sum(r["greedy7_ms"] for r in rows)
    lr = sum(r["learned_ms"] for r in rows)
    an = sum(r["analytic_ms"] for r in rows)
    log("total (%s): tuned greedy %.1f ms, greedy k=5 %.1f ms, greedy k=6 %.1f ms, greedy k=7 %.1f ms, "
        "analytic %.1f ms, learned %.1f ms (learned vs tuned greedy: %.1f%% faster)"
        % (dtype, tg, g5, g6, g7, an, lr, 100 * (tg - lr) / tg))
    return rows


def cmd_compare(args):
    import torch  # noqa: F401
    qsim.load_tuning()
    rows = compare(n_list=[int(x) for x in args.n.split(",")], seeds=range(args.seed0, args.seed0 + args.seeds),
                   dtype=args.dtype)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(rows, f, indent=1)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("record")
    r.add_argument("--seeds", type=int, default=10)
    r.add_argument("--depth", type=int, default=40)
    r.add_argument("--n", default="27,28,29,30", help="state sizes")
    r.add_argument("--dtypes", default="c64,c128")
    r.add_argument("--kmax", default="2,3,4,5,6,7", help="k_max of the recorded schedules")
    r.add_argument("--append", default=None, help="record file to extend")
    r.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--data", required=True)
    t.add_argument("--steps", type=int, default=4000)
    t.add_argument("--out", required=True)
    c = sub.add_parser("compare")
    c.add_argument("--n", default="28,29,30")
    c.add_argument("--seed0", type=int, default=100)
    c.add_argument("--seeds", type=int, default=4)
    c.add_argument("--dtype", default="c64", choices=["c64", "c128"])
    c.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    {"record": cmd_record, "train": cmd_train, "compare": cmd_compare}[args.cmd](args)


if __name__ == "__main__":
    main()
