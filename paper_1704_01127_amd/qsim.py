"""ctypes binding of libqsim.so (the C ABI in include/qsim.h).

Argument marshalling only: every step of a simulation runs in the library's
HIP kernels on the GPU. PyTorch provides the device memory (state vector and
workspace) and the stream. The binding fails loudly when the library has not
been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsim.so")

C64, C128 = 1, 2
INIT_ZERO, INIT_UNIFORM, INIT_KEEP = 0, 1, 2
SCHED_PER_GATE, SCHED_GREEDY, SCHED_ANALYTIC, SCHED_LEARNED = 0, 1, 2, 3
GATE_KIND = {"H": 0, "T": 1, "SX": 2, "SY": 3, "X": 4, "Y": 5, "Z": 6, "CZ": 7, "TDG": 8,
             "SXDG": 9, "SYDG": 10, "PHASE": 11, "U": 12}
STATUS = {0: "QSIM_OK", -1: "QSIM_E_INVALID", -2: "QSIM_E_UNSUPPORTED", -3: "QSIM_E_DEVICE"}
OK, E_INVALID, E_UNSUPPORTED, E_DEVICE = 0, -1, -2, -3
SCHEDULERS = {"per_gate": 0, "greedy": 1, "analytic": 2, "learned": 3}


class QsimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


MAX_CLUSTER = 7       # widest cluster (QSIM_MAX_CLUSTER): per-op qubit lists have this many entries
MAX_GATE_QUBITS = 6   # widest single gate


class Gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("k", ctypes.c_int32), ("qubits", ctypes.c_int32 * 6),
                ("theta", ctypes.c_double), ("mat", ctypes.POINTER(ctypes.c_double))]


class RunOpts(ctypes.Structure):
    _fields_ = [("kmax", ctypes.c_int32), ("scheduler", ctypes.c_int32),
                ("skip_trailing_diag", ctypes.c_int32), ("fuse_diag", ctypes.c_int32),
                ("skip_initial_h", ctypes.c_int32), ("record_timings", ctypes.c_int32),
                ("schedule_dtype", ctypes.c_int32), ("fused_stats", ctypes.c_int32)]


class RunStats(ctypes.Structure):
    _fields_ = [("n_ops", ctypes.c_int32), ("n_clusters_by_k", ctypes.c_int32 * 8),
                ("n_diag_ops", ctypes.c_int32), ("n_gates_applied", ctypes.c_int32),
                ("n_gates_fused_epilogue", ctypes.c_int32), ("schedule_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double)]

    def as_dict(self):
        return dict(n_ops=self.n_ops, n_clusters_by_k=list(self.n_clusters_by_k),
                    n_diag_ops=self.n_diag_ops, n_gates_applied=self.n_gates_applied,
                    n_gates_fused_epilogue=self.n_gates_fused_epilogue,
                    schedule_ms=self.schedule_ms, total_ms=self.total_ms)


class StageOpts(ctypes.Structure):
    _fields_ = [("n_local", ctypes.c_int32), ("specialize", ctypes.c_int32), ("search", ctypes.c_int32),
                ("early_swaps", ctypes.c_int32), ("kmax", ctypes.c_int32), ("fuse_diag", ctypes.c_int32),
                ("skip_initial_h", ctypes.c_int32), ("skip_trailing_diag", ctypes.c_int32)]


class BatchCircuit(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_gates", ctypes.c_int32), ("gates", ctypes.POINTER(Gate)),
                ("dev_amps", ctypes.c_void_p)]


class BatchStats(ctypes.Structure):
    _fields_ = [("n_circuits", ctypes.c_int32), ("n_ops", ctypes.c_int32), ("n_clusters", ctypes.c_int32),
                ("n_items", ctypes.c_int32), ("grid", ctypes.c_int32), ("n_gates_applied", ctypes.c_int32),
                ("plan_ms", ctypes.c_double), ("run_ms", ctypes.c_double), ("workspace_bytes", ctypes.c_size_t)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def lib():
    """Load libqsim.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libqsim.so is not built: run `python -c 'import __graft_entry__ as g; "
                              "g.build()'` (hipcc, gfx950) first")
        # PyTorch ships its own HIP runtime; load it first so that the library
        # binds to the same runtime instead of mapping a second one.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32p, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
        sig = {
            "qsim_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
            "qsim_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, vp,
                                           ctypes.c_size_t, vp, ctypes.c_int, ctypes.POINTER(vp)]),
            "qsim_destroy": (ctypes.c_int, [vp]),
            "qsim_init_state": (ctypes.c_int, [vp, ctypes.c_int]),
            "qsim_apply_cluster": (ctypes.c_int, [vp, ctypes.c_int, i32p, dp]),
            "qsim_apply_diag": (ctypes.c_int, [vp, ctypes.c_int, i32p, ctypes.c_int, i32p, dp]),
            "qsim_apply_gate": (ctypes.c_int, [vp, ctypes.POINTER(Gate)]),
            "qsim_run_circuit": (ctypes.c_int, [vp, ctypes.POINTER(Gate), ctypes.c_int,
                                                ctypes.POINTER(RunOpts), ctypes.POINTER(RunStats)]),
            "qsim_probs": (ctypes.c_int, [vp, vp, ctypes.c_int, dp, dp, dp]),
            "qsim_compare": (ctypes.c_int, [vp, vp, ctypes.c_int, dp, dp]),
            "qsim_sync": (ctypes.c_int, [vp]),
            "qsim_state_changed": (ctypes.c_int, [vp]),
            "qsim_permute_qubits": (ctypes.c_int, [vp, ctypes.c_int, i32p, i32p]),
            "qsim_probs_noalloc": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, vp, ctypes.c_size_t, vp, vp,
                                                  ctypes.c_int, dp, dp, dp]),
            "qsim_noalloc_scratch_bytes": (ctypes.c_size_t, []),
            "qsim_last_error": (ctypes.c_char_p, []),
            "qsim_op_timings": (ctypes.c_int, [vp, i32p, i32p, i32p, i32p, ctypes.POINTER(ctypes.c_float),
                                               ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
            "qsim_set_option": (ctypes.c_int, [ctypes.c_int, ctypes.c_int]),
            "qsim_set_cost_table": (ctypes.c_int, [ctypes.c_int, dp, ctypes.c_int]),
            "qsim_cost_feature_count": (ctypes.c_int, []),
            "qsim_cost_features": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, i32p, ctypes.c_int,
                                                  ctypes.POINTER(ctypes.c_float)]),
            "qsim_mlp_param_count": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int]),
            "qsim_set_cost_model": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_double,
                                                   ctypes.c_double]),
            "qsim_cost_model_predict_us": (ctypes.c_double, [ctypes.c_int, ctypes.c_int, ctypes.c_int, i32p,
                                                             ctypes.c_int]),
            "qsim_mlp_predict_host": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int, vp]),
            "qsim_mlp_scratch_floats": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
            "qsim_mlp_forward": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, vp, vp, ctypes.c_int, vp, vp]),
            "qsim_mlp_backward": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, vp, vp, vp, ctypes.c_int, vp, vp, vp,
                                                 vp]),
            "qsim_mlp_adam": (ctypes.c_int, [ctypes.c_int, vp, vp, vp, vp, ctypes.c_int, ctypes.c_float,
                                             ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]),
            "qsim_set_tune_entry": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
            "qsim_get_tune_entry": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
            "qsim_get_option": (ctypes.c_int, [ctypes.c_int]),
            "qsim_schedule": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(Gate), ctypes.c_int,
                                             ctypes.POINTER(RunOpts), i32p, i32p, i32p, i32p, i32p,
                                             ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
        }
        sig.update({
            "qsim_stage_schedule": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(Gate), ctypes.c_int,
                                                   ctypes.POINTER(StageOpts), i32p, i32p, i32p, ctypes.c_int,
                                                   ctypes.POINTER(ctypes.c_int)]),
            "qsim_batch_plan": (ctypes.c_int, [ctypes.POINTER(BatchCircuit), ctypes.c_int, ctypes.POINTER(RunOpts),
                                               ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_size_t)]),
            "qsim_batch_run": (ctypes.c_int, [vp, vp, ctypes.c_size_t, vp, ctypes.c_uint32,
                                              ctypes.POINTER(BatchStats)]),
            "qsim_batch_destroy": (ctypes.c_int, [vp]),
        })
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise QsimError(status, lib().qsim_last_error().decode())


def _i32(seq) -> ctypes.Array:
    seq = list(seq)
    return (ctypes.c_int32 * max(1, len(seq)))(*seq)


def gate_array(gates: Sequence) -> tuple:
    """Marshal gates (objects with .name, .qubits and .mat, or tuples
    (name, qubits[, mat or theta])) into a qsim_gate array. Returns the array
    and the list of numpy buffers it points into (keep it alive)."""
    arr = (Gate * max(1, len(gates)))()
    keep = []
    for i, g in enumerate(gates):
        if isinstance(g, tuple):
            name, qubits = g[0], tuple(g[1])
            extra = g[2] if len(g) > 2 else None
        else:
            name, qubits, extra = g.name, tuple(g.qubits), getattr(g, "mat", None)
        arr[i].kind = GATE_KIND[name]
        arr[i].k = len(qubits)
        if len(qubits) > MAX_GATE_QUBITS:
            raise ValueError("a gate acts on at most %d qubits" % MAX_GATE_QUBITS)
        for j, q in enumerate(qubits):
            arr[i].qubits[j] = int(q)
        if name == "U":
            m = np.ascontiguousarray(extra, dtype=np.complex128)
            if m.shape != (2 ** len(qubits), 2 ** len(qubits)):
                raise ValueError("dense gate matrix must be 2^k x 2^k")
            keep.append(m)
            arr[i].mat = m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        elif name == "PHASE":
            arr[i].theta = float(extra)
    return arr, keep


class Gates:
    """A gate list already in the library's qsim_gate layout (gate_array),
    for callers that run the same circuit repeatedly: run_circuit and
    schedule take it in place of a gate sequence and pass the array as is."""

    def __init__(self, gates: Sequence):
        self.arr, self.keep = gate_array(gates)
        self.n = len(gates)

    def __len__(self) -> int:
        return self.n


def _as_array(gates) -> tuple:
    """(qsim_gate array, count, buffers to keep alive) of a Gates or a sequence."""
    if isinstance(gates, Gates):
        return gates.arr, gates.n, gates.keep
    arr, keep = gate_array(gates)
    return arr, len(gates), keep


def run_opts(kmax=5, scheduler="greedy", fuse_diag=False, skip_trailing_diag=False,
             skip_initial_h=False, record_timings=False, fused_stats=False) -> RunOpts:
    o = RunOpts()
    o.kmax = kmax
    o.scheduler = SCHEDULERS[scheduler] if isinstance(scheduler, str) else int(scheduler)
    o.fuse_diag = int(fuse_diag)
    o.skip_trailing_diag = int(skip_trailing_diag)
    o.skip_initial_h = int(skip_initial_h)
    o.record_timings = int(record_timings)
    o.fused_stats = int(fused_stats)
    return o


def schedule(n: int, gates, dtype: int = C64, **opts) -> dict:
    """Host-only: the schedule the library would run (no GPU needed); gates
    as a sequence or a prepared Gates."""
    arr, ng, keep = _as_array(gates)
    o = run_opts(**opts)
    o.schedule_dtype = dtype
    cap = max(1, ng)
    gate_op = (ctypes.c_int32 * max(1, ng))()
    gate_role = (ctypes.c_int32 * max(1, ng))()
    op_kind = (ctypes.c_int32 * cap)()
    op_k = (ctypes.c_int32 * cap)()
    op_q = (ctypes.c_int32 * (MAX_CLUSTER * cap))()
    nops = ctypes.c_int()
    _check(lib().qsim_schedule(n, arr, ng, ctypes.byref(o), gate_op, gate_role, op_kind, op_k, op_q,
                               cap, ctypes.byref(nops)))
    m = nops.value
    return dict(gate_op=list(gate_op)[:ng], gate_role=list(gate_role)[:ng], op_kind=list(op_kind)[:m],
                op_k=list(op_k)[:m],
                op_qubits=[list(op_q[MAX_CLUSTER * o_:MAX_CLUSTER * (o_ + 1)]) for o_ in range(m)])


def stage_schedule(n: int, gates: Sequence, n_local: int, specialize: int = 1, search: bool = True,
                   early_swaps: bool = True, kmax: int = 5, fuse_diag: bool = False, skip_initial_h: bool = True,
                   skip_trailing_diag: bool = True) -> dict:
    """Host-only: stages of a circuit on 2^(n - n_local) memories
    (qsim_stage_schedule). Returns gate_stage, stage_loc (per stage, the bit
    location of every qubit), stage_clusters and n_swaps."""
    arr, keep = gate_array(gates)
    o = StageOpts(n_local, specialize, int(search), int(early_swaps), kmax, int(fuse_diag), int(skip_initial_h),
                  int(skip_trailing_diag))
    ng = len(gates)
    ns = ctypes.c_int()
    L = lib()
    st = L.qsim_stage_schedule(n, arr, ng, ctypes.byref(o), None, None, None, 0, ctypes.byref(ns))
    if st not in (OK, E_INVALID) or ns.value <= 0:
        _check(st)
    m = ns.value
    gate_stage = (ctypes.c_int32 * max(1, ng))()
    loc = (ctypes.c_int32 * (m * n))()
    clus = (ctypes.c_int32 * m)()
    _check(L.qsim_stage_schedule(n, arr, ng, ctypes.byref(o), gate_stage, loc, clus, m, ctypes.byref(ns)))
    return dict(gate_stage=list(gate_stage)[:ng], stage_loc=[list(loc[s * n:(s + 1) * n]) for s in range(m)],
                stage_clusters=list(clus)[:m], n_swaps=m - 1)


OPT_CLUSTER_VARIANT = 1
OPT_BATCH_GRID = 2
OPT_BATCH_PAD = 3
OPT_BATCH_ITEM_TILES = 4
OPT_K6_KERNEL = 5
OPT_FOLD_INIT = 6
OPT_PAIR = 7
OPT_PAIR_TILE = 8
OPT_CLUSTER_SETS = 9
OPT_BATCH_ORDER = 10
OPT_CHECK_UNITARY = 11
OPT_MAP_QUBITS = 12
OPT_FOLD_TABLE = 13
OPT_DEVIATIONS = 14


def set_option(option: int, value: int):
    _check(lib().qsim_set_option(option, value))


def get_option(option: int) -> int:
    return int(lib().qsim_get_option(option))


def set_cost_table(dtype: int, us_by_k, n_ref: int):
    """Analytic scheduler costs: us_by_k[k] microseconds per op at n_ref qubits
    (k = 0: diagonal pass, 1..7). A table without the k = 7 entry (7 values)
    prices 7-qubit clusters as 6-qubit ones."""
    us = [float(x) for x in us_by_k]
    if len(us) == MAX_CLUSTER:
        us.append(us[-1])
    if len(us) != MAX_CLUSTER + 1:
        raise ValueError("cost table needs %d or %d entries" % (MAX_CLUSTER, MAX_CLUSTER + 1))
    a = (ctypes.c_double * (MAX_CLUSTER + 1))(*us)
    _check(lib().qsim_set_cost_table(dtype, a, n_ref))


def cost_features(n: int, dtype: int, qubits, n_epi: int = 0) -> np.ndarray:
    """Feature vector of an op as the library computes it (k = len(qubits), sorted)."""
    L = lib()
    out = np.zeros(L.qsim_cost_feature_count(), np.float32)
    qs = sorted(int(q) for q in qubits)
    _check(L.qsim_cost_features(n, dtype, len(qs), _i32(qs), n_epi,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return out


def _fp(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def set_cost_model(params=None, n_in=0, n_hidden=0, feat_mean=None, feat_std=None, y_mean=0.0, y_std=1.0):
    """Load (or with params=None unload) the learned cost model into the scheduler."""
    if params is None:
        _check(lib().qsim_set_cost_model(None, 0, 0, None, None, 0.0, 1.0))
        return
    p = np.ascontiguousarray(params, np.float32)
    m = np.ascontiguousarray(feat_mean, np.float32)
    sd = np.ascontiguousarray(feat_std, np.float32)
    _check(lib().qsim_set_cost_model(_fp(p), n_in, n_hidden, _fp(m), _fp(sd), float(y_mean), float(y_std)))


def cost_model_predict_us(n: int, dtype: int, qubits, n_epi: int = 0) -> float:
    qs = sorted(int(q) for q in qubits)
    return float(lib().qsim_cost_model_predict_us(n, dtype, len(qs), _i32(qs), n_epi))


def mlp_param_count(n_in: int, n_hidden: int) -> int:
    return int(lib().qsim_mlp_param_count(n_in, n_hidden))


def mlp_predict_host(params: np.ndarray, n_in: int, n_hidden: int, x: np.ndarray) -> np.ndarray:
    p = np.ascontiguousarray(params, np.float32)
    xx = np.ascontiguousarray(x, np.float32)
    y = np.zeros(xx.shape[0], np.float32)
    _check(lib().qsim_mlp_predict_host(_fp(p), n_in, n_hidden, _fp(xx), xx.shape[0], _fp(y)))
    return y


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


def mlp_forward(params, n_in: int, n_hidden: int, x, stream=None):
    """GPU forward pass (torch float32 device tensors); returns y [batch]."""
    import torch
    y = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    st = stream if stream is not None else torch.cuda.current_stream(x.device)
    _check(lib().qsim_mlp_forward(n_in, n_hidden, _dptr(params), _dptr(x), x.shape[0], _dptr(y),
                                  ctypes.c_void_p(st.cuda_stream)))
    return y


def mlp_backward(params, n_in: int, n_hidden: int, x, target, stream=None):
    """GPU gradient of the mean squared error; returns (grad [P], loss [1])."""
    import torch
    P = mlp_param_count(n_in, n_hidden)
    grad = torch.empty(P, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    scratch = torch.empty(int(lib().qsim_mlp_scratch_floats(n_in, n_hidden, x.shape[0])), dtype=torch.float32,
                          device=x.device)
    st = stream if stream is not None else torch.cuda.current_stream(x.device)
    _check(lib().qsim_mlp_backward(n_in, n_hidden, _dptr(params), _dptr(x), _dptr(target), x.shape[0],
                                   _dptr(grad), _dptr(loss), _dptr(scratch), ctypes.c_void_p(st.cuda_stream)))
    return grad, loss


def mlp_adam(params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(params.device)
    _check(lib().qsim_mlp_adam(params.numel(), _dptr(params), _dptr(grad), _dptr(m), _dptr(v), step, lr, beta1,
                               beta2, eps, ctypes.c_void_p(st.cuda_stream)))


def workspace_bytes(n: int, dtype: int, kmax: int = MAX_CLUSTER) -> int:
    return int(lib().qsim_workspace_bytes(n, dtype, kmax))


TUNE_PATH = os.path.join(_HERE, "tune_table.json")
COST_MODEL_PATH = os.path.join(_HERE, "cost_model.npz")
_tuning = {"loaded": False, "table": None, "model": None}


def load_tuning(path: Optional[str] = None, model_path: Optional[str] = None) -> dict:
    """Apply the autotuner's table (kernel variants, analytic costs) and the
    learned cost model, if their files exist. Called once by State()."""
    import json
    path = path or TUNE_PATH
    model_path = model_path or COST_MODEL_PATH
    if os.path.exists(path):
        with open(path) as f:
            t = json.load(f)
        L = lib()
        for dt, rows in t.get("variants", {}).items():
            code = C64 if dt == "c64" else C128
            for k, row in rows.items():
                for cls, v in enumerate(row):
                    _check(L.qsim_set_tune_entry(code, int(k), cls, int(v)))
        for dt, us in t.get("cost_us", {}).items():
            set_cost_table(C64 if dt == "c64" else C128, us, int(t["n_ref"]))
        if "batch" in t:  # launch shape of the batched kernel
            set_option(OPT_BATCH_ITEM_TILES, int(t["batch"]["item_tiles"]))
            set_option(OPT_BATCH_GRID, int(t["batch"]["grid"]))
            set_option(OPT_BATCH_PAD, int(t["batch"]["pad"]))
        _tuning["table"] = t
    if os.path.exists(model_path):
        m = np.load(model_path, allow_pickle=False)
        set_cost_model(m["params"], int(m["n_in"]), int(m["n_hidden"]), m["feat_mean"], m["feat_std"],
                       float(m["y_mean"]), float(m["y_std"]))
        _tuning["model"] = model_path
    _tuning["loaded"] = True
    return _tuning


def best_opts(n: int, dtype: str = "c64") -> dict:
    """(scheduler, kmax) the autotuner found fastest for the nearest size
    bucket at or below n (greedy, kmax 5 without a tune table)."""
    t = _tuning.get("table") or {}
    best = t.get("best", {}).get(dtype, {})
    sizes = sorted(int(x) for x in best)
    pick = [s for s in sizes if s <= n]
    if not pick:
        return dict(scheduler="greedy", kmax=5)
    b = best[str(pick[-1])]
    return dict(scheduler=b["scheduler"], kmax=int(b["kmax"]))


class State:
    """An n-qubit state vector in HBM (torch complex64 / complex128 tensor)."""

    def __init__(self, n: int, dtype: str = "c64", init: str = "zero", kmax: int = MAX_CLUSTER,
                 amps=None, stream=None, device: int = 0):
        import torch
        if not _tuning["loaded"] and not os.environ.get("QSIM_NO_TUNING"):
            load_tuning()
        self.n = n
        self.dt = C64 if dtype in ("c64", "complex64") else C128
        tdt = torch.complex64 if self.dt == C64 else torch.complex128
        dev = torch.device("cuda", device)
        self.amps = amps if amps is not None else torch.empty(2 ** n, dtype=tdt, device=dev)
        if self.amps.dtype != tdt or self.amps.numel() != 2 ** n or not self.amps.is_contiguous():
            raise ValueError("amps must be a contiguous %s tensor of 2^n elements" % tdt)
        self.workspace = torch.empty(workspace_bytes(n, self.dt, kmax), dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        initc = {"zero": INIT_ZERO, "uniform": INIT_UNIFORM, "keep": INIT_KEEP}[init]
        _check(lib().qsim_create(n, self.dt, ctypes.c_void_p(self.amps.data_ptr()),
                                 self.amps.numel() * self.amps.element_size(),
                                 ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                 ctypes.c_void_p(self.stream.cuda_stream), initc, ctypes.byref(h)))
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.qsim_destroy(h)
            self.h = None

    # -- state I/O (torch copies; no simulation arithmetic)
    def set_amps(self, values):
        import torch
        t = torch.as_tensor(values).to(self.amps.dtype)
        self.amps.copy_(t.to(self.amps.device))
        _check(lib().qsim_state_changed(self.h))

    def to_numpy(self) -> np.ndarray:
        self.sync()
        return self.amps.cpu().numpy()

    def init(self, init: str = "zero"):
        _check(lib().qsim_init_state(self.h, {"zero": INIT_ZERO, "uniform": INIT_UNIFORM}[init]))

    # -- operations
    def apply_cluster(self, qubits: Sequence[int], mat: np.ndarray):
        m = np.ascontiguousarray(mat, dtype=np.complex128)
        _check(lib().qsim_apply_cluster(self.h, len(qubits), _i32(qubits),
                                        m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def apply_diag(self, pairs: Iterable = (), phases: Iterable = ()):
        pairs = list(pairs)
        phases = list(phases)
        flat = [q for p in pairs for q in p]
        th = (ctypes.c_double * max(1, len(phases)))(*[float(t) for _, t in phases])
        _check(lib().qsim_apply_diag(self.h, len(pairs), _i32(flat), len(phases),
                                     _i32([q for q, _ in phases]), th))

    def permute_qubits(self, src: Sequence[int], dst: Sequence[int]):
        """Move the bit at location src[j] to location dst[j] (qsim_permute_qubits)."""
        if len(src) != len(dst):
            raise ValueError("src and dst must have the same length")
        _check(lib().qsim_permute_qubits(self.h, len(src), _i32(src), _i32(dst)))

    def apply_gate(self, gate):
        arr, keep = gate_array([gate])
        _check(lib().qsim_apply_gate(self.h, arr))

    def run_circuit(self, gates, **opts) -> dict:
        """Runs a gate sequence or a prepared Gates (same result)."""
        arr, ng, keep = _as_array(gates)
        o = run_opts(**opts)
        st = RunStats()
        _check(lib().qsim_run_circuit(self.h, arr, ng, ctypes.byref(o), ctypes.byref(st)))
        return st.as_dict()

    def probs(self, out=None):
        """(norm, sum p^2, entropy in nats); fills `out` (float32 or float64
        tensor of 2^n) with p_i when given."""
        import torch
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        ptr, odt = None, C64
        if out is not None:
            if out.numel() != 2 ** self.n or out.dtype not in (torch.float32, torch.float64):
                raise ValueError("out must hold 2^n float32 or float64")
            ptr, odt = ctypes.c_void_p(out.data_ptr()), (C64 if out.dtype == torch.float32 else C128)
        _check(lib().qsim_probs(self.h, ptr, odt, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def compare(self, ref) -> tuple:
        """(fidelity, max |psi - ref|) against a device tensor, in float64 on the GPU."""
        import torch
        dt = C64 if ref.dtype == torch.complex64 else C128
        if ref.numel() != 2 ** self.n or not ref.is_contiguous() or not ref.is_cuda:
            raise ValueError("ref must be a contiguous device tensor of 2^n amplitudes")
        f, m = ctypes.c_double(), ctypes.c_double()
        _check(lib().qsim_compare(self.h, ctypes.c_void_p(ref.data_ptr()), dt, ctypes.byref(f),
                                  ctypes.byref(m)))
        return f.value, m.value

    def op_timings(self) -> list:
        """Per-launch records of the last run with record_timings=True:
        dicts with kind, k, qubits, epi flags, n_epi and ms (HIP events on the
        state's stream); table: a folded start in its table form."""
        n = ctypes.c_int()
        L = lib()
        L.qsim_op_timings(self.h, None, None, None, None, None, 0, ctypes.byref(n))  # count only
        m = n.value
        if m == 0:
            return []
        kind, k, epi = (ctypes.c_int32 * m)(), (ctypes.c_int32 * m)(), (ctypes.c_int32 * m)()
        qs, ms = (ctypes.c_int32 * (MAX_CLUSTER * m))(), (ctypes.c_float * m)()
        _check(L.qsim_op_timings(self.h, kind, k, qs, epi, ms, m, ctypes.byref(n)))
        kinds = {0: "cluster", 1: "diag", 2: "gate1q", 3: "phase1q", 4: "cz", 5: "build", 6: "init_cluster",
                 8: "init_cluster2",
                 7: "pair", 9: "permute"}
        return [dict(kind=kinds[kind[i]], k=k[i], qubits=[q for q in qs[MAX_CLUSTER * i:MAX_CLUSTER * (i + 1)] if q >= 0],
                     epi=bool(epi[i] & 1), staged=bool(epi[i] & 2), mfma=bool(epi[i] & 4),
                     stats=bool(epi[i] & 8), table=bool(epi[i] & 16), n_epi=(epi[i] >> 8) & 255,
                     ms=float(ms[i]))
                for i in range(m)]

    def sync(self):
        _check(lib().qsim_sync(self.h))


def probs_noalloc(amps, out=None, stream=None) -> tuple:
    """qsim_probs_noalloc on a device tensor of 2^n complex amplitudes: (norm,
    sum p^2, entropy in nats), and p_i into `out` (float32 / float64, 2^n)
    when given. Uses the library's fixed device scratch, no workspace."""
    import torch
    n = int(amps.numel()).bit_length() - 1
    if amps.numel() != 2 ** n or not amps.is_contiguous() or amps.dtype not in (torch.complex64, torch.complex128):
        raise ValueError("amps must be a contiguous complex64/complex128 device tensor of 2^n elements")
    dt = C64 if amps.dtype == torch.complex64 else C128
    ptr, odt = None, C64
    if out is not None:
        if out.numel() != 2 ** n or out.dtype not in (torch.float32, torch.float64):
            raise ValueError("out must hold 2^n float32 or float64")
        ptr, odt = ctypes.c_void_p(out.data_ptr()), (C64 if out.dtype == torch.float32 else C128)
    st = stream if stream is not None else torch.cuda.current_stream(amps.device)
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().qsim_probs_noalloc(n, dt, ctypes.c_void_p(amps.data_ptr()), amps.numel() * amps.element_size(),
                                    ctypes.c_void_p(st.cuda_stream), ptr, odt, ctypes.byref(a), ctypes.byref(b),
                                    ctypes.byref(c)))
    return a.value, b.value, c.value


class Batch:
    """Many independent circuits run by one persistent launch (complex64).

    circuits: objects with .n and .gates (or (n, gates) tuples). The states
    are torch complex64 tensors (self.states[i]) owned here, as is the
    workspace; plan at construction, run() as often as wanted. kmax: largest
    cluster (1..6); None takes the tune table's batch choice (else 5)."""

    def __init__(self, circuits: Sequence, kmax: Optional[int] = None, scheduler: str = "greedy",
                 fuse_diag: bool = True, skip_trailing_diag: bool = False, skip_initial_h: bool = True, stream=None,
                 device: int = 0):
        import torch
        if not _tuning["loaded"] and not os.environ.get("QSIM_NO_TUNING"):
            load_tuning()
        if kmax is None:
            t = _tuning["table"] or {}
            kmax = int(t.get("batch", {}).get("kmax", 5))
        self.kmax = kmax
        dev = torch.device("cuda", device)
        self.ns = [int(c[0] if isinstance(c, tuple) else c.n) for c in circuits]
        gate_lists = [c[1] if isinstance(c, tuple) else c.gates for c in circuits]
        self.states = [torch.empty(2 ** n, dtype=torch.complex64, device=dev) for n in self.ns]
        arr = (BatchCircuit * max(1, len(circuits)))()
        keep = []
        for i, (n, gl) in enumerate(zip(self.ns, gate_lists)):
            ga, kp = gate_array(gl)
            keep.append((ga, kp))
            arr[i].n_qubits = n
            arr[i].n_gates = len(gl)
            arr[i].gates = ctypes.cast(ga, ctypes.POINTER(Gate))
            arr[i].dev_amps = self.states[i].data_ptr()
        o = run_opts(kmax=kmax, scheduler=scheduler, fuse_diag=fuse_diag, skip_trailing_diag=skip_trailing_diag,
                     skip_initial_h=skip_initial_h)
        h = ctypes.c_void_p()
        wsb = ctypes.c_size_t()
        _check(lib().qsim_batch_plan(arr, len(circuits), ctypes.byref(o), ctypes.byref(h), ctypes.byref(wsb)))
        self.h = h
        self.workspace = torch.empty(max(256, wsb.value), dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.qsim_batch_destroy(h)
            self.h = None

    def run(self, wait_limit_us: int = 0) -> dict:
        """Initialise and run every circuit; returns the launch statistics.
        wait_limit_us bounds each dependency wait (0: the library default)."""
        st = BatchStats()
        _check(lib().qsim_batch_run(self.h, ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                    ctypes.c_void_p(self.stream.cuda_stream), wait_limit_us, ctypes.byref(st)))
        return st.as_dict()

