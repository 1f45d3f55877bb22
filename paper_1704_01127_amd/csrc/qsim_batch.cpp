// Batched persistent launch (C ABI in include/qsim.h): many independent
// circuits, each scheduled into clusters (Sec. 3.6, step 2), applied by one
// persistent matrix-core kernel that takes work items from an atomic counter.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <future>
#include <queue>
#include <thread>
#include <vector>

#include "api_common.h"
#include "qsim.h"
#include "qsim_internal.h"
#include "scheduler.h"

using namespace qsim;
using namespace qsim::api;

namespace {

constexpr int kBatchK = 5;                           // smaller clusters are padded to 5 targets
constexpr int kBatchC = 6;                           // column bits of a 5-qubit tile
constexpr int kTileBits = kBatchK + kBatchC;         // 2^11 amplitudes per tile (6 + 5 for 6-qubit ops)
constexpr int kBatchMinQ = kTileBits;                // smallest state: one tile
constexpr int kBatchMaxQ = 30;
constexpr uint32_t kDefaultWaitUs = 10u * 1000 * 1000;  // longest dependency wait: 10 s

// One circuit's packed ops, built independently of the others.
struct Packed {
    std::vector<BatchOp> ops;      // psi / A / epi filled at run time
    std::vector<int> op_mat;       // per op: index into bops (-1: initialisation)
    std::vector<int64_t> mat_bytes;  // per bop: size of its matrix
    std::vector<int> op_epi;       // per op: index into epis (-1: none)
    std::vector<BuildOp> bops;     // gate0 relative to bgates, out_off unset
    std::vector<BuildGate> bgates; // dense_off relative to dense
    std::vector<double> dense;
    std::vector<EpiDesc> epis;
    int n_applied = 0;
    qsim_status st = QSIM_OK;
    std::string err;
};

// The five targets of a padded cluster: the op's qubits plus identity qubits.
void pad_targets(int n, const int* q, int k, int pad_policy, int* t) {
    uint64_t m = 0;
    for (int j = 0; j < k; ++j) m |= uint64_t(1) << q[j];
    int cnt = k;
    for (int j = 0; j < k; ++j) t[j] = q[j];
    if (pad_policy == 0) {
        for (int b = 0; b < n && cnt < kBatchK; ++b)
            if (!(m >> b & 1)) t[cnt++] = b;
    } else {
        for (int b = n - 1; b >= 0 && cnt < kBatchK; --b)
            if (!(m >> b & 1)) t[cnt++] = b;
    }
    std::sort(t, t + kBatchK);
}

Packed pack_circuit(const qsim_batch_circuit& c, const qsim_run_opts* opts, int circuit, int pad_policy) {
    Packed P;
    const int n = c.n_qubits;
    const std::vector<SGate> sg = to_sgates(c.gates, c.n_gates);
    SchedOpts so = to_sched_opts(opts);
    so.parallel = false;  // circuits are already planned on parallel threads
    const Schedule S = make_schedule(n, sg, so, cost_fn(opts, n, false));
    P.n_applied = S.n_applied;
    const uint64_t tiles = uint64_t(1) << (n - kTileBits);

    // from the uniform start with a cluster first, the start and that cluster
    // are one write-only op
    const bool fold = S.uniform_init && g_fold_init && !S.ops.empty() && S.ops[0].kind == OP_CLUSTER;
    if (!fold) {
        BatchOp init;
        std::memset(&init, 0, sizeof(init));
        init.kind = S.uniform_init ? 2 : 1;
        init.circuit = circuit;
        init.n = n;
        init.tiles = tiles;
        P.ops.push_back(init);
        P.op_mat.push_back(-1);
        P.op_epi.push_back(-1);
    }

    for (size_t oi = 0; oi < S.ops.size(); ++oi) {
        const SOp& op = S.ops[oi];
        const bool first_folded = fold && oi == 0;
        if (op.kind == OP_GATE) {
            P.st = QSIM_E_UNSUPPORTED;
            P.err = "per-gate ops are not batched";
            return P;
        }
        int q[kMaxK], t[kMaxK];
        int k = 0;
        std::vector<int> members, epi;
        if (op.kind == OP_CLUSTER) {
            k = op.k;
            for (int j = 0; j < k; ++j) q[j] = op.qubits[j];
            members = op.members;
            epi = op.epi;
        } else {
            // a diagonal pass: identity cluster whose store applies every gate
            epi = op.members;
        }
        if (k > 6) {
            P.st = QSIM_E_UNSUPPORTED;
            P.err = "batched clusters have at most 6 qubits";
            return P;
        }
        // 6-qubit clusters keep their targets (fp16-halves kernel); smaller
        // ones are padded to 5 (fp32 real-split kernel)
        const int kk = k == 6 ? 6 : kBatchK;
        if (k == 6) {
            for (int j = 0; j < 6; ++j) t[j] = q[j];
            std::sort(t, t + 6);
        } else {
            pad_targets(n, q, k, pad_policy, t);
        }
        int pos_of[64];
        for (int i = 0; i < 64; ++i) pos_of[i] = -1;
        for (int j = 0; j < kk; ++j) pos_of[t[j]] = j;

        BuildOp bo;
        std::memset(&bo, 0, sizeof(bo));
        bo.k = kk;
        bo.gate0 = (int)P.bgates.size();
        bo.layout = first_folded ? LAYOUT_PLAIN : kk == 6 ? LAYOUT_SPLIT16F : LAYOUT_MFMA32F;
        bo.is_double = first_folded ? 1 : 0;
        for (int gi : members) P.bgates.push_back(to_build_gate(c.gates[gi], pos_of, P.dense));
        EpiDesc e;
        if (qsim_status r = split_epilogue(pos_of, c.gates, epi, P.bgates, P.dense, e)) {
            P.st = r;
            P.err = "circuit " + std::to_string(circuit) + ": epilogue too long";
            return P;
        }
        bo.n_gates = (int)P.bgates.size() - bo.gate0;

        ClusterGeom g;
        std::memset(&g, 0, sizeof(g));
        for (int j = 0; j < kk; ++j) g.t[j] = t[j];
        g.n = n;
        g.k = kk;
        g.ncols = uint64_t(1) << (n - kk);
        BatchOp b;
        std::memset(&b, 0, sizeof(b));
        b.sg = make_stage_geom(g, kTileBits - kk, 7);  // 11 tile bits either way
        b.tiles = tiles;
        b.kind = first_folded ? 4 : kk == 6 ? 3 : 0;
        b.k = (uint32_t)kk;
        b.circuit = circuit;
        b.lowt = t[0] == 0;
        b.n = n;
        P.op_mat.push_back((int)P.bops.size());
        P.bops.push_back(bo);
        P.mat_bytes.push_back(matrix_bytes(kk, bo.layout, bo.is_double != 0));
        if (e.n_cc || e.n_mix || e.n_ph) {
            P.op_epi.push_back((int)P.epis.size());
            P.epis.push_back(e);
        } else {
            P.op_epi.push_back(-1);
        }
        P.ops.push_back(b);
    }
    return P;
}

}  // namespace

struct qsim_batch_s {
    int n_circuits = 0;
    std::vector<void*> amps;
    std::vector<BatchOp> ops;
    std::vector<int> op_mat, op_epi;
    std::vector<int64_t> mat_off;  // per bop: byte offset of its matrix in the matrix region
    int64_t mat_total = 0;
    std::vector<BatchItem> items;
    std::vector<BuildOp> bops;
    std::vector<BuildGate> bgates;
    std::vector<double> dense;
    std::vector<EpiDesc> epis;
    int n_applied = 0;
    uint32_t item_tiles = 128;
    double plan_ms = 0;
    // workspace layout (byte offsets)
    size_t off_ops = 0, off_items = 0, off_epis = 0, off_bops = 0, off_bgates = 0, off_dense = 0, off_mats = 0;
    size_t ws_bytes = 0;
};

namespace {
// Work-item (ticket) orders. Any order in which every op's items come after
// all items of its circuit's previous op is free of deadlock: an item waits
// only for items with smaller tickets.
//
// Level order: the j-th op of every circuit before any (j+1)-th, larger
// states first within a level.
void order_items_by_level(qsim_batch_s* b, const qsim_batch_circuit* circuits, const std::vector<Packed>& packed,
                          const std::vector<int>& op0, int n_circuits) {
    std::vector<int> order(n_circuits);
    for (int i = 0; i < n_circuits; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return circuits[x].n_qubits > circuits[y].n_qubits; });
    size_t levels = 0;
    for (int i = 0; i < n_circuits; ++i) levels = std::max(levels, packed[i].ops.size());
    for (size_t lv = 0; lv < levels; ++lv)
        for (int i : order) {
            if (lv >= packed[i].ops.size()) continue;
            const BatchOp& op = b->ops[op0[i] + lv];
            const uint64_t n_it = (op.tiles + b->item_tiles - 1) / b->item_tiles;
            for (uint64_t it = 0; it < n_it; ++it)
                b->items.push_back(BatchItem{(uint32_t)(op0[i] + lv), (uint32_t)(it * b->item_tiles)});
        }
}

// Critical path first: list scheduling of the items on kSimGroups simulated
// work-groups, an item taking time proportional to its tiles plus a fixed
// cost. An op's items become available when every item of the circuit's
// previous op has finished; a free work-group takes the available item whose
// circuit has the longest remaining chain (its remaining ops, each as long as
// one of its items). The order in which items are taken is the ticket order.
// In level order only the deepest circuits are left at the end, each op of a
// large state split into a few items, and most work-groups idle; on the
// 512-circuit workload that end is short (62.6 against 63.1 ms per launch)
// and the simulation adds about 3.5 ms of planning, so level order stays the
// default.
void order_items_critical_path(qsim_batch_s* b, const std::vector<Packed>& packed, const std::vector<int>& op0,
                               int n_circuits) {
    constexpr int kSimGroups = 256;
    constexpr double kItemCost = 4.0;  // fixed cost of an item, in tiles
    struct Avail {
        double prio;
        uint32_t op, tile0;
        bool operator<(const Avail& o) const {  // max-heap: larger prio, then smaller op, then smaller tile0
            if (prio != o.prio) return prio < o.prio;
            if (op != o.op) return op > o.op;
            return tile0 > o.tile0;
        }
    };
    // per op: circuit, index in the circuit, items, remaining chain
    const size_t n_ops = b->ops.size();
    std::vector<int> op_circ(n_ops), op_idx(n_ops);
    std::vector<uint32_t> op_items(n_ops), left(n_ops);
    std::vector<double> chain(n_ops);
    for (int i = 0; i < n_circuits; ++i) {
        const size_t m = packed[i].ops.size();
        double tail = 0.0;
        for (size_t j = m; j-- > 0;) {
            const size_t o = op0[i] + j;
            const BatchOp& op = b->ops[o];
            op_circ[o] = i;
            op_idx[o] = (int)j;
            op_items[o] = (uint32_t)((op.tiles + b->item_tiles - 1) / b->item_tiles);
            left[o] = op_items[o];
            tail += (double)std::min<uint64_t>(op.tiles, b->item_tiles) + kItemCost;
            chain[o] = tail;
        }
    }
    std::priority_queue<Avail> avail;
    auto release = [&](size_t o) {
        const BatchOp& op = b->ops[o];
        for (uint32_t it = 0; it < op_items[o]; ++it) avail.push(Avail{chain[o], (uint32_t)o, it * b->item_tiles});
    };
    for (int i = 0; i < n_circuits; ++i)
        if (!packed[i].ops.empty()) release(op0[i]);
    // running items: (finish time, op), earliest first
    using Run = std::pair<double, uint32_t>;
    std::priority_queue<Run, std::vector<Run>, std::greater<Run>> running;
    double now = 0.0;
    int idle = kSimGroups;
    b->items.reserve(b->items.size() + 1024);
    while (!avail.empty() || !running.empty()) {
        while (idle > 0 && !avail.empty()) {
            const Avail a = avail.top();
            avail.pop();
            b->items.push_back(BatchItem{a.op, a.tile0});
            const uint64_t tiles = std::min<uint64_t>(b->item_tiles, b->ops[a.op].tiles - a.tile0);
            running.push(Run{now + (double)tiles + kItemCost, a.op});
            --idle;
        }
        if (running.empty()) break;
        const Run r = running.top();
        running.pop();
        now = r.first;
        ++idle;
        if (--left[r.second] == 0) {  // the op is complete: the circuit's next op is available
            const int c = op_circ[r.second];
            if ((size_t)op_idx[r.second] + 1 < packed[c].ops.size()) release(r.second + 1);
        }
    }
}

// Diagonal order: circuit i's op j gets key i + j (circuits in the order
// given), items sorted by key, then by circuit. Op j of circuit i runs next
// to op j - 1 of circuit i + 1, so only about as many circuits as they have
// ops are in flight at once: when the circuits are pieces of one large state,
// the pieces in flight stay in the last-level (Infinity) cache between ops.
void order_items_diagonal(qsim_batch_s* b, const std::vector<Packed>& packed, const std::vector<int>& op0,
                          int n_circuits) {
    std::vector<std::pair<size_t, int>> keys;  // (i + j, i)
    for (int i = 0; i < n_circuits; ++i)
        for (size_t j = 0; j < packed[i].ops.size(); ++j) keys.emplace_back(i + j, i);
    std::sort(keys.begin(), keys.end());
    for (const auto& kv : keys) {
        const int i = kv.second;
        const size_t j = kv.first - i;
        const BatchOp& op = b->ops[op0[i] + j];
        const uint64_t n_it = (op.tiles + b->item_tiles - 1) / b->item_tiles;
        for (uint64_t it = 0; it < n_it; ++it)
            b->items.push_back(BatchItem{(uint32_t)(op0[i] + j), (uint32_t)(it * b->item_tiles)});
    }
}

}  // namespace

extern "C" {

qsim_status qsim_batch_plan(const qsim_batch_circuit* circuits, int n_circuits, const qsim_run_opts* opts,
                            qsim_batch* out, size_t* workspace_bytes) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!out) return fail(QSIM_E_INVALID, "null output handle");
    *out = nullptr;
    if (n_circuits < 1 || !circuits) return fail(QSIM_E_INVALID, "empty batch");
    if (!opts) return fail(QSIM_E_INVALID, "batch options are required");
    if (opts->scheduler == QSIM_SCHED_PER_GATE) return fail(QSIM_E_UNSUPPORTED, "per-gate runs are not batched");
    if (opts->scheduler < QSIM_SCHED_PER_GATE || opts->scheduler > QSIM_SCHED_LEARNED)
        return fail(QSIM_E_INVALID, "unknown scheduler");
    if (opts->kmax < 1 || opts->kmax > 6) return fail(QSIM_E_UNSUPPORTED, "batch kmax must be in [1, 6]");
    for (int i = 0; i < n_circuits; ++i) {
        const qsim_batch_circuit& c = circuits[i];
        const std::string at = "circuit " + std::to_string(i) + ": ";
        if (c.n_qubits < kBatchMinQ || c.n_qubits > kBatchMaxQ)
            return fail(QSIM_E_UNSUPPORTED, at + "batched states have 11 to 30 qubits");
        if (!c.dev_amps || (reinterpret_cast<uintptr_t>(c.dev_amps) & 255))
            return fail(QSIM_E_INVALID, at + "amplitudes must be a 256-byte aligned device buffer");
        if (c.n_gates < 0 || (c.n_gates && !c.gates)) return fail(QSIM_E_INVALID, at + "bad gate list");
        for (int g = 0; g < c.n_gates; ++g)
            if (qsim_status r = check_gate(c.n_qubits, c.gates[g], g)) return fail(r, at + qsim_last_error());
        for (int j = 0; j < i; ++j)
            if (circuits[j].dev_amps == c.dev_amps) return fail(QSIM_E_INVALID, at + "shares its amplitudes");
    }

    // schedule and pack the circuits in parallel
    std::vector<Packed> packed(n_circuits);
    const int pad = g_batch_pad;
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const int n_workers = (int)std::min<unsigned>(hw, (unsigned)n_circuits);
    std::vector<std::future<void>> fut;
    for (int w = 0; w < n_workers; ++w)
        fut.push_back(std::async(std::launch::async, [&, w] {
            for (int i = w; i < n_circuits; i += n_workers) packed[i] = pack_circuit(circuits[i], opts, i, pad);
        }));
    for (auto& f : fut) f.get();
    for (int i = 0; i < n_circuits; ++i)
        if (packed[i].st != QSIM_OK) return fail(packed[i].st, packed[i].err);

    auto b = new qsim_batch_s;
    b->n_circuits = n_circuits;
    b->item_tiles = (uint32_t)g_batch_item_tiles;
    std::vector<int> op0(n_circuits);  // first global op of each circuit
    for (int i = 0; i < n_circuits; ++i) {
        Packed& P = packed[i];
        b->amps.push_back(circuits[i].dev_amps);
        op0[i] = (int)b->ops.size();
        const int bop0 = (int)b->bops.size(), epi0 = (int)b->epis.size();
        const int bg0 = (int)b->bgates.size(), d0 = (int)b->dense.size();
        for (size_t j = 0; j < P.ops.size(); ++j) {
            b->ops.push_back(P.ops[j]);
            b->op_mat.push_back(P.op_mat[j] < 0 ? -1 : P.op_mat[j] + bop0);
            b->op_epi.push_back(P.op_epi[j] < 0 ? -1 : P.op_epi[j] + epi0);
        }
        for (size_t j = 0; j < P.bops.size(); ++j) {
            BuildOp bo = P.bops[j];
            bo.gate0 += bg0;
            bo.out_off = b->mat_total;
            b->mat_off.push_back(b->mat_total);
            b->mat_total += (int64_t)align256((size_t)P.mat_bytes[j]);
            b->bops.push_back(bo);
        }
        for (BuildGate bg : P.bgates) {
            if (bg.dense_off >= 0) bg.dense_off += d0;
            b->bgates.push_back(bg);
        }
        b->dense.insert(b->dense.end(), P.dense.begin(), P.dense.end());
        b->epis.insert(b->epis.end(), P.epis.begin(), P.epis.end());
        b->n_applied += P.n_applied;
    }

    // dep of each op = items of the circuit's earlier ops
    for (int i = 0; i < n_circuits; ++i) {
        uint32_t done = 0;
        for (size_t j = 0; j < packed[i].ops.size(); ++j) {
            BatchOp& op = b->ops[op0[i] + j];
            op.dep = done;
            done += (uint32_t)((op.tiles + b->item_tiles - 1) / b->item_tiles);
        }
    }
    if (g_batch_order == 0)
        order_items_by_level(b, circuits, packed, op0, n_circuits);
    else if (g_batch_order == 1)
        order_items_critical_path(b, packed, op0, n_circuits);
    else
        order_items_diagonal(b, packed, op0, n_circuits);
    // the order must hand out every item once, each op's items after all items
    // of its circuit's previous op (what keeps the waits of the kernel finite)
    {
        const size_t n_ops = b->ops.size();
        std::vector<char> first(n_ops, 0);
        for (int i = 0; i < n_circuits; ++i)
            if ((size_t)op0[i] < n_ops) first[op0[i]] = 1;
        std::vector<uint32_t> seen(n_ops, 0), need(n_ops, 0);
        size_t total = 0;
        for (size_t o = 0; o < n_ops; ++o) {
            need[o] = (uint32_t)((b->ops[o].tiles + b->item_tiles - 1) / b->item_tiles);
            total += need[o];
        }
        bool ok = b->items.size() == total;
        for (size_t k = 0; ok && k < b->items.size(); ++k) {
            const uint32_t o = b->items[k].op;
            ok = o < n_ops && (first[o] || seen[o - 1] == need[o - 1]) && seen[o] < need[o];
            if (ok) ++seen[o];
        }
        if (!ok) {
            delete b;
            return fail(QSIM_E_INVALID, "internal error: batch work items out of dependency order");
        }
    }
    if (b->items.size() >= (size_t(1) << 31)) {
        delete b;
        return fail(QSIM_E_UNSUPPORTED, "too many work items");
    }

    size_t off = align256((size_t(n_circuits) + 2) * sizeof(uint32_t));
    b->off_ops = off;
    off += align256(b->ops.size() * sizeof(BatchOp));
    b->off_items = off;
    off += align256(b->items.size() * sizeof(BatchItem));
    b->off_epis = off;
    off += align256(b->epis.size() * sizeof(EpiDesc));
    b->off_bops = off;
    off += align256(b->bops.size() * sizeof(BuildOp));
    b->off_bgates = off;
    off += align256(b->bgates.size() * sizeof(BuildGate));
    b->off_dense = off;
    off += align256(b->dense.size() * sizeof(double));
    b->off_mats = off;
    off += (size_t)b->mat_total;
    b->ws_bytes = off;
    b->plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (workspace_bytes) *workspace_bytes = b->ws_bytes;
    *out = b;
    return QSIM_OK;
}

qsim_status qsim_batch_run(qsim_batch b, void* dev_workspace, size_t ws_bytes, void* hip_stream,
                           uint32_t wait_limit_us, qsim_batch_stats* stats) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!b) return fail(QSIM_E_INVALID, "null batch handle");
    if (!dev_workspace || (reinterpret_cast<uintptr_t>(dev_workspace) & 255))
        return fail(QSIM_E_INVALID, "workspace must be a 256-byte aligned device buffer");
    if (ws_bytes < b->ws_bytes) return fail(QSIM_E_INVALID, "workspace too small");
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    char* ws = static_cast<char*>(dev_workspace);

    // descriptors with device addresses, uploaded in one copy
    std::vector<char> host(b->off_mats, 0);
    BatchOp* ops = reinterpret_cast<BatchOp*>(host.data() + b->off_ops);
    for (size_t j = 0; j < b->ops.size(); ++j) {
        ops[j] = b->ops[j];
        ops[j].psi = static_cast<float2*>(b->amps[b->ops[j].circuit]);
        ops[j].A = b->op_mat[j] < 0 ? nullptr
                                     : reinterpret_cast<const float*>(ws + b->off_mats + b->mat_off[b->op_mat[j]]);
        ops[j].epi = b->op_epi[j] < 0 ? nullptr
                                       : reinterpret_cast<const EpiDesc*>(ws + b->off_epis) + b->op_epi[j];
    }
    auto put = [&](size_t off, const void* src, size_t bytes) {
        if (bytes) std::memcpy(host.data() + off, src, bytes);
    };
    put(b->off_items, b->items.data(), b->items.size() * sizeof(BatchItem));
    put(b->off_epis, b->epis.data(), b->epis.size() * sizeof(EpiDesc));
    put(b->off_bops, b->bops.data(), b->bops.size() * sizeof(BuildOp));
    put(b->off_bgates, b->bgates.data(), b->bgates.size() * sizeof(BuildGate));
    put(b->off_dense, b->dense.data(), b->dense.size() * sizeof(double));
    HIP_TRY(hipMemcpyAsync(ws, host.data(), host.size(), hipMemcpyHostToDevice, st), "upload batch descriptors");
    HIP_TRY(launch_build(reinterpret_cast<const BuildOp*>(ws + b->off_bops), (int)b->bops.size(),
                         reinterpret_cast<const BuildGate*>(ws + b->off_bgates),
                         reinterpret_cast<const double*>(ws + b->off_dense), ws + b->off_mats, st),
            "matrix build launch");

    int dev = 0, cus = 0, clock_khz = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "device attribute");
    HIP_TRY(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev), "device attribute");
    // wall-clock ticks of the longest dependency wait
    const uint64_t wait_ticks =
        std::max<uint64_t>(1, uint64_t(wait_limit_us ? wait_limit_us : kDefaultWaitUs) *
                                  uint64_t(std::max(clock_khz, 1)) / 1000);
    const uint32_t n_items = (uint32_t)b->items.size();
    uint32_t grid = g_batch_grid > 0 ? (uint32_t)g_batch_grid : (uint32_t)std::max(cus, 1);  // one per CU (LDS)
    grid = std::max(1u, std::min(grid, n_items));
    uint32_t* counters = reinterpret_cast<uint32_t*>(ws);
    HIP_TRY(launch_batch(reinterpret_cast<const BatchOp*>(ws + b->off_ops),
                         reinterpret_cast<const BatchItem*>(ws + b->off_items), n_items, counters,
                         (uint32_t)b->n_circuits, b->item_tiles, wait_ticks, grid, st),
            "batch launch");
    uint32_t flags[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(flags, counters, sizeof(flags), hipMemcpyDeviceToHost, st), "read batch counters");
    HIP_TRY(hipStreamSynchronize(st), "batch run");
    const double run_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->n_circuits = b->n_circuits;
        stats->n_ops = (int32_t)b->ops.size();
        stats->n_clusters = (int32_t)b->bops.size();
        stats->n_items = (int32_t)n_items;
        stats->grid = (int32_t)grid;
        stats->n_gates_applied = b->n_applied;
        stats->plan_ms = b->plan_ms;
        stats->run_ms = run_ms;
        stats->workspace_bytes = b->ws_bytes;
    }
    if (flags[1]) return fail(QSIM_E_DEVICE, "a dependency wait of the batch kernel exceeded its time limit");
    if (flags[0] < n_items) return fail(QSIM_E_DEVICE, "the batch kernel did not take every work item");
    return QSIM_OK;
}

qsim_status qsim_batch_destroy(qsim_batch b) {
    delete b;
    return QSIM_OK;
}

}  // extern "C"
