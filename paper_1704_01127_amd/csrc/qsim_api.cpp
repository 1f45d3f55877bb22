// C ABI of the simulator (include/qsim.h): argument checks, the state handle,
// scheduling, cluster-matrix upload / build and kernel dispatch.
#include "qsim.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "api_common.h"
#include "qsim_internal.h"
#include "scheduler.h"

using namespace qsim;
using namespace qsim::api;

namespace {
thread_local std::string g_err;
}  // namespace

qsim_status qsim::api::fail(qsim_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

qsim_status qsim::api::hip_fail(hipError_t e, const char* where) {
    return fail(QSIM_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

namespace {

// Workspace layout (byte offsets, 256-aligned).
constexpr size_t kPartBytes = size_t(kReduceBlocks) * 8 * sizeof(double);  // partial sums
constexpr size_t kResOff = kPartBytes;                                     // 8 doubles
constexpr size_t kDescOff = kResOff + 256;
constexpr size_t kDescBytes = size_t(6) << 20;                             // descriptors + dense gates
constexpr size_t kMatOff = kDescOff + kDescBytes;
constexpr int kSlots = 64;                                                 // cluster matrices per chunk

size_t slot_bytes(bool dbl, int kmax) {
    // the largest layout for k <= kmax (real-split 2^(k+1) squared or complex 2^k squared: equal size)
    return (size_t)matrix_bytes(std::max(1, std::min(kmax, kMaxK)), LAYOUT_MFMA32F, dbl);
}

}  // namespace

// ------------------------------------------------------------ kernel-variant policy
namespace qsim {
namespace {
int g_cluster_variant = -1;
// [dtype][k][low_class]: a direct gather when no target is on the low bits,
// the LDS-staged variant otherwise (k = 6, complex64: from two low targets on;
// with one the direct kernel's loads still use whole cache lines)
// (k = 7 has the direct kernel only; its entries are not read)
int g_tune[2][kMaxK + 1][kLowClasses] = {
    {{0, 1, 1, 1}, {0, 1, 1, 1}, {0, 1, 1, 1}, {0, 1, 1, 1}, {0, 1, 1, 1}, {0, 1, 1, 1}, {0, 0, 1, 1}, {0, 0, 0, 0}},
    {{0, 1, 1, 1}, {0, 1, 1, 1}, {0, 1, 1, 1}, {0, 1, 1, 1}, {0, 1, 1, 1}, {0, 1, 1, 1}, {0, 1, 1, 1}, {0, 0, 0, 0}}};
}  // namespace
void set_cluster_variant(int v) { g_cluster_variant = v; }
int get_cluster_variant() { return g_cluster_variant; }
void set_tune_entry(bool dbl, int k, int cls, int variant) { g_tune[dbl][k][cls] = variant; }
int get_tune_entry(bool dbl, int k, int cls) { return g_tune[dbl][k][cls]; }
// Analytic cost model of the cost-driven scheduler: measured microseconds of
// one op by k (index 0 = diagonal pass) on a state of n_ref qubits, scaled by
// 2^(n - n_ref) (every op streams the whole state). Defaults: a k-independent
// cost, which reduces the cost-driven scheduler to "most gates per cluster".
int g_batch_grid = 0;
int g_batch_pad = 0;
int g_batch_item_tiles = 128;
int g_k6_kernel = 2;
int g_fold_init = 2;
int g_fold_table = 1;
int g_deviations = 1;
int g_pair = 0;
int g_pair_tile = 11;
int g_cluster_sets = 1;
int g_batch_order = 0;
int g_check_unitary = 0;  // host check of every dense matrix: max |M M^+ - I| <= 1e-10
int g_map_qubits = 0;     // runs from the uniform state: relabel qubits away from the slow bit locations
double g_cost_us[2][kMaxK + 1] = {{1, 1, 1, 1, 1, 1, 1, 1}, {1, 1, 1, 1, 1, 1, 1, 1}};
int g_cost_nref[2] = {30, 30};
int cluster_variant_for(bool dbl, const ClusterGeom& g, int layout) {
    if (layout == LAYOUT_PLAIN) return 0;
    if (g.k > 5 && (dbl || layout != LAYOUT_SPLIT16F)) return 0;  // k = 6: float, fp16-halves kernel only; k = 7: direct
    if (g_cluster_variant >= 0) return g_cluster_variant;
    return g_tune[dbl][g.k][low_class(g.t, g.k)];
}
}  // namespace qsim

namespace qsim {
bool learned_model_loaded();
double learned_cost_us(int n, bool dbl, int k, const int* qubits, int n_epi, int variant);
double learned_cost_best_us(int n, bool dbl, int k, const int* qubits, int n_epi, int* variant);
}  // namespace qsim

struct OpRecord {
    int kind;  // 0 cluster, 1 diagonal pass, 2 1-qubit gate, 3 1-qubit phase, 4 CZ, 5 matrix build,
               // 6 uniform initialisation folded into a cluster, 7 two clusters in one pass
    int k;
    int qubits[kMaxK];
    int flags;  // bit 0: diagonal epilogue, bit 1: LDS-staged kernel, bit 2: matrix-core kernel
    hipEvent_t ev0, ev1;
};

struct qsim_state_s {
    int n = 0;
    bool dbl = false;
    void* psi = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t st = nullptr;
    int kmax_ws = 6;  // largest k the workspace slots can hold
    // the last run's final cluster launch left the sums of p, p^2, -p ln p of
    // the current state in the workspace's partial area (stats_blocks of them)
    bool stats_ready = false;
    unsigned stats_blocks = 0;
    // op timing (record_timings): HIP events around every launch
    bool recording = false;
    std::vector<OpRecord> recs;
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
    ~qsim_state_s() {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

namespace {
bool is_named_1q(int kind) { return kind >= G_H && kind <= G_PHASE && kind != G_CZ; }
}  // namespace

qsim_status qsim::api::check_gate(int n, const qsim_gate& g, int idx) {
    const std::string at = "gate " + std::to_string(idx) + ": ";
    int nq;
    if (g.kind == G_CZ) nq = 2;
    else if (g.kind == G_DENSE) nq = g.k;
    else if (is_named_1q(g.kind)) nq = 1;
    else return fail(QSIM_E_INVALID, at + "unknown gate kind " + std::to_string(g.kind));
    if (g.kind == G_DENSE && (nq < 1 || nq > kMaxGateQ))
        return fail(QSIM_E_UNSUPPORTED, at + "dense gates need 1 <= k <= 6");
    if (g.kind == G_DENSE && !g.mat) return fail(QSIM_E_INVALID, at + "dense gate without a matrix");
    if (g.kind == G_DENSE && g_check_unitary) {
        // (M M^+)_{ij} = sum_l M_il conj(M_jl); row-major, (re, im) interleaved
        const int d = 1 << nq;
        double worst = 0.0;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j) {
                double re = 0.0, im = 0.0;
                for (int l = 0; l < d; ++l) {
                    const double ar = g.mat[2 * (i * d + l)], ai = g.mat[2 * (i * d + l) + 1];
                    const double br = g.mat[2 * (j * d + l)], bi = g.mat[2 * (j * d + l) + 1];
                    re += ar * br + ai * bi;
                    im += ai * br - ar * bi;
                }
                if (i == j) re -= 1.0;
                worst = std::max(worst, std::hypot(re, im));
            }
        if (!(worst <= 1e-10))
            return fail(QSIM_E_INVALID, at + "dense matrix is not unitary (max |M M^+ - I| = " +
                                            std::to_string(worst) + ")");
    }
    uint64_t m = 0;
    for (int j = 0; j < nq; ++j) {
        const int q = g.qubits[j];
        if (q < 0 || q >= n) return fail(QSIM_E_INVALID, at + "qubit " + std::to_string(q) + " out of range");
        if (m >> q & 1) return fail(QSIM_E_INVALID, at + "repeated qubit " + std::to_string(q));
        m |= uint64_t(1) << q;
    }
    return QSIM_OK;
}

int qsim::api::gate_nq(const qsim_gate& g) { return g.kind == G_CZ ? 2 : (g.kind == G_DENSE ? g.k : 1); }

BuildGate qsim::api::to_build_gate(const qsim_gate& g, const int* pos_of, std::vector<double>& dense) {
    BuildGate b;
    std::memset(&b, 0, sizeof(b));
    b.kind = g.kind;
    b.nq = gate_nq(g);
    for (int j = 0; j < b.nq; ++j) b.pos[j] = pos_of[g.qubits[j]];
    b.theta = g.theta;
    b.dense_off = -1;
    if (g.kind == G_DENSE) {
        b.dense_off = (int)dense.size();
        const int cnt = 2 << (2 * g.k);
        dense.insert(dense.end(), g.mat, g.mat + cnt);
    }
    return b;
}

qsim_status qsim::api::split_epilogue(const int* pos_of, const qsim_gate* gates, const std::vector<int>& epi_gates,
                                      std::vector<BuildGate>& bgates, std::vector<double>& dense, EpiDesc& e) {
    std::memset(&e, 0, sizeof(e));
    for (int gi : epi_gates) {
        const qsim_gate& g = gates[gi];
        if (g.kind == G_CZ) {
            const int a = g.qubits[0], b = g.qubits[1];
            const bool ta = pos_of[a] >= 0, tb = pos_of[b] >= 0;
            if (ta && tb) {
                bgates.push_back(to_build_gate(g, pos_of, dense));
            } else if (ta || tb) {
                if (e.n_mix >= kEpiMax) return fail(QSIM_E_UNSUPPORTED, "epilogue too long");
                e.mix[e.n_mix][0] = ta ? pos_of[a] : pos_of[b];
                e.mix[e.n_mix][1] = ta ? b : a;
                e.n_mix++;
            } else {
                if (e.n_cc >= kEpiMax) return fail(QSIM_E_UNSUPPORTED, "epilogue too long");
                e.cc[e.n_cc][0] = a;
                e.cc[e.n_cc][1] = b;
                e.n_cc++;
            }
        } else {
            const int q = g.qubits[0];
            if (pos_of[q] >= 0) {
                bgates.push_back(to_build_gate(g, pos_of, dense));
            } else {
                if (e.n_ph >= kEpiMax) return fail(QSIM_E_UNSUPPORTED, "epilogue too long");
                const double ang = gate_phase_angle(g.kind, g.theta);
                e.ph_q[e.n_ph] = q;
                e.ph[e.n_ph][0] = std::cos(ang);
                e.ph[e.n_ph][1] = std::sin(ang);
                e.n_ph++;
            }
        }
    }
    return QSIM_OK;
}

namespace {

// One chunk of work: descriptors packed on the host, uploaded once.
struct Chunk {
    std::vector<BuildOp> bops;
    std::vector<BuildGate> bgates;
    std::vector<double> dense;
    std::vector<EpiDesc> epis;
    struct Item {
        int kind;        // 0 cluster, 1 diag pass, 2 gate1q, 3 phase1q, 4 cz, 6 uniform init + cluster,
                         // 7 two 5-qubit clusters in one pass, 8 uniform init + two clusters
                         // (geom2 / slot2 / epi2: the first one)
        ClusterGeom geom;
        int layout;
        int slot;        // matrix slot (cluster)
        int epi;         // index into epis, -1 none
        ClusterGeom geom2;  // kind 7: the second cluster
        int slot2, epi2;
        int q0, q1;
        double m[8];
        bool stats;      // kind 0: also sum p, p^2, -p ln p of the stored state (the run's last op)
        int n_epi;       // diagonal gates the scheduler attached to the cluster (its epilogue)
        int variant;     // kind 0: matrix-core kernel variant chosen by the learned model, -1: the library's rule
        int omask, rmask;  // kind 8: the table form's shared and sign-flipped rows, omask -1: matrix cores
        int slot3;         // kind 8 table form: the table's slot
    };
    std::vector<Item> items;
    int slots_used = 0;
    size_t desc_bytes() const {
        return align256(bops.size() * sizeof(BuildOp)) + align256(bgates.size() * sizeof(BuildGate)) +
               align256(dense.size() * sizeof(double)) + align256(epis.size() * sizeof(EpiDesc));
    }
    void clear() {
        bops.clear(); bgates.clear(); dense.clear(); epis.clear(); items.clear(); slots_used = 0;
    }
};

// Queue a matrix build; a 7-qubit matrix is built by kBuildParts7 work-groups.
void push_build(Chunk& c, BuildOp bo) {
    const int parts = bo.k == 7 ? kBuildParts7 : 1;
    for (int p = 0; p < parts; ++p) {
        bo.part = p;
        c.bops.push_back(bo);
    }
}

hipError_t next_event(qsim_state_s* s, hipEvent_t* e) {
    if (s->pool_used == s->pool.size()) {
        hipEvent_t ne;
        hipError_t r = hipEventCreate(&ne);
        if (r != hipSuccess) return r;
        s->pool.push_back(ne);
    }
    *e = s->pool[s->pool_used++];
    return hipSuccess;
}

// Start / finish the timing record of one launch (no-ops unless recording).
hipError_t rec_begin(qsim_state_s* s, OpRecord& r) {
    if (!s->recording) return hipSuccess;
    hipError_t e = next_event(s, &r.ev0);
    if (e == hipSuccess) e = next_event(s, &r.ev1);
    if (e == hipSuccess) e = hipEventRecord(r.ev0, s->st);
    return e;
}
hipError_t rec_end(qsim_state_s* s, const OpRecord& r) {
    if (!s->recording) return hipSuccess;
    hipError_t e = hipEventRecord(r.ev1, s->st);
    if (e == hipSuccess) s->recs.push_back(r);
    return e;
}

qsim_status flush(qsim_state_s* s, Chunk& c) {
    if (c.items.empty()) return QSIM_OK;
    const size_t ob = 0;
    const size_t gb = ob + align256(c.bops.size() * sizeof(BuildOp));
    const size_t db = gb + align256(c.bgates.size() * sizeof(BuildGate));
    const size_t eb = db + align256(c.dense.size() * sizeof(double));
    const size_t total = eb + align256(c.epis.size() * sizeof(EpiDesc));
    if (total > kDescBytes) return fail(QSIM_E_UNSUPPORTED, "descriptor chunk too large");
    std::vector<char> host(total, 0);
    if (!c.bops.empty()) std::memcpy(host.data() + ob, c.bops.data(), c.bops.size() * sizeof(BuildOp));
    if (!c.bgates.empty()) std::memcpy(host.data() + gb, c.bgates.data(), c.bgates.size() * sizeof(BuildGate));
    if (!c.dense.empty()) std::memcpy(host.data() + db, c.dense.data(), c.dense.size() * sizeof(double));
    if (!c.epis.empty()) std::memcpy(host.data() + eb, c.epis.data(), c.epis.size() * sizeof(EpiDesc));
    char* dev = s->ws + kDescOff;
    char* mats = s->ws + kMatOff;
    if (total) HIP_TRY(hipMemcpyAsync(dev, host.data(), total, hipMemcpyHostToDevice, s->st), "upload descriptors");
    if (!c.bops.empty()) {
        OpRecord r;
        std::memset(&r, 0, sizeof(r));
        r.kind = 5;
        r.k = (int)c.bops.size();
        HIP_TRY(rec_begin(s, r), "event record");
        HIP_TRY(launch_build(reinterpret_cast<const BuildOp*>(dev + ob), (int)c.bops.size(),
                             reinterpret_cast<const BuildGate*>(dev + gb),
                             reinterpret_cast<const double*>(dev + db), mats, s->st),
                "matrix build launch");
        HIP_TRY(rec_end(s, r), "event record");
    }
    const EpiDesc* epis = reinterpret_cast<const EpiDesc*>(dev + eb);
    const size_t sb = slot_bytes(s->dbl, s->kmax_ws);
    for (const auto& it : c.items) {
        OpRecord r;
        std::memset(&r, 0, sizeof(r));
        r.kind = it.kind;
        const int variant =
            it.kind == 0 ? (it.variant >= 0 ? it.variant : cluster_variant_for(s->dbl, it.geom, it.layout)) : 0;
        if (it.kind == 0 || it.kind == 6 || it.kind == 7 || it.kind == 8) {
            r.k = it.geom.k;
            for (int j = 0; j < it.geom.k; ++j) r.qubits[j] = it.geom.t[j];
            r.flags = (it.epi >= 0 ? 1 : 0) | (variant == 1 ? 2 : 0) | (it.layout != LAYOUT_PLAIN ? 4 : 0) |
                      (it.stats ? 8 : 0) | (it.kind == 8 && it.omask >= 0 ? 16 : 0) | (std::min(it.n_epi, 255) << 8);
        } else if (it.kind >= 2) {
            r.k = it.kind == 4 ? 2 : 1;
            r.qubits[0] = it.q0;
            r.qubits[1] = it.q1;
        }
        HIP_TRY(rec_begin(s, r), "event record");
        hipError_t e = hipSuccess;
        switch (it.kind) {
            case 0: {
                double* sp = it.stats ? reinterpret_cast<double*>(s->ws) : nullptr;
                unsigned nb = 0;
                e = launch_cluster(s->psi, s->dbl, it.geom, mats + it.slot * sb, it.layout,
                                   it.epi >= 0 ? epis + it.epi : nullptr, variant, s->st, sp, sp ? &nb : nullptr);
                if (e == hipSuccess && sp) {
                    s->stats_ready = true;
                    s->stats_blocks = nb;
                }
                break;
            }
            case 1: e = launch_diag(s->psi, s->dbl, s->n, epis + it.epi, s->st); break;
            case 2: e = launch_gate1q(s->psi, s->dbl, s->n, it.q0, it.m, s->st); break;
            case 3: e = launch_phase1q(s->psi, s->dbl, s->n, it.q0, it.m[0], it.m[1], s->st); break;
            case 4: e = launch_cz(s->psi, s->dbl, s->n, it.q0, it.q1, s->st); break;
            case 6:
                e = launch_init_cluster(s->psi, s->dbl, it.geom, mats + it.slot * sb,
                                        it.epi >= 0 ? epis + it.epi : nullptr, s->st);
                break;
            case 8:
                e = launch_fold2(s->psi, it.geom, mats + it.slot * sb, it.epi >= 0 ? epis + it.epi : nullptr,
                                 it.epi2 >= 0 ? epis + it.epi2 : nullptr, it.geom2, mats + it.slot2 * sb, it.omask,
                                 it.rmask, it.omask >= 0 ? mats + it.slot3 * sb : nullptr, s->st);
                break;
            case 7: {
                int32_t t[2][5];
                for (int j = 0; j < 5; ++j) {
                    t[0][j] = it.geom.t[j];
                    t[1][j] = it.geom2.t[j];
                }
                const void* m2[2] = {mats + it.slot * sb, mats + it.slot2 * sb};
                const EpiDesc* e2[2] = {it.epi >= 0 ? epis + it.epi : nullptr, it.epi2 >= 0 ? epis + it.epi2 : nullptr};
                e = launch_multi(s->psi, s->n, it.q1, t, m2, e2, s->st);
                break;
            }
        }
        if (e != hipSuccess) return hip_fail(e, "kernel launch");
        HIP_TRY(rec_end(s, r), "event record");
    }
    c.clear();
    return QSIM_OK;
}

// Standalone diagonal pass over pairs and phases (global qubit indices): the
// kernel itself splits them by which index bits they read.
qsim_status diag_desc(int n, const std::vector<std::pair<int, int>>& pairs,
                      const std::vector<std::pair<int, double>>& phases, EpiDesc& e) {
    (void)n;
    std::memset(&e, 0, sizeof(e));
    if ((int)pairs.size() > kEpiMax) return fail(QSIM_E_UNSUPPORTED, "too many CZ pairs in a diagonal pass");
    if ((int)phases.size() > kEpiMax) return fail(QSIM_E_UNSUPPORTED, "too many phases in a diagonal pass");
    for (auto pr : pairs) {
        e.cc[e.n_cc][0] = std::min(pr.first, pr.second);
        e.cc[e.n_cc][1] = std::max(pr.first, pr.second);
        e.n_cc++;
    }
    for (auto ph : phases) {
        e.ph_q[e.n_ph] = ph.first;
        e.ph[e.n_ph][0] = std::cos(ph.second);
        e.ph[e.n_ph][1] = std::sin(ph.second);
        e.n_ph++;
    }
    return QSIM_OK;
}

// Add a cluster op (sorted qubits, member gates, epilogue gates) to the chunk;
// flushes first if the chunk is full. fold_init: the op is the first on the
// uniform state and is written by the folded initialisation kernel (plain
// complex128 matrix).
qsim_status add_cluster(qsim_state_s* s, Chunk& c, int k, const int* qubits, const qsim_gate* gates,
                        const std::vector<int>& members, const std::vector<int>& epi_gates,
                        bool fold_init = false) {
    size_t dense_need = 0;
    for (int gi : members) if (gates[gi].kind == G_DENSE) dense_need += size_t(2) << (2 * gates[gi].k);
    const size_t need = align256((c.bops.size() + kBuildParts7) * sizeof(BuildOp)) +
                        align256((c.bgates.size() + members.size() + epi_gates.size()) * sizeof(BuildGate)) +
                        align256((c.dense.size() + dense_need) * sizeof(double)) +
                        align256((c.epis.size() + 1) * sizeof(EpiDesc));
    if (c.slots_used >= kSlots || need > kDescBytes) {
        qsim_status r = flush(s, c);
        if (r != QSIM_OK) return r;
    }
    int pos_of[64];
    for (int i = 0; i < 64; ++i) pos_of[i] = -1;
    for (int j = 0; j < k; ++j) pos_of[qubits[j]] = j;
    BuildOp bo;
    std::memset(&bo, 0, sizeof(bo));
    bo.k = k;
    bo.gate0 = (int)c.bgates.size();
    bo.is_double = fold_init ? 1 : s->dbl;
    bo.layout = fold_init ? LAYOUT_PLAIN : cluster_layout(s->dbl, k, s->n);
    if (bo.layout < 0) return fail(QSIM_E_UNSUPPORTED, "no kernel for a cluster of this width on this state");
    bo.out_off = (int64_t)c.slots_used * (int64_t)slot_bytes(s->dbl, s->kmax_ws);
    for (int gi : members) c.bgates.push_back(to_build_gate(gates[gi], pos_of, c.dense));
    // epilogue: terms on target qubits only join the matrix, the rest go to the descriptor
    EpiDesc e;
    if (qsim_status r = split_epilogue(pos_of, gates, epi_gates, c.bgates, c.dense, e)) return r;
    bo.n_gates = (int)c.bgates.size() - bo.gate0;
    push_build(c, bo);
    Chunk::Item it;
    std::memset(&it, 0, sizeof(it));
    it.kind = fold_init ? 6 : 0;
    for (int j = 0; j < k; ++j) it.geom.t[j] = qubits[j];
    it.geom.n = s->n;
    it.geom.k = k;
    it.geom.ncols = uint64_t(1) << (s->n - k);
    it.layout = bo.layout;
    it.slot = c.slots_used++;
    it.epi = -1;
    it.n_epi = (int)epi_gates.size();
    it.variant = -1;
    if (e.n_cc || e.n_mix || e.n_ph) {
        it.epi = (int)c.epis.size();
        c.epis.push_back(e);
    }
    c.items.push_back(it);
    return QSIM_OK;
}

// The uniform start and the first two clusters A and B (B: 6 qubits, complex64,
// fp16-halves layout) in one write-only pass. A's matrix is built plain in
// complex128 without its epilogue; the epilogue is split relative to B's
// targets: terms on B's targets join B's matrix ahead of B's gates, the rest
// becomes a descriptor read per column of B.
qsim_status add_fold2(qsim_state_s* s, Chunk& c, const SOp& A, const SOp& B, const qsim_gate* gates) {
    size_t dense_need = 0, ng = 0;
    for (const SOp* op : {&A, &B}) {
        for (int gi : op->members) if (gates[gi].kind == G_DENSE) dense_need += size_t(2) << (2 * gates[gi].k);
        ng += op->members.size() + op->epi.size();
    }
    const size_t need = align256((c.bops.size() + 2 * kBuildParts7) * sizeof(BuildOp)) +
                        align256((c.bgates.size() + ng) * sizeof(BuildGate)) +
                        align256((c.dense.size() + dense_need) * sizeof(double)) +
                        align256((c.epis.size() + 2) * sizeof(EpiDesc));
    if (c.slots_used + 3 > kSlots || need > kDescBytes) {
        qsim_status r = flush(s, c);
        if (r != QSIM_OK) return r;
    }
    const int64_t sb = (int64_t)slot_bytes(s->dbl, s->kmax_ws);
    // A: plain complex128, its member gates only
    int posA[64], posB[64];
    for (int i = 0; i < 64; ++i) posA[i] = posB[i] = -1;
    for (int j = 0; j < A.k; ++j) posA[A.qubits[j]] = j;
    for (int j = 0; j < B.k; ++j) posB[B.qubits[j]] = j;
    BuildOp ba;
    std::memset(&ba, 0, sizeof(ba));
    ba.k = A.k;
    ba.gate0 = (int)c.bgates.size();
    ba.is_double = 1;
    ba.layout = LAYOUT_PLAIN;
    const int slotA = c.slots_used++;
    ba.out_off = slotA * sb;
    for (int gi : A.members) c.bgates.push_back(to_build_gate(gates[gi], posA, c.dense));
    ba.n_gates = (int)c.bgates.size() - ba.gate0;
    push_build(c, ba);
    // B: A's epilogue terms on B's targets, B's gates, B's own epilogue terms on its targets
    BuildOp bb;
    std::memset(&bb, 0, sizeof(bb));
    bb.k = B.k;
    bb.gate0 = (int)c.bgates.size();
    bb.is_double = 0;
    bb.layout = LAYOUT_SPLIT16F;
    const int slotB = c.slots_used++;
    bb.out_off = slotB * sb;
    EpiDesc e1, e2;
    if (qsim_status r = split_epilogue(posB, gates, A.epi, c.bgates, c.dense, e1)) return r;
    for (int gi : B.members) c.bgates.push_back(to_build_gate(gates[gi], posB, c.dense));
    if (qsim_status r = split_epilogue(posB, gates, B.epi, c.bgates, c.dense, e2)) return r;
    bb.n_gates = (int)c.bgates.size() - bb.gate0;
    // B's inputs vary with its rows shared with A (omask) and A's epilogue
    // signs on its rows (rmask): with few of these, B's outputs for each
    // pattern go into a table (B then built in plain complex128)
    int omask = 0, rmask = 0;
    for (int m = 0; m < B.k; ++m)
        if (posA[B.qubits[m]] >= 0) omask |= 1 << m;
    for (int i = 0; i < e1.n_mix; ++i) rmask |= 1 << e1.mix[i][0];
    const int tab_bits = __builtin_popcount((unsigned)omask) + __builtin_popcount((unsigned)rmask);
    const bool table = g_fold_table && __builtin_popcount((unsigned)omask) <= 2 &&
                       (1 << tab_bits) <= (B.k == 7 ? kFoldTab7Rows : kFoldTabRows) &&
                       sb >= (int64_t(8) << (B.k + tab_bits)) && sb >= (int64_t)matrix_bytes(B.k, LAYOUT_PLAIN, true);
    if (B.k == 7 && !table)  // the scheduler folds a 7-qubit second cluster only where the table form applies
        return fail(QSIM_E_UNSUPPORTED, "two-cluster start with a 7-qubit second cluster needs the table form");
    if (table) {
        bb.is_double = 1;
        bb.layout = LAYOUT_PLAIN;
    }
    push_build(c, bb);
    Chunk::Item it;
    std::memset(&it, 0, sizeof(it));
    it.kind = 8;
    it.layout = LAYOUT_SPLIT16F;
    for (int j = 0; j < B.k; ++j) it.geom.t[j] = B.qubits[j];
    it.geom.n = s->n;
    it.geom.k = B.k;
    it.geom.ncols = uint64_t(1) << (s->n - B.k);
    for (int j = 0; j < A.k; ++j) it.geom2.t[j] = A.qubits[j];
    it.geom2.n = s->n;
    it.geom2.k = A.k;
    it.geom2.ncols = uint64_t(1) << (s->n - A.k);
    it.slot = slotB;
    it.slot2 = slotA;
    it.omask = it.rmask = -1;
    if (table) {
        it.omask = omask;
        it.rmask = rmask;
        it.slot3 = c.slots_used++;
    }
    it.epi = it.epi2 = -1;
    if (e2.n_cc || e2.n_mix || e2.n_ph) {
        it.epi = (int)c.epis.size();
        c.epis.push_back(e2);
    }
    if (e1.n_cc || e1.n_mix || e1.n_ph) {
        it.epi2 = (int)c.epis.size();
        c.epis.push_back(e1);
    }
    c.items.push_back(it);
    return QSIM_OK;
}

qsim_status add_diag(qsim_state_s* s, Chunk& c, const std::vector<std::pair<int, int>>& pairs,
                     const std::vector<std::pair<int, double>>& phases) {
    if (c.desc_bytes() + 2 * sizeof(EpiDesc) + 1024 > kDescBytes) {
        qsim_status r = flush(s, c);
        if (r != QSIM_OK) return r;
    }
    EpiDesc e;
    qsim_status r = diag_desc(s->n, pairs, phases, e);
    if (r != QSIM_OK) return r;
    Chunk::Item it;
    std::memset(&it, 0, sizeof(it));
    it.kind = 1;
    it.epi = (int)c.epis.size();
    c.epis.push_back(e);
    c.items.push_back(it);
    return QSIM_OK;
}

// The five targets of a cluster in a pair: its qubits, then qubits of `prefer`
// (the pair's union), then the lowest others (identity on the added ones).
void pad5(int n, const int* q, int k, uint64_t prefer, int* t) {
    uint64_t m = 0;
    for (int j = 0; j < k; ++j) {
        t[j] = q[j];
        m |= uint64_t(1) << q[j];
    }
    int cnt = k;
    for (int b = 0; b < n && cnt < 5; ++b)
        if ((prefer >> b & 1) && !(m >> b & 1)) { t[cnt++] = b; m |= uint64_t(1) << b; }
    for (int b = 0; b < n && cnt < 5; ++b)
        if (!(m >> b & 1)) { t[cnt++] = b; m |= uint64_t(1) << b; }
    std::sort(t, t + 5);
}

// Two consecutive clusters of at most 5 qubits (complex64, n >= 11) applied
// in one pass (fp16-halves matrices): the pair's qubits fit one 11-bit tile.
qsim_status add_pair(qsim_state_s* s, Chunk& c, const SOp& A, const SOp* Bp, const qsim_gate* gates) {
    const SOp& B = Bp ? *Bp : A;
    const int m_ops = Bp ? 2 : 1;
    size_t dense_need = 0, ng = 0;
    for (const SOp* op : {&A, &B}) {
        for (int gi : op->members) if (gates[gi].kind == G_DENSE) dense_need += size_t(2) << (2 * gates[gi].k);
        ng += op->members.size() + op->epi.size();
    }
    const size_t need = align256((c.bops.size() + 2) * sizeof(BuildOp)) +
                        align256((c.bgates.size() + ng) * sizeof(BuildGate)) +
                        align256((c.dense.size() + dense_need) * sizeof(double)) +
                        align256((c.epis.size() + 2) * sizeof(EpiDesc));
    if (c.slots_used + 2 > kSlots || need > kDescBytes) {
        qsim_status r = flush(s, c);
        if (r != QSIM_OK) return r;
    }
    uint64_t U = 0;
    for (const SOp* op : {&A, &B})
        for (int j = 0; j < op->k; ++j) U |= uint64_t(1) << op->qubits[j];
    int t[2][5];
    pad5(s->n, A.qubits, A.k, U, t[0]);
    for (int j = 0; j < 5; ++j) U |= uint64_t(1) << t[0][j];
    pad5(s->n, B.qubits, B.k, U, t[1]);
    Chunk::Item it;
    std::memset(&it, 0, sizeof(it));
    it.kind = 7;
    it.layout = LAYOUT_SPLIT16F;
    it.q1 = m_ops;  // clusters in the pass
    const SOp* ops[2] = {&A, &B};
    for (int m = 0; m < m_ops; ++m) {
        int pos_of[64];
        for (int i = 0; i < 64; ++i) pos_of[i] = -1;
        for (int j = 0; j < 5; ++j) pos_of[t[m][j]] = j;
        BuildOp bo;
        std::memset(&bo, 0, sizeof(bo));
        bo.k = 5;
        bo.gate0 = (int)c.bgates.size();
        bo.is_double = 0;
        bo.layout = LAYOUT_SPLIT16F;
        const int slot = c.slots_used++;
        bo.out_off = (int64_t)slot * (int64_t)slot_bytes(s->dbl, s->kmax_ws);
        for (int gi : ops[m]->members) c.bgates.push_back(to_build_gate(gates[gi], pos_of, c.dense));
        EpiDesc e;
        if (qsim_status r = split_epilogue(pos_of, gates, ops[m]->epi, c.bgates, c.dense, e)) return r;
        bo.n_gates = (int)c.bgates.size() - bo.gate0;
        push_build(c, bo);
        int epi = -1;
        if (e.n_cc || e.n_mix || e.n_ph) {
            epi = (int)c.epis.size();
            c.epis.push_back(e);
        }
        ClusterGeom& g = m == 0 ? it.geom : it.geom2;
        for (int j = 0; j < 5; ++j) g.t[j] = t[m][j];
        g.n = s->n;
        g.k = 5;
        g.ncols = uint64_t(1) << (s->n - 5);
        (m == 0 ? it.slot : it.slot2) = slot;
        (m == 0 ? it.epi : it.epi2) = epi;
    }
    c.items.push_back(it);
    return QSIM_OK;
}

// A single gate with the per-gate kernels.
qsim_status add_gate(qsim_state_s* s, Chunk& c, const qsim_gate* gates, int gi) {
    const qsim_gate& g = gates[gi];
    if (g.kind == G_DENSE) {
        int qs[6];
        for (int j = 0; j < g.k; ++j) qs[j] = g.qubits[j];
        std::sort(qs, qs + g.k);
        return add_cluster(s, c, g.k, qs, gates, std::vector<int>{gi}, {});
    }
    Chunk::Item it;
    std::memset(&it, 0, sizeof(it));
    it.epi = -1;
    if (g.kind == G_CZ) {
        it.kind = 4;
        it.q0 = g.qubits[0];
        it.q1 = g.qubits[1];
    } else if (gate_is_diagonal(g.kind)) {
        it.kind = 3;
        it.q0 = g.qubits[0];
        const double ang = gate_phase_angle(g.kind, g.theta);
        it.m[0] = std::cos(ang);
        it.m[1] = std::sin(ang);
    } else {
        it.kind = 2;
        it.q0 = g.qubits[0];
        gate2x2(g.kind, g.theta, it.m);
    }
    c.items.push_back(it);
    return QSIM_OK;
}

qsim_status check_state(qsim_state s) {
    if (!s) return fail(QSIM_E_INVALID, "null state handle");
    return QSIM_OK;
}

}  // namespace

std::vector<SGate> qsim::api::to_sgates(const qsim_gate* gates, int n_gates) {
    std::vector<SGate> sg(n_gates);
    for (int i = 0; i < n_gates; ++i) {
        sg[i].kind = gates[i].kind;
        sg[i].nq = gate_nq(gates[i]);
        for (int j = 0; j < sg[i].nq; ++j) sg[i].q[j] = gates[i].qubits[j];
        sg[i].diag = gate_is_diagonal(gates[i].kind);
    }
    return sg;
}

// Cost function of the cost-driven schedulers (empty for the others).
OpCostFn qsim::api::cost_fn(const qsim_run_opts* o, int n, bool dbl) {
    if (!o || o->scheduler == QSIM_SCHED_PER_GATE || o->scheduler == QSIM_SCHED_GREEDY) return OpCostFn();
    if (o->scheduler == QSIM_SCHED_LEARNED && learned_model_loaded()) {
        return [n, dbl](int k, const int* q, int n_epi) { return learned_cost_us(n, dbl, k, q, n_epi, -1); };
    }
    const double scale = std::ldexp(1.0, n - g_cost_nref[dbl]);
    const double* us = g_cost_us[dbl];
    return [scale, us](int k, const int*, int) { return us[k] * scale; };
}

// The folded start qsim_run_circuit gives a run from the uniform state (see
// its fold / fold2 conditions), for the scheduler's pricing.
int qsim::api::fold_start_for(bool dbl, int n) {
    if (!g_fold_init) return 0;
    if (g_fold_init == 2 && !dbl && cluster_layout(false, 6, n) == LAYOUT_SPLIT16F) return g_fold_table ? 3 : 2;
    return 1;
}

SchedOpts qsim::api::to_sched_opts(const qsim_run_opts* o) {
    SchedOpts so;
    so.cluster_sets = g_cluster_sets != 0;
    so.deviations = g_deviations != 0;
    if (!o) return so;
    so.kmax = o->kmax;
    so.mode = o->scheduler == QSIM_SCHED_PER_GATE ? 0 : (o->scheduler == QSIM_SCHED_GREEDY ? 1 : 2);
    if (o->scheduler == QSIM_SCHED_LEARNED && !learned_model_loaded()) so.mode = 1;  // fixed-k greedy fallback
    so.fuse_diag = o->fuse_diag != 0;
    so.skip_trailing_diag = o->skip_trailing_diag != 0;
    so.skip_initial_h = o->skip_initial_h != 0;
    return so;
}

extern "C" {

size_t qsim_workspace_bytes(int n_qubits, qsim_dtype dt, int kmax) {
    (void)n_qubits;
    return kMatOff + size_t(kSlots) * slot_bytes(dt == QSIM_C128, kmax <= 0 ? kMaxK : kmax);
}

qsim_status qsim_create(int n_qubits, qsim_dtype dt, void* dev_amps, size_t amps_bytes, void* dev_workspace,
                        size_t ws_bytes, void* hip_stream, qsim_init init, qsim_state* out) {
    if (!out) return fail(QSIM_E_INVALID, "out is null");
    *out = nullptr;
    if (dt != QSIM_C64 && dt != QSIM_C128) return fail(QSIM_E_INVALID, "unknown dtype");
    const bool dbl = dt == QSIM_C128;
    if (n_qubits < 1 || n_qubits > (dbl ? 33 : 34))
        return fail(QSIM_E_UNSUPPORTED, "n_qubits must be in [1, 34] (complex64) or [1, 33] (complex128)");
    if (!dev_amps || !dev_workspace) return fail(QSIM_E_INVALID, "null device buffer");
    if ((reinterpret_cast<uintptr_t>(dev_amps) & 255) || (reinterpret_cast<uintptr_t>(dev_workspace) & 255))
        return fail(QSIM_E_INVALID, "device buffers must be 256-byte aligned");
    const size_t need = (size_t(1) << n_qubits) * (dbl ? 16 : 8);
    if (amps_bytes < need) return fail(QSIM_E_INVALID, "state buffer too small");
    // the workspace decides the largest cluster it can hold
    int kws = 0;
    for (int k = kMaxK; k >= 1; --k)
        if (ws_bytes >= qsim_workspace_bytes(n_qubits, dt, k)) { kws = k; break; }
    if (kws == 0) return fail(QSIM_E_INVALID, "workspace too small");
    if (init != QSIM_INIT_ZERO && init != QSIM_INIT_UNIFORM && init != QSIM_INIT_KEEP)
        return fail(QSIM_E_INVALID, "unknown init");
    auto* s = new qsim_state_s;
    s->n = n_qubits;
    s->dbl = dbl;
    s->psi = dev_amps;
    s->ws = static_cast<char*>(dev_workspace);
    s->ws_bytes = ws_bytes;
    s->st = static_cast<hipStream_t>(hip_stream);
    s->kmax_ws = kws;
    if (init != QSIM_INIT_KEEP) {
        hipError_t e = launch_init(s->psi, s->n, s->dbl, init == QSIM_INIT_ZERO ? 0 : 1, s->st);
        if (e != hipSuccess) { delete s; return hip_fail(e, "init launch"); }
    }
    *out = s;
    return QSIM_OK;
}

qsim_status qsim_destroy(qsim_state s) {
    delete s;
    return QSIM_OK;
}

qsim_status qsim_init_state(qsim_state s, qsim_init init) {
    if (qsim_status r = check_state(s)) return r;
    s->stats_ready = false;
    if (init == QSIM_INIT_KEEP) return QSIM_OK;
    if (init != QSIM_INIT_ZERO && init != QSIM_INIT_UNIFORM) return fail(QSIM_E_INVALID, "unknown init");
    HIP_TRY(launch_init(s->psi, s->n, s->dbl, init == QSIM_INIT_ZERO ? 0 : 1, s->st), "init launch");
    return QSIM_OK;
}

qsim_status qsim_apply_cluster(qsim_state s, int k, const int32_t* qubits, const double* mat) {
    if (qsim_status r = check_state(s)) return r;
    s->stats_ready = false;
    if (!qubits || !mat) return fail(QSIM_E_INVALID, "null argument");
    if (k < 1 || k > kMaxGateQ) return fail(QSIM_E_UNSUPPORTED, "k must be in [1, 6]");
    if (k > s->kmax_ws) return fail(QSIM_E_UNSUPPORTED, "workspace sized for smaller clusters");
    if (k > s->n) return fail(QSIM_E_INVALID, "k exceeds the number of qubits");
    qsim_gate g;
    std::memset(&g, 0, sizeof(g));
    g.kind = G_DENSE;
    g.k = k;
    for (int j = 0; j < k; ++j) g.qubits[j] = qubits[j];
    g.mat = mat;
    if (qsim_status r = check_gate(s->n, g, 0)) return r;
    Chunk c;
    if (qsim_status r = add_gate(s, c, &g, 0)) return r;
    return flush(s, c);
}

qsim_status qsim_apply_diag(qsim_state s, int n_pairs, const int32_t* cz_pairs, int n_phase,
                            const int32_t* phase_qubits, const double* phase_theta) {
    if (qsim_status r = check_state(s)) return r;
    s->stats_ready = false;
    if (n_pairs < 0 || n_phase < 0) return fail(QSIM_E_INVALID, "negative count");
    if ((n_pairs && !cz_pairs) || (n_phase && (!phase_qubits || !phase_theta)))
        return fail(QSIM_E_INVALID, "null argument");
    if (n_pairs > kEpiMax || n_phase > kEpiMax) return fail(QSIM_E_UNSUPPORTED, "at most 64 pairs and 64 phases");
    std::vector<std::pair<int, int>> pairs;
    std::vector<std::pair<int, double>> phases;
    for (int i = 0; i < n_pairs; ++i) {
        const int a = cz_pairs[2 * i], b = cz_pairs[2 * i + 1];
        if (a < 0 || a >= s->n || b < 0 || b >= s->n || a == b) return fail(QSIM_E_INVALID, "bad CZ pair");
        pairs.emplace_back(a, b);
    }
    for (int i = 0; i < n_phase; ++i) {
        const int q = phase_qubits[i];
        if (q < 0 || q >= s->n) return fail(QSIM_E_INVALID, "bad phase qubit");
        phases.emplace_back(q, phase_theta[i]);
    }
    Chunk c;
    if (qsim_status r = add_diag(s, c, pairs, phases)) return r;
    return flush(s, c);
}

namespace {
// Tile geometry of a bit permutation (m <= kPermMaxBits moving locations):
// the moving locations and the lowest fixed ones, up to 12 bits, so loads
// and stores run over the lowest bits.
PermGeom perm_geom(int n, int m, const int32_t* from, const int32_t* to) {
    PermGeom pg{};
    uint64_t tile = 0;
    for (int j = 0; j < m; ++j) tile |= uint64_t(1) << from[j];
    const int nt = std::min(n, kPermMaxBits);
    for (int b = 0; b < n && __builtin_popcountll(tile) < nt; ++b) tile |= uint64_t(1) << b;
    int tau_of[64];
    for (int b = 0; b < n; ++b)
        if (tile >> b & 1) {
            tau_of[b] = pg.nt;
            pg.tb[pg.nt++] = b;
        }
    for (int j = 0; j < pg.nt; ++j) pg.to[j] = j;
    for (int j = 0; j < m; ++j) pg.to[tau_of[from[j]]] = tau_of[to[j]];
    return pg;
}

// Bit locations for a run that starts from the uniform state (any relabelling
// of it is the same state, so the first layout is free). Cluster kernels are
// slowest with targets on the lowest six locations (a scattered gather) or the
// top three (measured per target position at 28 qubits): the qubits the
// schedule's clusters use least go there. At most six transpositions (twelve
// moving locations), so one permutation pass restores the order at the end.
// Returns loc[q] (the identity when nothing moves).
std::vector<int> choose_layout(int n, const Schedule& S) {
    std::vector<int> loc(n);
    for (int q = 0; q < n; ++q) loc[q] = q;
    if (n < 16) return loc;
    std::vector<int> use(n, 0);
    for (const SOp& op : S.ops)
        if (op.kind == OP_CLUSTER)
            for (int j = 0; j < op.k; ++j) use[op.qubits[j]] += 8 - op.k;  // narrower clusters suffer more
    auto slow = [&](int l) { return l < 6 || l >= n - 3; };
    int n_slow = 0;
    for (int l = 0; l < n; ++l) n_slow += slow(l);
    std::vector<int> order(n);
    for (int q = 0; q < n; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return use[a] < use[b]; });
    std::vector<char> want_slow(n, 0);  // the least used qubits
    for (int i = 0; i < n_slow; ++i) want_slow[order[i]] = 1;
    std::vector<int> out, in;  // heavily used qubits on slow locations, lightly used ones elsewhere
    for (int i = n - 1; i >= 0; --i)
        if (slow(loc[order[i]]) && !want_slow[order[i]]) out.push_back(order[i]);
    for (int i = 0; i < n; ++i)
        if (!slow(loc[order[i]]) && want_slow[order[i]]) in.push_back(order[i]);
    const size_t swaps = std::min<size_t>({out.size(), in.size(), size_t(kPermMaxBits / 2)});
    for (size_t i = 0; i < swaps; ++i) std::swap(loc[out[i]], loc[in[i]]);
    return loc;
}
}  // namespace

qsim_status qsim_permute_qubits(qsim_state s, int m, const int32_t* from, const int32_t* to) {
    if (qsim_status r = check_state(s)) return r;
    if (m < 0 || m > kPermMaxBits) return fail(QSIM_E_UNSUPPORTED, "at most 12 bit locations per permutation");
    if (m && (!from || !to)) return fail(QSIM_E_INVALID, "null argument");
    uint64_t sf = 0, st = 0;
    for (int j = 0; j < m; ++j) {
        if (from[j] < 0 || from[j] >= s->n || to[j] < 0 || to[j] >= s->n)
            return fail(QSIM_E_INVALID, "bit location out of range");
        if ((sf >> from[j] & 1) || (st >> to[j] & 1)) return fail(QSIM_E_INVALID, "repeated bit location");
        sf |= uint64_t(1) << from[j];
        st |= uint64_t(1) << to[j];
    }
    if (sf != st) return fail(QSIM_E_INVALID, "from and to must list the same bit locations");
    bool identity = true;
    for (int j = 0; j < m; ++j) identity &= from[j] == to[j];
    if (identity) return QSIM_OK;
    s->stats_ready = false;
    HIP_TRY(launch_permute(s->psi, s->dbl, s->n, perm_geom(s->n, m, from, to), s->st), "permute launch");
    return QSIM_OK;
}

qsim_status qsim_apply_gate(qsim_state s, const qsim_gate* gate) {
    if (qsim_status r = check_state(s)) return r;
    s->stats_ready = false;
    if (!gate) return fail(QSIM_E_INVALID, "null gate");
    if (qsim_status r = check_gate(s->n, *gate, 0)) return r;
    if (gate->kind == G_DENSE && gate->k > s->kmax_ws)
        return fail(QSIM_E_UNSUPPORTED, "workspace sized for smaller clusters");
    Chunk c;
    if (qsim_status r = add_gate(s, c, gate, 0)) return r;
    return flush(s, c);
}

qsim_status qsim_run_circuit(qsim_state s, const qsim_gate* gates, int n_gates, const qsim_run_opts* opts,
                             qsim_run_stats* stats) {
    const auto t0 = std::chrono::steady_clock::now();
    if (qsim_status r = check_state(s)) return r;
    if (n_gates < 0 || (n_gates && !gates)) return fail(QSIM_E_INVALID, "bad gate list");
    for (int i = 0; i < n_gates; ++i)
        if (qsim_status r = check_gate(s->n, gates[i], i)) return r;
    SchedOpts so = to_sched_opts(opts);
    if (so.mode != 0 && (so.kmax < 1 || so.kmax > kMaxK)) return fail(QSIM_E_UNSUPPORTED, "kmax must be in [1, 7]");
    so.kmax = std::min(so.kmax, max_cluster_k(s->dbl, s->n));  // 7 only where a 7-qubit kernel exists
    so.fold_start = fold_start_for(s->dbl, s->n);
    if (so.mode != 0 && so.kmax > s->kmax_ws) return fail(QSIM_E_UNSUPPORTED, "workspace sized for smaller clusters");
    s->stats_ready = false;
    for (int i = 0; i < n_gates; ++i)
        if (gates[i].kind == G_DENSE && gates[i].k > s->kmax_ws)
            return fail(QSIM_E_UNSUPPORTED, "workspace sized for smaller clusters");
    const std::vector<SGate> sgates = to_sgates(gates, n_gates);
    Schedule S = make_schedule(s->n, sgates, so, cost_fn(opts, s->n, s->dbl));
    // the folded start (the relabelling below keeps it)
    const int fold_kind = S.uniform_init && g_fold_init ? schedule_fold_kind(S.ops, sgates, so.fold_start) : 0;
    // qubit mapping: from the uniform state the first layout is free; the run
    // applies the relabelled gates and one permutation pass restores the order
    std::vector<qsim_gate> mapped;
    int32_t pfrom[kPermMaxBits], pto[kPermMaxBits];
    int pm = 0;
    if (g_map_qubits && S.uniform_init && so.mode != 0) {
        const std::vector<int> loc = choose_layout(s->n, S);
        for (int q = 0; q < s->n; ++q)
            if (loc[q] != q) {
                pfrom[pm] = loc[q];
                pto[pm] = q;
                ++pm;
            }
        if (pm) {  // the same schedule on the relabelled qubits
            mapped.assign(gates, gates + n_gates);
            for (qsim_gate& g : mapped)
                for (int j = 0; j < gate_nq(g); ++j) g.qubits[j] = loc[g.qubits[j]];
            gates = mapped.data();
            for (SOp& op : S.ops) {
                for (int j = 0; j < op.k; ++j) op.qubits[j] = loc[op.qubits[j]];
                if (op.kind == OP_CLUSTER) std::sort(op.qubits, op.qubits + op.k);
            }
        }
    }
    const auto t1 = std::chrono::steady_clock::now();

    qsim_run_stats st;
    std::memset(&st, 0, sizeof(st));
    st.n_gates_applied = S.n_applied;
    const bool rec = opts && opts->record_timings;
    if (rec) {
        // the events of the previous run are reused: wait until they have fired
        HIP_TRY(hipStreamSynchronize(s->st), "stream sync");
        s->recs.clear();
        s->pool_used = 0;
    }
    s->recording = rec;
    struct RecOff {
        qsim_state_s* s;
        ~RecOff() { s->recording = false; }
    } rec_off{s};
    // the uniform start and a leading cluster are written in one pass; with a
    // second cluster of 6 qubits (complex64, fp16-halves kernel) that one too
    const bool fold = fold_kind >= 1;
    const bool fold2 = fold_kind >= 2;  // kinds 2-4: complex64, 6-qubit clusters on the fp16-halves kernel
    // the learned model also picks each cluster's kernel variant (unless one is forced)
    const bool learned_variants = opts && opts->scheduler == QSIM_SCHED_LEARNED && so.mode == 2 &&
                                  learned_model_loaded() && get_cluster_variant() < 0;
    // consecutive clusters of <= 5 qubits on a complex64 state go in pairs
    const bool pairing = g_pair && !s->dbl && s->n >= 11 && s->kmax_ws >= 5 && so.mode != 0;
    auto small = [&](size_t i) { return S.ops[i].kind == OP_CLUSTER && S.ops[i].k <= 5; };
    if (S.uniform_init && !fold) HIP_TRY(launch_init(s->psi, s->n, s->dbl, 1, s->st), "init launch");
    Chunk c;
    for (size_t oi = 0; oi < S.ops.size(); ++oi) {
        const SOp& op = S.ops[oi];
        qsim_status r = QSIM_OK;
        if (oi == 0 && fold2) {
            const SOp& op2 = S.ops[1];
            r = add_fold2(s, c, op, op2, gates);
            st.n_clusters_by_k[op.k]++;
            st.n_clusters_by_k[op2.k]++;
            st.n_gates_fused_epilogue += (int)(op.epi.size() + op2.epi.size());
            ++oi;
        } else if (oi == 0 && fold) {
            r = add_cluster(s, c, op.k, op.qubits, gates, op.members, op.epi, true);
            st.n_clusters_by_k[op.k]++;
            st.n_gates_fused_epilogue += (int)op.epi.size();
        } else if (pairing && g_pair == 1 && oi + 1 < S.ops.size() && small(oi) && small(oi + 1)) {
            const SOp& op2 = S.ops[oi + 1];
            r = add_pair(s, c, op, &op2, gates);
            st.n_clusters_by_k[op.k]++;
            st.n_clusters_by_k[op2.k]++;
            st.n_gates_fused_epilogue += (int)(op.epi.size() + op2.epi.size());
            ++oi;
        } else if (pairing && g_pair == 2 && small(oi)) {
            r = add_pair(s, c, op, nullptr, gates);  // one cluster through the same kernel
            st.n_clusters_by_k[op.k]++;
            st.n_gates_fused_epilogue += (int)op.epi.size();
        } else if (op.kind == OP_GATE) {
            r = add_gate(s, c, gates, op.members[0]);
        } else if (op.kind == OP_DIAG) {
            std::vector<std::pair<int, int>> pairs;
            std::vector<std::pair<int, double>> phases;
            for (int gi : op.members) {
                if (gates[gi].kind == G_CZ) pairs.emplace_back(gates[gi].qubits[0], gates[gi].qubits[1]);
                else phases.emplace_back(gates[gi].qubits[0], gate_phase_angle(gates[gi].kind, gates[gi].theta));
            }
            r = add_diag(s, c, pairs, phases);
            st.n_diag_ops++;
        } else {
            r = add_cluster(s, c, op.k, op.qubits, gates, op.members, op.epi);
            if (r == QSIM_OK && learned_variants) {  // the variant the model predicts faster for these targets
                int v = -1;
                learned_cost_best_us(s->n, s->dbl, op.k, op.qubits, (int)op.epi.size(), &v);
                c.items.back().variant = v;
            }
            st.n_clusters_by_k[op.k]++;
            st.n_gates_fused_epilogue += (int)op.epi.size();
        }
        if (r != QSIM_OK) return r;
        st.n_ops++;
    }
    // fused_stats: the last op, when it is a cluster of a kernel that can, also
    // sums the quantities qsim_probs reports, so they need no further pass
    if (opts && opts->fused_stats && !c.items.empty()) {
        Chunk::Item& last = c.items.back();
        // the sums come from the direct kernels: a staged choice of the model
        // gives way, since the sums save a whole pass over the state
        const ClusterGeom& lg = last.geom;
        if (last.kind == 0 && last.variant == 1 && cluster_stats_supported(s->dbl, lg.n, lg.k, last.layout, 0))
            last.variant = 0;
        const int v = last.variant >= 0 ? last.variant : cluster_variant_for(s->dbl, lg, last.layout);
        if (last.kind == 0 && cluster_stats_supported(s->dbl, lg.n, lg.k, last.layout, v)) last.stats = true;
    }
    if (qsim_status r = flush(s, c)) return r;
    if (pm) {  // back to the caller's qubit order (sums of a fused_stats pass do not change)
        OpRecord r;
        std::memset(&r, 0, sizeof(r));
        r.kind = 9;
        r.k = pm;
        for (int j = 0; j < std::min(pm, kMaxK); ++j) r.qubits[j] = pto[j];
        HIP_TRY(rec_begin(s, r), "event record");
        HIP_TRY(launch_permute(s->psi, s->dbl, s->n, perm_geom(s->n, pm, pfrom, pto), s->st), "permute launch");
        HIP_TRY(rec_end(s, r), "event record");
        st.n_ops++;
    }
    const auto t2 = std::chrono::steady_clock::now();
    st.schedule_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    st.total_ms = std::chrono::duration<double, std::milli>(t2 - t0).count();
    if (stats) *stats = st;
    return QSIM_OK;
}

qsim_status qsim_probs(qsim_state s, void* dev_out, qsim_dtype out_dt, double* norm, double* sum_p2,
                       double* entropy_nats) {
    if (qsim_status r = check_state(s)) return r;
    if (dev_out && out_dt != QSIM_C64 && out_dt != QSIM_C128) return fail(QSIM_E_INVALID, "unknown out dtype");
    double* part = reinterpret_cast<double*>(s->ws);
    double* res = reinterpret_cast<double*>(s->ws + kResOff);
    if (!dev_out && s->stats_ready) {  // the sums of the last run's final pass
        HIP_TRY(launch_reduce_stats(part, s->stats_blocks, res, s->st), "stats reduce launch");
    } else {
        s->stats_ready = false;  // the partial area is rewritten
        HIP_TRY(launch_stats(s->psi, s->dbl, s->n, dev_out, out_dt == QSIM_C128, part, res, s->st), "stats launch");
    }
    double h[8];
    HIP_TRY(hipMemcpyAsync(h, res, 8 * sizeof(double), hipMemcpyDeviceToHost, s->st), "stats copy");
    HIP_TRY(hipStreamSynchronize(s->st), "stats sync");
    if (norm) *norm = h[0];
    if (sum_p2) *sum_p2 = h[1];
    if (entropy_nats) *entropy_nats = h[2];
    return QSIM_OK;
}

qsim_status qsim_compare(qsim_state s, const void* dev_ref, qsim_dtype ref_dt, double* fidelity,
                         double* max_abs_diff) {
    if (qsim_status r = check_state(s)) return r;
    if (!dev_ref) return fail(QSIM_E_INVALID, "null reference");
    if (ref_dt != QSIM_C64 && ref_dt != QSIM_C128) return fail(QSIM_E_INVALID, "unknown reference dtype");
    double* part = reinterpret_cast<double*>(s->ws);
    double* res = reinterpret_cast<double*>(s->ws + kResOff);
    s->stats_ready = false;  // the partial area is rewritten
    HIP_TRY(launch_compare(s->psi, s->dbl, s->n, dev_ref, ref_dt == QSIM_C128, part, res, s->st), "compare launch");
    double h[8];
    HIP_TRY(hipMemcpyAsync(h, res, 8 * sizeof(double), hipMemcpyDeviceToHost, s->st), "compare copy");
    HIP_TRY(hipStreamSynchronize(s->st), "compare sync");
    const double dot2 = h[0] * h[0] + h[1] * h[1];
    if (fidelity) *fidelity = (h[2] > 0 && h[3] > 0) ? dot2 / (h[2] * h[3]) : 0.0;
    if (max_abs_diff) *max_abs_diff = h[4];
    return QSIM_OK;
}

qsim_status qsim_state_changed(qsim_state s) {
    if (qsim_status r = check_state(s)) return r;
    s->stats_ready = false;  // the sums a fused_stats run left describe the old amplitudes
    return QSIM_OK;
}

qsim_status qsim_sync(qsim_state s) {
    if (qsim_status r = check_state(s)) return r;
    HIP_TRY(hipStreamSynchronize(s->st), "stream sync");
    HIP_TRY(hipGetLastError(), "pending error");
    return QSIM_OK;
}

const char* qsim_last_error(void) { return g_err.c_str(); }

qsim_status qsim_set_option(int option, int value) {
    if (option == QSIM_OPT_CLUSTER_VARIANT) {
        if (value < -1 || value > 1) return fail(QSIM_E_INVALID, "cluster variant must be -1, 0 or 1");
        set_cluster_variant(value);
        return QSIM_OK;
    }
    if (option == QSIM_OPT_BATCH_GRID) {
        if (value < 0 || value > (1 << 20)) return fail(QSIM_E_INVALID, "batch grid must be in [0, 2^20]");
        g_batch_grid = value;
        return QSIM_OK;
    }
    if (option == QSIM_OPT_BATCH_PAD) {
        if (value < 0 || value > 1) return fail(QSIM_E_INVALID, "batch padding must be 0 or 1");
        g_batch_pad = value;
        return QSIM_OK;
    }
    if (option == QSIM_OPT_K6_KERNEL) {
        if (value < 0 || value > 2) return fail(QSIM_E_INVALID, "k = 6 kernel must be 0, 1 or 2");
        g_k6_kernel = value;
        return QSIM_OK;
    }
    if (option == QSIM_OPT_FOLD_INIT) {
        if (value < 0 || value > 2) return fail(QSIM_E_INVALID, "fold_init must be 0, 1 or 2");
        g_fold_init = value;
        return QSIM_OK;
    }
    if (option == QSIM_OPT_DEVIATIONS) {
        if (value < 0 || value > 1) return fail(QSIM_E_INVALID, "deviations must be 0 or 1");
        g_deviations = value;
        return QSIM_OK;
    }
    if (option == QSIM_OPT_FOLD_TABLE) {
        if (value < 0 || value > 1) return fail(QSIM_E_INVALID, "fold_table must be 0 or 1");
        g_fold_table = value;
        return QSIM_OK;
    }
    if (option == QSIM_OPT_PAIR_TILE) {
        if (value != 10 && value != 11) return fail(QSIM_E_INVALID, "pair tile bits must be 10 or 11");
        g_pair_tile = value;
        return QSIM_OK;
    }
    if (option == QSIM_OPT_PAIR) {
        if (value < 0 || value > 2) return fail(QSIM_E_INVALID, "pair must be 0, 1 or 2");
        g_pair = value;
        return QSIM_OK;
    }
    if (option == QSIM_OPT_CLUSTER_SETS) {
        if (value < 0 || value > 1) return fail(QSIM_E_INVALID, "cluster_sets must be 0 or 1");
        g_cluster_sets = value;
        return QSIM_OK;
    }
    if (option == QSIM_OPT_BATCH_ORDER) {
        if (value < 0 || value > 2) return fail(QSIM_E_INVALID, "batch order must be 0, 1 or 2");
        g_batch_order = value;
        return QSIM_OK;
    }
    if (option == QSIM_OPT_CHECK_UNITARY) {
        if (value < 0 || value > 1) return fail(QSIM_E_INVALID, "check_unitary must be 0 or 1");
        g_check_unitary = value;
        return QSIM_OK;
    }
    if (option == QSIM_OPT_MAP_QUBITS) {
        if (value < 0 || value > 1) return fail(QSIM_E_INVALID, "map_qubits must be 0 or 1");
        g_map_qubits = value;
        return QSIM_OK;
    }
    if (option == QSIM_OPT_BATCH_ITEM_TILES) {
        if (value < 1 || value > 4096 || (value & (value - 1)))
            return fail(QSIM_E_INVALID, "tiles per batch item must be a power of two in [1, 4096]");
        g_batch_item_tiles = value;
        return QSIM_OK;
    }
    return fail(QSIM_E_INVALID, "unknown option");
}

qsim_status qsim_set_tune_entry(qsim_dtype dt, int k, int low_class, int variant) {
    if (dt != QSIM_C64 && dt != QSIM_C128) return fail(QSIM_E_INVALID, "unknown dtype");
    if (k < 1 || k > kMaxK || low_class < 0 || low_class >= kLowClasses || variant < 0 || variant > 1)
        return fail(QSIM_E_INVALID, "tune entry out of range");
    set_tune_entry(dt == QSIM_C128, k, low_class, variant);
    return QSIM_OK;
}

qsim_status qsim_set_cost_table(qsim_dtype dt, const double* us_by_k, int n_ref) {
    if (dt != QSIM_C64 && dt != QSIM_C128) return fail(QSIM_E_INVALID, "unknown dtype");
    if (!us_by_k || n_ref < 1 || n_ref > 40) return fail(QSIM_E_INVALID, "bad cost table");
    for (int k = 0; k <= kMaxK; ++k)
        if (!(us_by_k[k] > 0.0)) return fail(QSIM_E_INVALID, "costs must be positive");
    for (int k = 0; k <= kMaxK; ++k) g_cost_us[dt == QSIM_C128][k] = us_by_k[k];
    g_cost_nref[dt == QSIM_C128] = n_ref;
    return QSIM_OK;
}

int qsim_get_tune_entry(qsim_dtype dt, int k, int low_class) {
    if ((dt != QSIM_C64 && dt != QSIM_C128) || k < 1 || k > kMaxK || low_class < 0 || low_class >= kLowClasses)
        return -1;
    return get_tune_entry(dt == QSIM_C128, k, low_class);
}

int qsim_get_option(int option) {
    if (option == QSIM_OPT_CLUSTER_VARIANT) return get_cluster_variant();
    if (option == QSIM_OPT_BATCH_GRID) return g_batch_grid;
    if (option == QSIM_OPT_BATCH_PAD) return g_batch_pad;
    if (option == QSIM_OPT_BATCH_ITEM_TILES) return g_batch_item_tiles;
    if (option == QSIM_OPT_K6_KERNEL) return g_k6_kernel;
    if (option == QSIM_OPT_FOLD_INIT) return g_fold_init;
    if (option == QSIM_OPT_FOLD_TABLE) return g_fold_table;
    if (option == QSIM_OPT_DEVIATIONS) return g_deviations;
    if (option == QSIM_OPT_PAIR) return g_pair;
    if (option == QSIM_OPT_PAIR_TILE) return g_pair_tile;
    if (option == QSIM_OPT_CLUSTER_SETS) return g_cluster_sets;
    if (option == QSIM_OPT_BATCH_ORDER) return g_batch_order;
    if (option == QSIM_OPT_CHECK_UNITARY) return g_check_unitary;
    if (option == QSIM_OPT_MAP_QUBITS) return g_map_qubits;
    return -1;
}

qsim_status qsim_op_timings(qsim_state s, int32_t* op_kind, int32_t* op_k, int32_t* op_qubits,
                            int32_t* op_epi, float* ms, int cap, int* n_ops) {
    if (qsim_status r = check_state(s)) return r;
    HIP_TRY(hipStreamSynchronize(s->st), "stream sync");
    if (n_ops) *n_ops = (int)s->recs.size();
    if ((int)s->recs.size() > cap) return fail(QSIM_E_INVALID, "cap too small");
    for (size_t i = 0; i < s->recs.size(); ++i) {
        const OpRecord& r = s->recs[i];
        if (op_kind) op_kind[i] = r.kind;
        if (op_k) op_k[i] = r.k;
        if (op_qubits)
            for (int j = 0; j < QSIM_MAX_CLUSTER; ++j)  // diagonal passes and builds have no qubit list
                op_qubits[QSIM_MAX_CLUSTER * i + j] = (r.kind != 1 && r.kind != 5 && j < r.k) ? r.qubits[j] : -1;
        if (op_epi) op_epi[i] = r.flags;
        if (ms) {
            float t = 0.f;
            HIP_TRY(hipEventElapsedTime(&t, r.ev0, r.ev1), "event time");
            ms[i] = t;
        }
    }
    return QSIM_OK;
}

qsim_status qsim_schedule(int n_qubits, const qsim_gate* gates, int n_gates, const qsim_run_opts* opts,
                          int32_t* gate_op, int32_t* gate_role, int32_t* op_kind, int32_t* op_k,
                          int32_t* op_qubits, int op_cap, int* n_ops) {
    if (n_qubits < 1 || n_qubits > 64) return fail(QSIM_E_UNSUPPORTED, "n_qubits out of range");
    if (n_gates < 0 || (n_gates && !gates)) return fail(QSIM_E_INVALID, "bad gate list");
    for (int i = 0; i < n_gates; ++i)
        if (qsim_status r = check_gate(n_qubits, gates[i], i)) return r;
    SchedOpts so = to_sched_opts(opts);
    if (so.mode != 0 && (so.kmax < 1 || so.kmax > kMaxK)) return fail(QSIM_E_UNSUPPORTED, "kmax must be in [1, 7]");
    const bool sdbl = opts && opts->schedule_dtype == QSIM_C128;
    so.kmax = std::min(so.kmax, max_cluster_k(sdbl, n_qubits));  // as qsim_run_circuit would
    so.fold_start = fold_start_for(sdbl, n_qubits);
    const Schedule S = make_schedule(n_qubits, to_sgates(gates, n_gates), so, cost_fn(opts, n_qubits, sdbl));
    if (n_ops) *n_ops = (int)S.ops.size();
    if ((int)S.ops.size() > op_cap) return fail(QSIM_E_INVALID, "op_cap too small");
    if (gate_op)
        for (int i = 0; i < n_gates; ++i) gate_op[i] = -1;
    for (int o = 0; o < (int)S.ops.size(); ++o) {
        const SOp& op = S.ops[o];
        if (op_kind) op_kind[o] = op.kind;
        if (op_k) op_k[o] = op.k;
        if (op_qubits)
            for (int j = 0; j < QSIM_MAX_CLUSTER; ++j) op_qubits[QSIM_MAX_CLUSTER * o + j] = j < op.k ? op.qubits[j] : -1;
        for (int gi : op.members) {
            if (gate_op) gate_op[gi] = o;
            if (gate_role) gate_role[gi] = op.kind == OP_DIAG ? 2 : 0;
        }
        for (int gi : op.epi) {
            if (gate_op) gate_op[gi] = o;
            if (gate_role) gate_role[gi] = 1;
        }
    }
    return QSIM_OK;
}

qsim_status qsim_stage_schedule(int n_qubits, const qsim_gate* gates, int n_gates, const qsim_stage_opts* opts,
                                int32_t* gate_stage, int32_t* stage_loc, int32_t* stage_clusters, int max_stages,
                                int* n_stages) {
    if (n_qubits < 1 || n_qubits > 64) return fail(QSIM_E_UNSUPPORTED, "n_qubits out of range");
    if (!opts) return fail(QSIM_E_INVALID, "null options");
    if (n_gates < 0 || (n_gates && !gates)) return fail(QSIM_E_INVALID, "bad gate list");
    for (int i = 0; i < n_gates; ++i)
        if (qsim_status r = check_gate(n_qubits, gates[i], i)) return r;
    if (opts->n_local < 1 || opts->n_local > n_qubits || 2 * opts->n_local < n_qubits)
        return fail(QSIM_E_INVALID, "n_local must be in [n_qubits / 2, n_qubits]");
    if (opts->kmax < 0 || opts->kmax > kMaxK) return fail(QSIM_E_UNSUPPORTED, "kmax must be in [0, 7]");
    StageOpts so;
    so.n_local = opts->n_local;
    so.spec_cz = opts->specialize & 1;
    so.spec_diag1 = (opts->specialize & 2) != 0;
    so.search = opts->search != 0;
    so.early_swaps = opts->early_swaps != 0;
    so.kmax = opts->kmax;
    so.fuse_diag = opts->fuse_diag != 0;
    so.skip_initial_h = opts->skip_initial_h != 0;
    so.skip_trailing_diag = opts->skip_trailing_diag != 0;
    const StagePlan P = make_stage_plan(n_qubits, to_sgates(gates, n_gates), so);
    if (!P.ok) return fail(QSIM_E_INVALID, "a gate gathers more qubits than n_local locations hold");
    const int ns = (int)P.loc.size();
    if (n_stages) *n_stages = ns;
    if (ns > max_stages) return fail(QSIM_E_INVALID, "max_stages too small");
    if (gate_stage)
        for (int i = 0; i < n_gates; ++i) gate_stage[i] = P.gate_stage[i];
    for (int st = 0; st < ns; ++st) {
        if (stage_loc)
            for (int q = 0; q < n_qubits; ++q) stage_loc[st * n_qubits + q] = P.loc[st][q];
        if (stage_clusters) stage_clusters[st] = so.kmax > 0 ? P.n_clusters[st] : -1;
    }
    return QSIM_OK;
}

}  // extern "C"
