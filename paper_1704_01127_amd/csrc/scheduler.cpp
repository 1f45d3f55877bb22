// Clustering scheduler (Haener & Steiger, Sec. 3.6.1, step 2; Table 1).
//
// Gates on different qubits commute, gates on a common qubit keep their
// order, so the circuit is a DAG of per-qubit gate queues; a gate is ready
// when it heads the queue of every qubit it touches. Clusters are grown
// greedily: starting from a seed, repeatedly take the ready gate that adds the
// fewest new qubits while the cluster stays within kmax qubits. A small local
// search tries every ready gate as the seed and keeps the cluster with the
// most gates, before the remaining gates are assigned to further clusters.
//
// Cost-driven mode (analytic or learned cost model): the complete greedy
// schedule is built for every cap k <= kmax and the one with the smallest
// predicted total time is kept (per-cluster "gates per microsecond" choices
// are myopic: a wide cluster can look cheap per gate and still leave more
// total work).
//
// Extensions for the GPU kernels (both exact, as diagonal gates commute):
//   * a cluster made only of diagonal gates becomes a diagonal pass, which
//     then absorbs every ready diagonal gate;
//   * with fuse_diag, once no gate fits a cluster any more, ready diagonal
//     gates are attached to it and applied while its results are stored; a
//     qubit touched by such a gate accepts only diagonal gates afterwards.
#include "scheduler.h"

#include <algorithm>
#include <cstring>
#include <future>

#include "qsim_internal.h"

namespace qsim {
namespace {

inline int popc(uint64_t x) { return __builtin_popcountll(x); }

struct Dag {
    int n;
    const std::vector<SGate>* g;
    std::vector<std::vector<int>> queue;  // per qubit, gate indices in program order
    std::vector<uint64_t> mask;           // per gate, qubit bit mask

    bool ready(const std::vector<int>& head, int gi) const {
        const SGate& s = (*g)[gi];
        for (int j = 0; j < s.nq; ++j) {
            const auto& qq = queue[s.q[j]];
            const int h = head[s.q[j]];
            if (h >= (int)qq.size() || qq[h] != gi) return false;
        }
        return true;
    }
    void pop(std::vector<int>& head, int gi) const {
        const SGate& s = (*g)[gi];
        for (int j = 0; j < s.nq; ++j) head[s.q[j]]++;
    }
    // Ready gates, ascending index.
    void ready_list(const std::vector<int>& head, std::vector<int>& out) const {
        out.clear();
        for (int q = 0; q < n; ++q) {
            if (head[q] >= (int)queue[q].size()) continue;
            const int gi = queue[q][head[q]];
            if (ready(head, gi)) out.push_back(gi);
        }
        std::sort(out.begin(), out.end());
        out.erase(std::unique(out.begin(), out.end()), out.end());
    }
};

struct Grown {
    uint64_t Q = 0;
    std::vector<int> members, epi;
    std::vector<int> head;
    int n_gates() const { return (int)(members.size() + epi.size()); }
};

// Grow a cluster from `seed` with at most `kcap` qubits.
Grown grow(const Dag& d, const std::vector<int>& head0, int seed, int kcap, bool fuse_diag) {
    const auto& G = *d.g;
    Grown r;
    r.head = head0;
    r.Q = d.mask[seed];
    r.members.push_back(seed);
    d.pop(r.head, seed);
    uint64_t sealed = 0;
    int n_epi_cz = 0, n_epi_ph = 0;
    std::vector<int> rl;
    for (;;) {
        d.ready_list(r.head, rl);
        // a gate that joins the matrix: fewest new qubits, then lowest index
        int best = -1, best_new = 1 << 30;
        for (int gi : rl) {
            const uint64_t m = d.mask[gi];
            if ((m & sealed) || popc(r.Q | m) > kcap) continue;
            const int nw = popc(m & ~r.Q);
            if (nw < best_new) { best = gi; best_new = nw; }
        }
        if (best >= 0) {
            r.members.push_back(best);
            r.Q |= d.mask[best];
            d.pop(r.head, best);
            continue;
        }
        if (!fuse_diag) break;
        // nothing fits: attach the lowest-index ready diagonal gate
        for (int gi : rl) {
            if (!G[gi].diag) continue;
            const bool cz = G[gi].kind == G_CZ;
            if ((cz && n_epi_cz >= kEpiMax) || (!cz && n_epi_ph >= kEpiMax)) continue;
            best = gi;
            break;
        }
        if (best < 0) break;
        r.epi.push_back(best);
        sealed |= d.mask[best];
        if (G[best].kind == G_CZ) ++n_epi_cz; else ++n_epi_ph;
        d.pop(r.head, best);
    }
    return r;
}

bool all_diag(const std::vector<SGate>& G, const Grown& c) {
    for (int i : c.members) if (!G[i].diag) return false;
    return true;
}

// Greedy clustering with at most kcap qubits per cluster (gates with more
// qubits form a cluster of their own width).
std::vector<SOp> greedy_ops(int n, const std::vector<SGate>& gates, const std::vector<char>& dropped, int n_applied,
                            int kcap_in, bool fuse_diag) {
    const int ng = (int)gates.size();
    std::vector<SOp> out;
    Dag d;
    d.n = n;
    d.g = &gates;
    d.queue.assign(n, {});
    d.mask.assign(ng, 0);
    for (int i = 0; i < ng; ++i) {
        for (int j = 0; j < gates[i].nq; ++j) d.mask[i] |= uint64_t(1) << gates[i].q[j];
        if (dropped[i]) continue;
        for (int j = 0; j < gates[i].nq; ++j) d.queue[gates[i].q[j]].push_back(i);
    }
    std::vector<int> head(n, 0);
    int remaining = n_applied;
    std::vector<int> rl;
    const int kmax = kcap_in;

    while (remaining > 0) {
        d.ready_list(head, rl);
        Grown best;
        int best_score = -1;
        for (int seed : rl) {
            // a gate wider than kmax (a dense gate) forms a cluster of its own width
            const int khi = std::max(kmax, popc(d.mask[seed]));
            Grown c = grow(d, head, seed, khi, fuse_diag);
            if (c.n_gates() > best_score) { best_score = c.n_gates(); best = std::move(c); }
        }
        SOp op;
        if (all_diag(gates, best)) {
            // a diagonal pass: take every ready diagonal gate, repeatedly
            op.kind = OP_DIAG;
            int ncz = 0, nph = 0;
            for (;;) {
                d.ready_list(head, rl);
                bool took = false;
                for (int gi : rl) {
                    if (!gates[gi].diag) continue;
                    const bool cz = gates[gi].kind == G_CZ;
                    if ((cz && ncz >= kEpiMax) || (!cz && nph >= kEpiMax)) continue;
                    (cz ? ncz : nph)++;
                    op.members.push_back(gi);
                    d.pop(head, gi);
                    took = true;
                }
                if (!took) break;
            }
            std::sort(op.members.begin(), op.members.end());
            remaining -= (int)op.members.size();
        } else {
            op.kind = OP_CLUSTER;
            for (int q = 0; q < n; ++q)
                if (best.Q >> q & 1) op.qubits[op.k++] = q;
            op.members = best.members;
            op.epi = best.epi;
            std::sort(op.members.begin(), op.members.end());
            std::sort(op.epi.begin(), op.epi.end());
            head = best.head;
            remaining -= best.n_gates();
        }
        out.push_back(std::move(op));
    }
    return out;
}

}  // namespace

Schedule make_schedule(int n, const std::vector<SGate>& gates, const SchedOpts& o, const OpCostFn& cost) {
    Schedule S;
    const int ng = (int)gates.size();
    S.dropped.assign(ng, 0);

    // Leading H on every qubit -> uniform initialisation (Sec. 3.6).
    if (o.skip_initial_h && n > 0) {
        std::vector<int> first(n, -1);
        for (int i = 0; i < ng; ++i)
            for (int j = 0; j < gates[i].nq; ++j)
                if (first[gates[i].q[j]] < 0) first[gates[i].q[j]] = i;
        bool ok = true;
        for (int q = 0; q < n && ok; ++q) ok = first[q] >= 0 && gates[first[q]].kind == G_H;
        if (ok) {
            for (int q = 0; q < n; ++q) S.dropped[first[q]] = 1;
            S.uniform_init = true;
        }
    }
    // Trailing diagonal gates change phases only (Sec. 3.6).
    if (o.skip_trailing_diag) {
        std::vector<char> later_dense(n, 0);
        for (int i = ng - 1; i >= 0; --i) {
            if (S.dropped[i]) continue;
            const SGate& g = gates[i];
            if (g.diag) {
                bool any = false;
                for (int j = 0; j < g.nq; ++j) any |= later_dense[g.q[j]] != 0;
                if (!any) S.dropped[i] = 1;
            } else {
                for (int j = 0; j < g.nq; ++j) later_dense[g.q[j]] = 1;
            }
        }
    }
    for (int i = 0; i < ng; ++i) S.n_applied += !S.dropped[i];

    if (o.mode == 0) {
        for (int i = 0; i < ng; ++i) {
            if (S.dropped[i]) continue;
            SOp op;
            op.kind = OP_GATE;
            op.k = gates[i].nq;
            for (int j = 0; j < gates[i].nq; ++j) op.qubits[j] = gates[i].q[j];
            op.members.push_back(i);
            S.ops.push_back(std::move(op));
        }
        return S;
    }

    const int kmax = std::max(1, std::min(o.kmax, kMaxK));
    if (o.mode == 1 || !cost) {
        S.ops = greedy_ops(n, gates, S.dropped, S.n_applied, kmax, o.fuse_diag);
        return S;
    }
    // cost-driven: the complete greedy schedule for every cap, the one with
    // the smallest predicted total time wins (schedules built in parallel)
    std::vector<std::future<std::vector<SOp>>> futs;
    for (int kc = 1; kc <= kmax; ++kc)
        futs.push_back(std::async(std::launch::async, [&, kc]() {
            return greedy_ops(n, gates, S.dropped, S.n_applied, kc, o.fuse_diag);
        }));
    double best_cost = 0.0;
    for (int kc = 1; kc <= kmax; ++kc) {
        std::vector<SOp> ops = futs[kc - 1].get();
        double total = 0.0;
        for (const SOp& op : ops) {
            if (op.kind == OP_DIAG) total += cost(0, op.qubits, 0);
            else total += cost(op.k, op.qubits, (int)op.epi.size());
        }
        if (kc == 1 || total < best_cost) {
            best_cost = total;
            S.ops = std::move(ops);
        }
    }
    return S;
}

}  // namespace qsim
