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
// Cost-driven mode (analytic or learned cost model): complete candidate
// schedules - greedy with caps kmax - 2 .. kmax, and greedy with kmax where a
// full-width cluster may give way to the (kmax - 1)-qubit cluster of the same
// seed when that is predicted cheaper per gate - are built, and the one with
// the smallest predicted total time is kept. (Per-cluster choices alone are
// myopic: a cluster can look cheap per gate and still leave more total work;
// the final comparison is between whole schedules.)
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

// Take gate gi: advance the heads of its qubits and update the ready list
// (ascending gate index): gi leaves it, and only the new heads of gi's qubits
// can become ready.
void take(const Dag& d, std::vector<int>& head, std::vector<int>& rl, int gi) {
    d.pop(head, gi);
    rl.erase(std::lower_bound(rl.begin(), rl.end(), gi));
    const SGate& s = (*d.g)[gi];
    for (int j = 0; j < s.nq; ++j) {
        const auto& qq = d.queue[s.q[j]];
        const int h = head[s.q[j]];
        if (h >= (int)qq.size()) continue;
        const int g2 = qq[h];
        if (!d.ready(head, g2)) continue;
        auto it = std::lower_bound(rl.begin(), rl.end(), g2);
        if (it == rl.end() || *it != g2) rl.insert(it, g2);
    }
}

// Grow a cluster from `seed` with at most `kcap` qubits; rl0 is the ready
// list at head0.
Grown grow(const Dag& d, const std::vector<int>& head0, const std::vector<int>& rl0, int seed, int kcap,
           bool fuse_diag) {
    const auto& G = *d.g;
    Grown r;
    r.head = head0;
    std::vector<int> rl = rl0;
    r.Q = d.mask[seed];
    r.members.push_back(seed);
    take(d, r.head, rl, seed);
    uint64_t sealed = 0;
    int n_epi_cz = 0, n_epi_ph = 0;
    for (;;) {
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
            take(d, r.head, rl, best);
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
        take(d, r.head, rl, best);
    }
    return r;
}

bool all_diag(const std::vector<SGate>& G, const Grown& c) {
    for (int i : c.members) if (!G[i].diag) return false;
    return true;
}

// Predicted time of a grown cluster (sorted qubits from its mask).
double grown_cost(const OpCostFn& cost, const Grown& c, int n) {
    int q[64], k = 0;
    for (int b = 0; b < n; ++b)
        if (c.Q >> b & 1) q[k++] = b;
    return cost(k, q, (int)c.epi.size());
}

// Greedy clustering with at most kcap qubits per cluster (gates with more
// qubits form a cluster of their own width). With a cost function (`trim`),
// a cluster that reached kcap qubits is compared with the cluster the same
// seed grows under kcap - 1, and the one with the smaller predicted time per
// gate is taken.
std::vector<SOp> greedy_ops(int n, const std::vector<SGate>& gates, const std::vector<char>& dropped, int n_applied,
                            int kcap_in, bool fuse_diag, const OpCostFn* trim = nullptr) {
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
        int best_score = -1, best_seed = -1;
        for (int seed : rl) {
            // a gate wider than kmax (a dense gate) forms a cluster of its own width
            const int khi = std::max(kmax, popc(d.mask[seed]));
            Grown c = grow(d, head, rl, seed, khi, fuse_diag);
            if (c.n_gates() > best_score) { best_score = c.n_gates(); best = std::move(c); best_seed = seed; }
        }
        if (trim && kmax > 1 && popc(best.Q) == kmax && popc(d.mask[best_seed]) < kmax) {
            Grown small = grow(d, head, rl, best_seed, kmax - 1, fuse_diag);
            if (!all_diag(gates, small) && !all_diag(gates, best)) {
                const double per_big = grown_cost(*trim, best, n) / best.n_gates();
                const double per_small = grown_cost(*trim, small, n) / small.n_gates();
                if (per_small < per_big) best = std::move(small);
            }
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
    // cost-driven: complete candidate schedules, the one with the smallest
    // predicted total time wins (built in parallel). Candidates: the greedy
    // schedule for each cap kmax - 2 .. kmax (smaller caps only add passes)
    // and the cost-trimmed greedy schedule for kmax.
    const int k_lo = std::max(1, kmax - 2);
    std::vector<std::future<std::vector<SOp>>> futs;
    for (int kc = k_lo; kc <= kmax; ++kc)
        futs.push_back(std::async(std::launch::async, [&, kc]() {
            return greedy_ops(n, gates, S.dropped, S.n_applied, kc, o.fuse_diag);
        }));
    if (kmax > 1)
        futs.push_back(std::async(std::launch::async, [&]() {
            return greedy_ops(n, gates, S.dropped, S.n_applied, kmax, o.fuse_diag, &cost);
        }));
    double best_cost = 0.0;
    for (size_t c = 0; c < futs.size(); ++c) {
        std::vector<SOp> ops = futs[c].get();
        double total = 0.0;
        for (const SOp& op : ops) {
            if (op.kind == OP_DIAG) total += cost(0, op.qubits, 0);
            else total += cost(op.k, op.qubits, (int)op.epi.size());
        }
        if (c == 0 || total < best_cost) {
            best_cost = total;
            S.ops = std::move(ops);
        }
    }
    return S;
}

}  // namespace qsim
