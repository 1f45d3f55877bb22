// Stage finding for a state split over 2^g memories (Haener & Steiger,
// Sec. 3.6.1 steps 1 and 3, with the global-gate specialisation of Sec. 3.5).
//
// The n qubits sit at bit locations 0..n-1 of the amplitude index; locations
// below l are local (inside one memory), the g = n - l above are global. A gate
// can run without communication when every qubit it must gather is local: all
// of its qubits in general; none for a CZ when CZ is specialised (on global
// qubits it is a conditional phase or a local Z), none for a diagonal
// single-qubit gate when those are specialised too (a phase).
//
// Step 1: a stage is the largest set of remaining gates that can run with the
// current layout - gates on different qubits commute, so it is the closure of
// the ready gates that need no global qubit, and it is unique. After a stage,
// up to g global qubits are swapped with as many local qubits (one
// all-to-all, Sec. 3.4) and the next stage is grown. Which qubits: either
// every global qubit with the local qubits at the lowest locations (the
// paper's upper bound), or a cheap search. Its rule pairs the global qubit
// needed soonest with the local qubit needed furthest ahead, and so on, while
// the global one is needed sooner (the earliest remaining gate then always
// runs: it waits for global qubits only, and every other local qubit is
// needed no sooner). Candidates are that exchange, the full swap with the
// furthest-ahead local qubits, these with one local qubit exchanged for a
// near miss, and the lowest locations; each is played out to the end of the
// circuit by the same rule and the one with the fewest swaps wins. The first
// layout is free (the run starts from a product state) and is searched the
// same way.
//
// Step 2 (Sec. 3.6.1): the gates of each stage are clustered by the clustering
// scheduler; only local qubits count towards a cluster's width (a specialised
// CZ with one global qubit acts as a diagonal gate on its local qubit).
//
// Step 3: the last cluster of a stage tends to hold few gates. If every gate
// in it can also run after the following swap (the qubits it gathers stay
// local), the swap is moved ahead of it; the move is kept when the two stages
// then need fewer clusters. The number of swaps does not change.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "qsim_internal.h"
#include "scheduler.h"

namespace qsim {
namespace {

struct Circ {
    int n = 0, l = 0;
    const std::vector<SGate>* g = nullptr;
    std::vector<char> skip;                 // gates left out of the run
    std::vector<std::vector<int>> queue;    // per qubit: gates in program order (skips excluded)
    std::vector<uint64_t> need;             // per gate: qubits that must be local
    int n_live = 0;
};

uint64_t needs_local(const SGate& s, const StageOpts& o) {
    if (s.kind == G_CZ && o.spec_cz) return 0;
    if (s.nq == 1 && s.diag && o.spec_diag1) return 0;
    uint64_t m = 0;
    for (int j = 0; j < s.nq; ++j) m |= uint64_t(1) << s.q[j];
    return m;
}

// Progress through the circuit: queue heads per qubit.
struct Progress {
    std::vector<int> head;
    int done = 0;
};

// Run the stage closure for the local-qubit mask `local`: take every ready
// gate whose gathered qubits are local, until none is left. Records the
// stage of each gate taken when `stage_of` is given.
int grow_stage(const Circ& c, Progress& p, uint64_t local, std::vector<int>* stage_of, int stage) {
    const auto& G = *c.g;
    std::vector<int> work;
    for (int q = 0; q < c.n; ++q) work.push_back(q);
    int taken = 0;
    while (!work.empty()) {
        const int q = work.back();
        work.pop_back();
        for (;;) {
            const auto& qq = c.queue[q];
            if (p.head[q] >= (int)qq.size()) break;
            const int gi = qq[p.head[q]];
            const SGate& s = G[gi];
            bool ready = true;
            for (int j = 0; j < s.nq && ready; ++j) {
                const auto& qj = c.queue[s.q[j]];
                ready = p.head[s.q[j]] < (int)qj.size() && qj[p.head[s.q[j]]] == gi;
            }
            if (!ready || (c.need[gi] & ~local)) break;
            for (int j = 0; j < s.nq; ++j) {
                p.head[s.q[j]]++;
                if (s.q[j] != q) work.push_back(s.q[j]);
            }
            if (stage_of) (*stage_of)[gi] = stage;
            ++taken;
        }
    }
    p.done += taken;
    return taken;
}

// Program position of the next gate that gathers qubit q (n_gates if none).
int next_gather(const Circ& c, const Progress& p, int q) {
    const auto& qq = c.queue[q];
    for (int j = p.head[q]; j < (int)qq.size(); ++j)
        if (c.need[qq[j]] >> q & 1) return qq[j];
    return (int)c.g->size();
}

// Local qubits ordered by how far ahead their next gather lies (furthest
// first), global qubits by how soon (soonest first); ties: lower location.
std::vector<int> furthest_first(const Circ& c, const Progress& p, const std::vector<int>& loc, bool global = false,
                                std::vector<int>* next = nullptr) {
    std::vector<int> L;
    for (int q = 0; q < c.n; ++q)
        if ((loc[q] >= c.l) == global) L.push_back(q);
    std::vector<int> nx(c.n);
    for (int q : L) nx[q] = next_gather(c, p, q);
    std::stable_sort(L.begin(), L.end(), [&](int a, int b) {
        if (nx[a] != nx[b]) return global ? nx[a] < nx[b] : nx[a] > nx[b];
        return loc[a] < loc[b];
    });
    if (next) *next = nx;
    return L;
}

struct Swap {
    std::vector<int> in, out;  // global qubits made local, local qubits made global
};

// The exchange rule: the global qubit needed soonest against the local qubit
// needed furthest ahead, pair by pair, while the global one is needed sooner.
Swap exchange(const Circ& c, const Progress& p, const std::vector<int>& loc) {
    std::vector<int> ng, nl;
    const std::vector<int> G = furthest_first(c, p, loc, true, &ng);
    const std::vector<int> L = furthest_first(c, p, loc, false, &nl);
    Swap s;
    for (size_t i = 0; i < G.size() && i < L.size(); ++i) {
        if (ng[G[i]] >= nl[L[i]]) break;
        s.in.push_back(G[i]);
        s.out.push_back(L[i]);
    }
    return s;
}

// Every global qubit in, `out` (as many local qubits) out.
Swap full_swap(const Circ& c, const std::vector<int>& loc, const std::vector<int>& out) {
    Swap s;
    for (int q = 0; q < c.n; ++q)
        if (loc[q] >= c.l) s.in.push_back(q);
    s.out.assign(out.begin(), out.begin() + std::min(out.size(), s.in.size()));
    return s;
}

// Apply a swap: pairs in ascending location order on both sides; each
// incoming qubit takes the location of its outgoing partner and vice versa.
void do_swap(std::vector<int>& loc, Swap s) {
    auto by_loc = [&](int a, int b) { return loc[a] < loc[b]; };
    std::sort(s.out.begin(), s.out.end(), by_loc);
    std::sort(s.in.begin(), s.in.end(), by_loc);
    std::vector<int> lo, hi;
    for (int q : s.out) lo.push_back(loc[q]);
    for (int q : s.in) hi.push_back(loc[q]);
    for (size_t i = 0; i < s.in.size(); ++i) {
        loc[s.in[i]] = lo[i];
        loc[s.out[i]] = hi[i];
    }
}

uint64_t local_mask(const Circ& c, const std::vector<int>& loc) {
    uint64_t m = 0;
    for (int q = 0; q < c.n; ++q)
        if (loc[q] < c.l) m |= uint64_t(1) << q;
    return m;
}

std::vector<int> lowest_out(const Circ& c, const std::vector<int>& loc) {
    std::vector<int> out;
    for (int q = 0; q < c.n; ++q)
        if (loc[q] < c.n - c.l) out.push_back(q);
    return out;
}

// Swaps needed from (p, loc) to the end of the circuit under the exchange
// rule. Returns -1 when the circuit cannot finish (a gate gathers more
// qubits than there are local locations).
int play_out(const Circ& c, Progress p, std::vector<int> loc) {
    int swaps = 0;
    grow_stage(c, p, local_mask(c, loc), nullptr, 0);
    while (p.done < c.n_live) {
        do_swap(loc, exchange(c, p, loc));
        ++swaps;
        if (grow_stage(c, p, local_mask(c, loc), nullptr, 0) == 0) return -1;
    }
    return swaps;
}

// Candidate swaps at the end of a stage.
std::vector<Swap> swap_candidates(const Circ& c, const Progress& p, const std::vector<int>& loc) {
    std::vector<Swap> cand;
    const Swap ex = exchange(c, p, loc);
    cand.push_back(ex);
    const std::vector<int> ff = furthest_first(c, p, loc);
    cand.push_back(full_swap(c, loc, ff));
    // one outgoing qubit exchanged for one of the first near misses
    for (const Swap base : {ex, cand[1]}) {
        const int m = (int)base.out.size();
        const int n_in = std::min(m, 4), n_miss = std::min((int)ff.size() - m, 4);
        for (int i = 0; i < n_in; ++i)
            for (int j = 0; j < n_miss; ++j) {
                Swap v = base;
                v.out[m - 1 - i] = ff[m + j];
                cand.push_back(v);
            }
    }
    cand.push_back(full_swap(c, loc, lowest_out(c, loc)));
    return cand;
}

// Gates of one stage as the clustering scheduler sees them: only local qubits
// count; a specialised CZ with one global qubit acts on its local qubit as a
// diagonal gate, one on two global qubits is a global phase.
std::vector<SGate> stage_view(const Circ& c, const std::vector<int>& members, const std::vector<int>& loc) {
    std::vector<SGate> out;
    for (int gi : members) {
        const SGate& s = (*c.g)[gi];
        SGate t = s;
        int nl = 0;
        for (int j = 0; j < s.nq; ++j)
            if (loc[s.q[j]] < c.l) t.q[nl++] = s.q[j];
        if (nl == s.nq) {
            out.push_back(s);
        } else if (nl > 0 && s.diag) {
            t.nq = nl;
            t.kind = G_Z;  // a diagonal gate on the local qubits; its phase does not change the count
            out.push_back(t);
        }
        // no local qubit: a phase on whole memories, no pass over the state
    }
    return out;
}

int count_clusters(const Circ& c, const std::vector<int>& members, const std::vector<int>& loc, int kmax,
                   bool fuse_diag) {
    if (members.empty()) return 0;
    SchedOpts so;
    so.kmax = kmax;
    so.mode = 1;
    so.fuse_diag = fuse_diag;
    so.parallel = false;
    return (int)make_schedule(c.n, stage_view(c, members, loc), so, OpCostFn()).ops.size();
}

// The members of the last cluster of a stage.
std::vector<int> last_cluster(const Circ& c, const std::vector<int>& members, const std::vector<int>& loc, int kmax,
                              bool fuse_diag) {
    SchedOpts so;
    so.kmax = kmax;
    so.mode = 1;
    so.fuse_diag = fuse_diag;
    so.parallel = false;
    const std::vector<SGate> view = stage_view(c, members, loc);
    const Schedule S = make_schedule(c.n, view, so, OpCostFn());
    std::vector<int> out;
    if (S.ops.empty()) return out;
    // map view indices back to gate indices: stage_view keeps members in order, dropping global-only gates
    std::vector<int> back;
    for (int gi : members) {
        const SGate& s = (*c.g)[gi];
        int nl = 0;
        for (int j = 0; j < s.nq; ++j) nl += loc[s.q[j]] < c.l;
        if (nl == s.nq || (nl > 0 && s.diag)) back.push_back(gi);
    }
    const SOp& op = S.ops.back();
    for (int v : op.members) out.push_back(back[v]);
    for (int v : op.epi) out.push_back(back[v]);
    return out;
}

}  // namespace

StagePlan make_stage_plan(int n, const std::vector<SGate>& gates, const StageOpts& o) {
    StagePlan P;
    Circ c;
    c.n = n;
    c.l = o.n_local;
    c.g = &gates;
    bool uniform = false;
    mark_skips(n, gates, o.skip_initial_h, o.skip_trailing_diag, c.skip, uniform);
    c.queue.assign(n, {});
    c.need.assign(gates.size(), 0);
    for (int i = 0; i < (int)gates.size(); ++i) {
        if (c.skip[i]) continue;
        ++c.n_live;
        c.need[i] = needs_local(gates[i], o);
        for (int j = 0; j < gates[i].nq; ++j) c.queue[gates[i].q[j]].push_back(i);
    }
    P.gate_stage.assign(gates.size(), -1);

    // first layout: identity, or searched (it costs nothing: no state yet)
    std::vector<int> loc(n);
    std::iota(loc.begin(), loc.end(), 0);
    Progress p;
    p.head.assign(n, 0);
    if (o.search && c.l < n) {
        std::vector<std::vector<int>> starts{loc};
        // the qubits gathered latest start global
        std::vector<int> nx(n);
        for (int q = 0; q < n; ++q) nx[q] = next_gather(c, p, q);
        std::vector<int> order(n);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nx[a] < nx[b]; });
        std::vector<int> l2(n);
        for (int i = 0; i < n; ++i) l2[order[i]] = i;
        starts.push_back(l2);
        int best = -1;
        for (const auto& s : starts) {
            const int sw = play_out(c, p, s);
            if (sw >= 0 && (best < 0 || sw < best)) {
                best = sw;
                loc = s;
            }
        }
    }

    int stage = 0;
    P.loc.push_back(loc);
    grow_stage(c, p, local_mask(c, loc), &P.gate_stage, stage);
    while (p.done < c.n_live) {
        Swap sw = exchange(c, p, loc);
        if (!o.search) {
            // every global qubit with the lowest local locations, unless that
            // leaves the next gate waiting (then the exchange rule)
            const Swap low = full_swap(c, loc, lowest_out(c, loc));
            std::vector<int> l2 = loc;
            do_swap(l2, low);
            Progress p2 = p;
            if (grow_stage(c, p2, local_mask(c, l2), nullptr, 0) > 0) sw = low;
        } else {
            int best = -1;
            for (const Swap& cand : swap_candidates(c, p, loc)) {
                std::vector<int> l2 = loc;
                do_swap(l2, cand);
                Progress p2 = p;
                if (grow_stage(c, p2, local_mask(c, l2), nullptr, 0) == 0) continue;
                const int rest = play_out(c, p2, l2);
                if (rest >= 0 && (best < 0 || rest < best)) {
                    best = rest;
                    sw = cand;
                }
            }
        }
        do_swap(loc, sw);
        ++stage;
        P.loc.push_back(loc);
        if (grow_stage(c, p, local_mask(c, loc), &P.gate_stage, stage) == 0) {
            P.ok = false;  // a gate gathers more qubits than the local locations hold
            return P;
        }
    }
    const int ns = (int)P.loc.size();
    auto members_of = [&](int s) {
        std::vector<int> m;
        for (int i = 0; i < (int)gates.size(); ++i)
            if (P.gate_stage[i] == s) m.push_back(i);
        return m;
    };
    // step 3: move the swap ahead of a stage's last cluster when its gates can
    // run after the swap and the two stages then need fewer clusters
    if (o.kmax > 0 && o.early_swaps) {
        for (int s = 0; s + 1 < ns; ++s) {
            for (int iter = 0; iter < 8; ++iter) {
                std::vector<int> ms = members_of(s), mt = members_of(s + 1);
                if (ms.empty()) break;
                const std::vector<int> last = last_cluster(c, ms, P.loc[s], o.kmax, o.fuse_diag);
                if (last.empty()) break;
                const uint64_t local_next = local_mask(c, P.loc[s + 1]);
                bool movable = true;
                for (int gi : last) movable &= (c.need[gi] & ~local_next) == 0;
                if (!movable) break;
                const int before = count_clusters(c, ms, P.loc[s], o.kmax, o.fuse_diag) +
                                   count_clusters(c, mt, P.loc[s + 1], o.kmax, o.fuse_diag);
                std::vector<int> ms2, mt2;
                std::vector<char> moved(gates.size(), 0);
                for (int gi : last) moved[gi] = 1;
                for (int gi : ms)
                    if (!moved[gi]) ms2.push_back(gi);
                mt2 = mt;
                mt2.insert(mt2.end(), last.begin(), last.end());
                std::sort(mt2.begin(), mt2.end());  // program order (the moved gates precede the stage's own)
                const int after = count_clusters(c, ms2, P.loc[s], o.kmax, o.fuse_diag) +
                                  count_clusters(c, mt2, P.loc[s + 1], o.kmax, o.fuse_diag);
                if (after >= before) break;
                for (int gi : last) P.gate_stage[gi] = s + 1;
                ++P.n_moved;
            }
        }
    }
    if (o.kmax > 0)
        for (int s = 0; s < ns; ++s) P.n_clusters.push_back(count_clusters(c, members_of(s), P.loc[s], o.kmax,
                                                                           o.fuse_diag));
    return P;
}

}  // namespace qsim
