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
// schedules - greedy with caps kmax - 2 .. kmax (with and without the
// candidate qubit sets below), and greedy with kmax where a full-width
// cluster may give way to the (kmax - 1)-qubit cluster of the same seed when
// that is predicted cheaper per gate - are built, and the one with the
// smallest predicted total time is kept. Narrower caps are skipped when the
// model predicts their clusters not cheap enough to pay for their extra passes. (Per-cluster choices alone are
// myopic: a cluster can look cheap per gate and still leave more total work;
// the final comparison is between whole schedules.)
//
// Runs from the uniform state write their start in one write-only pass with
// the first cluster, or with the first two when the second has 6 qubits
// (SchedOpts::fold_start); candidates are compared with that pass priced as
// write-only (kFold1Share, kFold2Share of a pass), and with clusters wider
// than 6 also in a form whose first two clusters have at most 6 qubits.
//
// Candidate clusters besides the seeded ones: the closure of a dense qubit
// set of the interaction graph (every ready gate inside the set joins, until
// none is left). Growing gate by gate from a seed tends to give chains of
// qubits; a compact set (a 2 x 3 block of a grid) holds more gates per pass.
// Greedy mode builds the schedule with and without these candidates and keeps
// the one with fewer ops; cost-driven mode adds them to its candidates.
//
// Extensions for the GPU kernels (both exact, as diagonal gates commute):
//   * a cluster made only of diagonal gates becomes a diagonal pass, which
//     then absorbs every ready diagonal gate;
//   * with fuse_diag, once no gate fits a cluster any more, ready diagonal
//     gates are attached to it and applied while its results are stored; a
//     qubit touched by such a gate accepts only diagonal gates afterwards;
//     when the schedule is complete, such a gate moves into the matrix of the
//     next cluster on its qubits where that cluster holds them all.
#include "scheduler.h"

#include <pthread.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <exception>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>

#include "qsim_internal.h"

namespace qsim {
static_assert(kSchedMaxK == kMaxK, "schedule ops hold the widest cluster");
namespace {

inline int popc(uint64_t x) { return __builtin_popcountll(x); }

// Candidate schedules are built on a process-wide pool of worker threads,
// started on first use: starting a thread per candidate cost as much host
// time as building the candidates. A call hands over a batch of tasks and
// works on it too; a task's exception is rethrown in the caller. Batches are
// shared: a worker that comes late to a finished batch only reads its task
// counter, never the caller's data. After fork() the child starts a pool of
// its own.
class TaskPool {
  public:
    static TaskPool& get() {
        static std::once_flag once;
        std::call_once(once, [] { pthread_atfork(nullptr, nullptr, [] { instance() = nullptr; }); });
        std::lock_guard<std::mutex> l(create_mutex());
        if (!instance()) {
            const int hw = (int)std::thread::hardware_concurrency();
            instance() = new TaskPool(std::max(1, std::min(15, hw - 1)));  // kept until the process ends
        }
        return *instance();
    }
    void run(std::vector<std::function<void()>> fs) {
        if (fs.empty()) return;
        auto b = std::make_shared<Batch>();
        b->n = (int)fs.size();
        b->fs = std::move(fs);
        {
            std::lock_guard<std::mutex> l(m_);
            q_.push_back(b);
        }
        cv_.notify_all();
        work(*b);
        std::unique_lock<std::mutex> l(b->m);
        b->cv.wait(l, [&] { return b->done == b->n; });
        if (b->error) std::rethrow_exception(b->error);
    }

  private:
    struct Batch {
        std::vector<std::function<void()>> fs;
        int n = 0;
        std::atomic<int> next{0};
        std::mutex m;
        std::condition_variable cv;
        int done = 0;  // under m
        std::exception_ptr error;
    };
    static TaskPool*& instance() {
        static TaskPool* p = nullptr;
        return p;
    }
    static std::mutex& create_mutex() {
        static std::mutex m;
        return m;
    }
    static void work(Batch& b) {
        for (;;) {
            const int i = b.next.fetch_add(1);
            if (i >= b.n) return;
            std::exception_ptr e;
            try {
                b.fs[i]();
            } catch (...) {
                e = std::current_exception();
            }
            std::lock_guard<std::mutex> l(b.m);
            if (e && !b.error) b.error = e;
            if (++b.done == b.n) b.cv.notify_all();
        }
    }
    explicit TaskPool(int workers) {
        for (int i = 0; i < workers; ++i) std::thread([this] { loop(); }).detach();
    }
    void loop() {
        for (;;) {
            std::shared_ptr<Batch> b;
            {
                std::unique_lock<std::mutex> l(m_);
                cv_.wait(l, [&] { return !q_.empty(); });
                b = q_.front();
                if (b->next.load() >= b->n) {  // every task taken: the batch leaves the queue
                    q_.pop_front();
                    continue;
                }
            }
            work(*b);
        }
    }
    std::mutex m_;
    std::condition_variable cv_;
    std::deque<std::shared_ptr<Batch>> q_;
};

// Results of the tasks, in order: on the pool when parallel, else one after
// another on this thread. Only tasks with want[i] (all when want is null) run.
// On the pool they start by descending first_key[i] (longest expected first,
// so that the short ones fill the workers that finish early).
template <typename T>
std::vector<T> run_tasks(bool parallel, const std::vector<std::function<T()>>& fns,
                         const std::vector<char>* want = nullptr, const std::vector<int>* first_key = nullptr) {
    std::vector<T> out(fns.size());
    if (!parallel) {
        for (size_t i = 0; i < fns.size(); ++i)
            if (!want || (*want)[i]) out[i] = fns[i]();
        return out;
    }
    std::vector<int> order(fns.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    if (first_key)
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return (*first_key)[a] > (*first_key)[b]; });
    std::vector<std::function<void()>> jobs;
    for (int i : order)
        if (!want || (*want)[i]) jobs.push_back([&fns, &out, i] { out[i] = fns[i](); });
    TaskPool::get().run(std::move(jobs));
    return out;
}

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

// Queue heads and ready list (ascending gate index) of one growth, on fixed
// arrays: a state has at most 64 qubits, so at most 64 gates are ready, and
// the many trial growths of a step need no heap memory.
struct Frontier {
    int head[64];
    int rl[64];
    int nrl = 0;
};

bool ready_at(const Dag& d, const int* head, int gi) {
    const SGate& s = (*d.g)[gi];
    for (int j = 0; j < s.nq; ++j) {
        const auto& qq = d.queue[s.q[j]];
        const int h = head[s.q[j]];
        if (h >= (int)qq.size() || qq[h] != gi) return false;
    }
    return true;
}

// Take gate gi: advance the heads of its qubits and update the ready list:
// gi leaves it, and only the new heads of gi's qubits can become ready.
void take(const Dag& d, Frontier& f, int gi) {
    const SGate& s = (*d.g)[gi];
    for (int j = 0; j < s.nq; ++j) f.head[s.q[j]]++;
    int* end = f.rl + f.nrl;
    int* p = std::lower_bound(f.rl, end, gi);
    std::memmove(p, p + 1, (end - p - 1) * sizeof(int));
    --f.nrl;
    for (int j = 0; j < s.nq; ++j) {
        const auto& qq = d.queue[s.q[j]];
        const int h = f.head[s.q[j]];
        if (h >= (int)qq.size()) continue;
        const int g2 = qq[h];
        if (!ready_at(d, f.head, g2)) continue;
        end = f.rl + f.nrl;
        p = std::lower_bound(f.rl, end, g2);
        if (p != end && *p == g2) continue;
        std::memmove(p + 1, p, (end - p) * sizeof(int));
        *p = g2;
        ++f.nrl;
    }
}

// Grow a cluster from `seed` with at most `kcap` qubits, starting at f0. With
// `within` != 0 there is no seed (seed = -1) and the cluster is the closure
// of that qubit set: every gate that becomes ready and lies inside it joins
// the matrix. Returns the number of gates taken (matrix and diagonal
// epilogue); `out`, when given, receives the cluster.
int grow(const Dag& d, const Frontier& f0, int seed, int kcap, bool fuse_diag, uint64_t within, Grown* out) {
    const auto& G = *d.g;
    Frontier f = f0;
    uint64_t Q = 0;
    int n_mat = 0, n_epi_cz = 0, n_epi_ph = 0;
    if (seed >= 0) {
        Q = d.mask[seed];
        ++n_mat;
        if (out) out->members.push_back(seed);
        take(d, f, seed);
    }
    for (;;) {
        // a gate that joins the matrix: fewest new qubits, then lowest index
        int best = -1, best_new = 1 << 30;
        for (int i = 0; i < f.nrl; ++i) {
            const int gi = f.rl[i];
            const uint64_t m = d.mask[gi];
            if (within ? (m & ~within) != 0 : popc(Q | m) > kcap) continue;
            const int nw = popc(m & ~Q);
            if (nw < best_new) {
                best = gi;
                best_new = nw;
                if (nw == 0) break;  // nothing beats it, and later gates have higher indices
            }
        }
        if (best < 0) break;
        ++n_mat;
        if (out) out->members.push_back(best);
        Q |= d.mask[best];
        take(d, f, best);
    }
    // nothing fits: attach ready diagonal gates, lowest index first. Their
    // qubits are sealed, and every gate they make ready touches one, so no
    // further matrix gate can join; a gate made ready has a higher index than
    // the one taken, so one forward pass over the ready list finds them all.
    if (fuse_diag && n_mat > 0) {
        for (int i = 0; i < f.nrl;) {
            const int gi = f.rl[i];
            const bool cz = G[gi].kind == G_CZ;
            if (!G[gi].diag || (cz && n_epi_cz >= kEpiMax) || (!cz && n_epi_ph >= kEpiMax)) {
                ++i;
                continue;
            }
            if (out) out->epi.push_back(gi);
            if (cz) ++n_epi_cz; else ++n_epi_ph;
            take(d, f, gi);  // removes rl[i]; gates it makes ready sort after it
        }
    }
    if (out) {
        out->Q = Q;
        out->head.assign(f.head, f.head + d.n);
    }
    return n_mat + n_epi_cz + n_epi_ph;
}

// Gates the closure of qubit set S takes into its matrix from `head`: every
// gate inside S that reaches the head of all its qubits. Only the queues of
// S's qubits matter (the diagonal gates a cluster carries afterwards never add
// matrix gates), so this count ranks the candidate sets cheaply.
int closure_size(const Dag& d, const std::vector<int>& head, uint64_t S) {
    const auto& G = *d.g;
    int h[64];
    for (uint64_t m = S; m; m &= m - 1) h[__builtin_ctzll(m)] = head[__builtin_ctzll(m)];
    // taking a gate never makes another one unready, so the closure is the
    // same in any order: a worklist of qubits whose queue head moved
    int cnt = 0;
    for (uint64_t pending = S; pending;) {
        const int q = __builtin_ctzll(pending);
        pending &= pending - 1;
        const auto& qq = d.queue[q];
        while (h[q] < (int)qq.size()) {
            const int gi = qq[h[q]];
            const uint64_t gm = d.mask[gi];
            if (gm & ~S) break;
            bool at_head = true;
            for (int j = 0; j < G[gi].nq && at_head; ++j) {
                const int p = G[gi].q[j];
                at_head = h[p] < (int)d.queue[p].size() && d.queue[p][h[p]] == gi;
            }
            if (!at_head) break;
            for (int j = 0; j < G[gi].nq; ++j) h[G[gi].q[j]]++;
            ++cnt;
            pending |= gm & ~(uint64_t(1) << q);
        }
    }
    return cnt;
}

bool all_diag(const std::vector<SGate>& G, const Grown& c) {
    for (int i : c.members) if (!G[i].diag) return false;
    return true;
}

// Diagonal gates a cluster carries to its store (fuse_diag) move into the
// matrix of the next cluster that holds all their qubits, when that is the
// first later op with a non-diagonal gate on any of them: in between they
// meet only gates on other qubits and diagonal gates, which commute with them
// (Sec. 3.5). In a matrix they cost nothing; at a store, a phase or a sign
// that depends on a target bit is arithmetic on every amplitude.
void absorb_epilogues(std::vector<SOp>& ops, const std::vector<SGate>& gates) {
    const size_t no = ops.size();
    auto mask_of = [&](int gi) {
        uint64_t m = 0;
        for (int j = 0; j < gates[gi].nq; ++j) m |= uint64_t(1) << gates[gi].q[j];
        return m;
    };
    std::vector<uint64_t> nondiag(no, 0), held(no, 0);
    for (size_t o = 0; o < no; ++o) {
        for (int gi : ops[o].members)
            if (!gates[gi].diag) nondiag[o] |= mask_of(gi);
        if (ops[o].kind == OP_CLUSTER)
            for (int j = 0; j < ops[o].k; ++j) held[o] |= uint64_t(1) << ops[o].qubits[j];
    }
    for (size_t i = 0; i < no; ++i) {
        if (ops[i].kind != OP_CLUSTER || ops[i].epi.empty()) continue;
        std::vector<int> keep;
        for (int gi : ops[i].epi) {
            const uint64_t Q = mask_of(gi);
            size_t t = i + 1;
            while (t < no && !(nondiag[t] & Q)) ++t;
            if (t < no && ops[t].kind == OP_CLUSTER && (Q & ~held[t]) == 0) {
                auto& m = ops[t].members;
                m.insert(std::lower_bound(m.begin(), m.end(), gi), gi);  // program order in the matrix
            } else {
                keep.push_back(gi);
            }
        }
        ops[i].epi = std::move(keep);
    }
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
// first_cap > 0: the first two clusters have at most first_cap qubits (so
// that a folded start can take them both).
// dev_step >= 0: at that step (op index) the cluster taken is the dev_rank-th
// best of the distinct candidates (by gates taken, ties in the order the
// greedy choice breaks them; rank 0 is the greedy choice) instead of the
// best; an empty schedule when there are not that many.
std::vector<SOp> greedy_ops(int n, const std::vector<SGate>& gates, const std::vector<char>& dropped, int n_applied,
                            int kcap_in, bool fuse_diag, const OpCostFn* trim = nullptr,
                            const std::vector<uint64_t>* sets = nullptr, int first_cap = 0, int dev_step = -1,
                            int dev_rank = 0) {
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
    // closure sizes of the candidate sets, recomputed only for sets with a
    // qubit whose queue head moved since (the size depends on those heads only)
    std::vector<int> csize(sets ? sets->size() : 0, 0);
    uint64_t moved = ~uint64_t(0);
    std::vector<int> head_before;
    int n_clusters = 0;

    while (remaining > 0) {
        d.ready_list(head, rl);
        Frontier f0;
        for (int q = 0; q < n; ++q) f0.head[q] = head[q];
        f0.nrl = (int)rl.size();
        std::copy(rl.begin(), rl.end(), f0.rl);
        const int kcur = (first_cap > 0 && n_clusters < 2) ? std::min(kmax, first_cap) : kmax;
        int best_score = -1, best_seed = -1, best_cap = kcur;
        uint64_t best_within = 0;
        // the deviating step lists every candidate: (score, seed, cap, within, qubits)
        const bool dev = (int)out.size() == dev_step;
        struct DevCand {
            int score, seed, cap;
            uint64_t within, Q;
        };
        std::vector<DevCand> devc;
        for (int seed : rl) {
            // a gate wider than the cap (a dense gate) forms a cluster of its own width
            const int khi = std::max(kcur, popc(d.mask[seed]));
            Grown g;
            const int c = grow(d, f0, seed, khi, fuse_diag, 0, dev ? &g : nullptr);
            if (dev) devc.push_back({c, seed, khi, 0, g.Q});
            if (c > best_score) {
                best_score = c;
                best_seed = seed;
                best_cap = khi;
            }
        }
        // closures of the candidate qubit sets compete with the seeded
        // clusters: ranked by their matrix gates, the top kTopSets are grown
        // in full (with the diagonal gates they carry)
        if (sets) {
            constexpr size_t kTopSets = 8;
            std::vector<std::pair<int, uint64_t>> ranked;
            ranked.reserve(sets->size());
            for (size_t i = 0; i < sets->size(); ++i) {
                const uint64_t S = (*sets)[i];
                if (S & moved) csize[i] = closure_size(d, head, S);
                if (csize[i] > 0) ranked.emplace_back(-csize[i], S);
            }
            const size_t top = std::min(kTopSets, ranked.size());
            std::partial_sort(ranked.begin(), ranked.begin() + top, ranked.end());
            for (size_t i = 0; i < top; ++i) {
                if (popc(ranked[i].second) > kcur) continue;
                Grown g;
                const int c = grow(d, f0, -1, kcur, fuse_diag, ranked[i].second, dev ? &g : nullptr);
                if (dev && c > 0) devc.push_back({c, -1, kcur, ranked[i].second, g.Q});
                if (c > best_score) {  // c > 0: the closure took a matrix gate
                    best_score = c;
                    best_seed = -1;
                    best_cap = kcur;
                    best_within = ranked[i].second;
                }
            }
        }
        if (dev) {
            std::stable_sort(devc.begin(), devc.end(),
                             [](const DevCand& a, const DevCand& b) { return a.score > b.score; });
            std::vector<DevCand> uniq;
            for (const DevCand& c : devc) {
                bool dup = false;
                for (const DevCand& u : uniq) dup |= u.Q == c.Q && u.score == c.score;
                if (!dup) uniq.push_back(c);
            }
            if (dev_rank >= (int)uniq.size()) return {};
            const DevCand& ch = uniq[dev_rank];
            best_score = ch.score;
            best_seed = ch.seed;
            best_cap = ch.cap;
            best_within = ch.within;
        }
        Grown best;
        grow(d, f0, best_seed, best_cap, fuse_diag, best_within, &best);
        if (trim && best_seed >= 0 && kcur > 1 && popc(best.Q) == kcur && popc(d.mask[best_seed]) < kcur) {
            Grown small;
            grow(d, f0, best_seed, kcur - 1, fuse_diag, 0, &small);
            if (!all_diag(gates, small) && !all_diag(gates, best)) {
                const double per_big = grown_cost(*trim, best, n) / best.n_gates();
                const double per_small = grown_cost(*trim, small, n) / small.n_gates();
                if (per_small < per_big) best = std::move(small);
            }
        }
        head_before = head;
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
            ++n_clusters;
        }
        out.push_back(std::move(op));
        moved = 0;
        for (int q = 0; q < n; ++q)
            if (head[q] != head_before[q]) moved |= uint64_t(1) << q;
    }
    if (fuse_diag) absorb_epilogues(out, gates);
    return out;
}

// Candidate qubit sets for clusters: dense connected k-qubit sets of the
// interaction graph (two qubits are joined when a gate acts on both). From
// every edge, a set grows by the outside neighbour with the most edges into
// it; all neighbours that tie are followed. Sets whose internal edge count is
// within `slack` (0 and 1) of the largest are kept. On a grid circuit, k = 6 and slack
// 0 give the 2 x 3 and 3 x 2 blocks: a cluster there takes more gates per
// qubit than one grown gate by gate. Each level is capped at kSetCap sets.
void dense_sets(int n, const std::vector<SGate>& gates, const std::vector<char>& dropped, int k,
                std::vector<uint64_t>& slack0, std::vector<uint64_t>& slack1) {
    constexpr size_t kSetCap = 4096;
    slack0.clear();
    slack1.clear();
    std::vector<uint64_t> level;
    if (k < 2 || n > 64) return;
    std::vector<uint64_t> adj(n, 0);
    for (size_t i = 0; i < gates.size(); ++i) {
        if (dropped[i]) continue;
        for (int a = 0; a < gates[i].nq; ++a)
            for (int b = 0; b < gates[i].nq; ++b)
                if (a != b) adj[gates[i].q[a]] |= uint64_t(1) << gates[i].q[b];
    }
    for (int a = 0; a < n; ++a)
        for (int b = a + 1; b < n; ++b)
            if (adj[a] >> b & 1) level.push_back((uint64_t(1) << a) | (uint64_t(1) << b));
    for (int size = 2; size < k && !level.empty(); ++size) {
        std::vector<uint64_t> next;
        for (uint64_t S : level) {
            uint64_t nb = 0;
            for (uint64_t m = S; m; m &= m - 1) nb |= adj[__builtin_ctzll(m)];
            nb &= ~S;
            int top = -1;
            for (uint64_t m = nb; m; m &= m - 1) top = std::max(top, popc(adj[__builtin_ctzll(m)] & S));
            for (uint64_t m = nb; m; m &= m - 1) {
                const int q = __builtin_ctzll(m);
                if (popc(adj[q] & S) == top) next.push_back(S | (uint64_t(1) << q));
            }
        }
        std::sort(next.begin(), next.end());
        next.erase(std::unique(next.begin(), next.end()), next.end());
        if (next.size() > kSetCap) next.resize(kSetCap);
        level = std::move(next);
    }
    auto edges = [&](uint64_t S) {
        int e = 0;
        for (uint64_t m = S; m; m &= m - 1) e += popc(adj[__builtin_ctzll(m)] & S);
        return e / 2;
    };
    int top = 0;
    for (uint64_t S : level)
        if (popc(S) == k) top = std::max(top, edges(S));
    for (uint64_t S : level) {
        if (popc(S) != k) continue;
        const int e = edges(S);
        if (e >= top) slack0.push_back(S);
        if (e >= top - 1) slack1.push_back(S);
    }
}

// The start a schedule gets from a folded initialisation (SchedOpts::
// fold_start): 2 when its first two ops are clusters of <= 6 and 6 qubits
// (one write-only pass for both, the second multiplied on the matrix cores),
// 3 when that start takes the table form, 4 when the second cluster has 7
// qubits (the first <= 7) and the table form applies (it is the only form for
// a 7-qubit second cluster), 1 when its first op is a cluster, else 0.
int fold_kind(const std::vector<SOp>& ops, const std::vector<SGate>& gates, int fold) {
    if (fold <= 0 || ops.empty() || ops[0].kind != OP_CLUSTER) return 0;
    if (fold >= 2 && ops.size() >= 2 && ops[1].kind == OP_CLUSTER &&
        ((ops[0].k <= 6 && ops[1].k == 6) || ops[1].k == 7)) {
        if (fold < 3 && ops[1].k == 6) return 2;
        // the table form: rows of the second cluster shared with the first,
        // and rows the first one's diagonal gates couple to a column qubit
        uint64_t t1 = 0, t2 = 0, flipped = 0;
        for (int j = 0; j < ops[0].k; ++j) t1 |= uint64_t(1) << ops[0].qubits[j];
        for (int j = 0; j < ops[1].k; ++j) t2 |= uint64_t(1) << ops[1].qubits[j];
        for (int gi : ops[0].epi) {
            const SGate& g = gates[gi];
            if (g.nq != 2) continue;
            const uint64_t a = uint64_t(1) << g.q[0], b = uint64_t(1) << g.q[1];
            if (((t2 & a) != 0) != ((t2 & b) != 0)) flipped |= t2 & (a | b);
        }
        const int shared = popc(t1 & t2), bits = shared + popc(flipped);
        if (ops[1].k == 6) return shared <= 2 && bits <= kFoldTableBits6 ? 3 : 2;
        if (fold >= 3 && shared <= 2 && bits <= kFoldTableBits7) return 4;
    }
    return 1;
}

// Passes of a schedule with its start counted as the write-only pass it becomes.
double effective_passes(const std::vector<SOp>& ops, const std::vector<SGate>& gates, int fold) {
    switch (fold_kind(ops, gates, fold)) {
        case 4: return (double)ops.size() - 2 + kFold7TableShare;
        case 3: return (double)ops.size() - 2 + kFold2TableShare;
        case 2: return (double)ops.size() - 2 + kFold2Share;
        case 1: return (double)ops.size() - 1 + kFold1Share;
        default: return (double)ops.size();
    }
}

}  // namespace

void mark_skips(int n, const std::vector<SGate>& gates, bool skip_initial_h, bool skip_trailing_diag,
                std::vector<char>& dropped, bool& uniform_init) {
    const int ng = (int)gates.size();
    dropped.assign(ng, 0);
    uniform_init = false;
    // Leading H on every qubit -> uniform initialisation (Sec. 3.6).
    if (skip_initial_h && n > 0) {
        std::vector<int> first(n, -1);
        for (int i = 0; i < ng; ++i)
            for (int j = 0; j < gates[i].nq; ++j)
                if (first[gates[i].q[j]] < 0) first[gates[i].q[j]] = i;
        bool ok = true;
        for (int q = 0; q < n && ok; ++q) ok = first[q] >= 0 && gates[first[q]].kind == G_H;
        if (ok) {
            for (int q = 0; q < n; ++q) dropped[first[q]] = 1;
            uniform_init = true;
        }
    }
    // Trailing diagonal gates change phases only (Sec. 3.6).
    if (skip_trailing_diag) {
        std::vector<char> later_dense(n, 0);
        for (int i = ng - 1; i >= 0; --i) {
            if (dropped[i]) continue;
            const SGate& g = gates[i];
            if (g.diag) {
                bool any = false;
                for (int j = 0; j < g.nq; ++j) any |= later_dense[g.q[j]] != 0;
                if (!any) dropped[i] = 1;
            } else {
                for (int j = 0; j < g.nq; ++j) later_dense[g.q[j]] = 1;
            }
        }
    }
}

int schedule_fold_kind(const std::vector<SOp>& ops, const std::vector<SGate>& gates, int fold_start) {
    return fold_kind(ops, gates, fold_start);
}

Schedule make_schedule(int n, const std::vector<SGate>& gates, const SchedOpts& o, const OpCostFn& cost) {
    Schedule S;
    const int ng = (int)gates.size();
    mark_skips(n, gates, o.skip_initial_h, o.skip_trailing_diag, S.dropped, S.uniform_init);
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
    // candidate qubit sets (dense sets of the interaction graph, two slacks)
    std::vector<uint64_t> sets0, sets1;
    if (o.cluster_sets && kmax >= 2) dense_sets(n, gates, S.dropped, kmax, sets0, sets1);
    // with a two-cluster folded start and clusters wider than 6, candidates
    // whose first two clusters have at most 6 qubits are built as well
    const int fold = S.uniform_init ? o.fold_start : 0;
    const int first_caps = (fold >= 2 && kmax > 6) ? 2 : 1;
    // the one-deviation schedules of the widest cap, with the larger family of
    // sets (slack 1: it holds the slack-0 sets)
    const std::vector<uint64_t>* dev_sets = sets1.empty() ? &sets0 : &sets1;
    const bool deviations =
        o.deviations && o.parallel && o.cluster_sets && n >= kDevMinQubits && kmax >= 2 && !dev_sets->empty();
    if (o.mode == 1 || !cost) {
        // the greedy schedules with and without the candidate sets (and with
        // a 6-qubit start); the one with the fewest passes wins, the start
        // counted as the write-only pass it becomes (ties: the earlier)
        std::vector<std::function<std::vector<SOp>()>> fns;
        for (int fc = 0; fc < first_caps; ++fc) {
            const int cap = fc ? 6 : 0;
            fns.push_back([&, cap]() {
                return greedy_ops(n, gates, S.dropped, S.n_applied, kmax, o.fuse_diag, nullptr, nullptr, cap);
            });
            if (sets0.empty()) continue;
            fns.push_back([&, cap]() {
                return greedy_ops(n, gates, S.dropped, S.n_applied, kmax, o.fuse_diag, nullptr, &sets0, cap);
            });
            fns.push_back([&, cap]() {
                return greedy_ops(n, gates, S.dropped, S.n_applied, kmax, o.fuse_diag, nullptr, &sets1, cap);
            });
        }
        const size_t ndev0 = fns.size();
        if (deviations)
            for (int st = 0; st < kDevSteps; ++st)
                for (int r = 1; r <= kDevRanks; ++r)
                    fns.push_back([&, st, r]() {
                        return greedy_ops(n, gates, S.dropped, S.n_applied, kmax, o.fuse_diag, nullptr, dev_sets, 0,
                                          st, r);
                    });
        std::vector<int> key(fns.size(), 0);  // start the deviations and the set-based schedules first
        for (size_t i = 0; i < fns.size(); ++i) key[i] = i >= ndev0 ? 2 : (i % 3 ? 1 : 0);
        std::vector<std::vector<SOp>> res = run_tasks(o.parallel, fns, nullptr, &key);
        double best = 0.0;
        for (size_t c = 0; c < res.size(); ++c) {
            std::vector<SOp>& ops = res[c];
            if (c >= ndev0 && ops.empty()) continue;  // no candidate of that rank
            const double p = effective_passes(ops, gates, fold);
            if (c == 0 || p < best) {
                best = p;
                S.ops = std::move(ops);
            }
        }
        return S;
    }
    // cost-driven: complete candidate schedules, the one with the smallest
    // predicted total time wins (built in parallel). Candidates: for each cap
    // kmax - 2 .. kmax (smaller caps only add passes) the greedy schedule and
    // the greedy schedules with each family of candidate qubit sets of that
    // size - so the schedule the plain greedy scheduler would pick at any of
    // these caps is always among them - and the cost-trimmed greedy schedule
    // for kmax.
    const int k_lo = std::max(1, kmax - 2);
    using Cand = std::pair<std::vector<SOp>, double>;
    // The one-deviation search only widens the choice of full-width
    // schedules: it runs where a full-width cluster is predicted to cost no
    // more per qubit than one of one qubit fewer (each cost averaged over low,
    // middle, high and spread target sets). On complex128 the 6-qubit
    // clusters are bound by the fp64 matrix cores and it would only cost host
    // time.
    auto typical = [&](int k) {
        int sets[4][kMaxK];
        for (int j = 0; j < k; ++j) {
            sets[0][j] = j;
            sets[1][j] = n / 2 - k / 2 + j;
            sets[2][j] = n - k + j;
            sets[3][j] = k > 1 ? (int)((long)j * (n - 1) / (k - 1)) : 0;
        }
        double c = 0.0;
        for (auto& q : sets) c += cost(k, q, 0);
        return c / 4;
    };
    const double full_per_qubit = typical(kmax) / kmax;
    const bool cd_deviations = deviations && (kmax < 2 || full_per_qubit <= typical(kmax - 1) / (kmax - 1));
    // narrower caps expected to pay (a cheaper cluster per qubit): their
    // gated candidates start with the others instead of in a second round
    bool narrow_likely = false;
    for (int kc = k_lo; kc < kmax; ++kc) narrow_likely |= typical(kc) / kc < full_per_qubit;
    auto priced = [&](std::vector<SOp> ops) {
        double total = 0.0, c0 = 0.0, c1 = 0.0;
        for (size_t i = 0; i < ops.size(); ++i) {
            const SOp& op = ops[i];
            const double c = op.kind == OP_DIAG ? cost(0, op.qubits, 0) : cost(op.k, op.qubits, (int)op.epi.size());
            total += c;
            if (i == 0) c0 = c;
            if (i == 1) c1 = c;
        }
        // the start's share: its clusters written by one write-only pass
        const int fk = fold_kind(ops, gates, fold);
        if (fk == 4) total -= c0 + (1.0 - kFold7TableShare) * c1;
        if (fk == 3) total -= c0 + (1.0 - kFold2TableShare) * c1;
        if (fk == 2) total -= c0 + (1.0 - kFold2Share) * c1;
        if (fk == 1) total -= (1.0 - kFold1Share) * c0;
        return Cand(std::move(ops), total);
    };
    // A narrower cap usually only adds passes, so its set families and the
    // cost-trimmed schedule (which mixes widths) count only where the cap's
    // plain greedy schedule is predicted cheaper than the full-width one: a
    // circuit whose gates do not pack into full-width clusters (or
    // complex128, whose 6-qubit clusters are bound by the fp64 matrix cores)
    // gets them, while prediction noise alone cannot make a narrower cap win
    // on the other circuits. In parallel all candidates are built together
    // (one round of latency) and the gate applies when choosing; one after
    // another, the gated ones are built only where their cap qualifies.
    std::vector<std::function<Cand()>> fns;
    std::vector<int> gate;  // 0: always a candidate; kc: only where cap kc qualifies
    std::vector<int> key;   // start order on the pool: the long searches (over candidate sets) first
    auto add = [&](int g, std::function<Cand()> f, int k = 0) {
        gate.push_back(g);
        fns.push_back(std::move(f));
        key.push_back(k);
    };
    for (int kc = k_lo; kc <= kmax; ++kc)  // the plain schedules first: their prices decide which caps qualify
        add(0, [&, kc]() { return priced(greedy_ops(n, gates, S.dropped, S.n_applied, kc, o.fuse_diag)); });
    if (first_caps > 1) {  // the widest cap after a 6-qubit start, with and without the candidate sets
        add(0, [&]() {
            return priced(greedy_ops(n, gates, S.dropped, S.n_applied, kmax, o.fuse_diag, nullptr, nullptr, 6));
        });
        for (const std::vector<uint64_t>* fs : {&sets0, &sets1})
            if (!fs->empty())
                add(
                    0,
                    [&, fs]() {
                        return priced(greedy_ops(n, gates, S.dropped, S.n_applied, kmax, o.fuse_diag, nullptr, fs, 6));
                    },
                    1);
    }
    // the one-deviation schedules (gate -1: kept only where they need fewer
    // passes than every other candidate - among schedules of as many passes
    // the other candidates already offer the model its choice)
    if (cd_deviations)
        for (int st = 0; st < kDevSteps; ++st)
            for (int r = 1; r <= kDevRanks; ++r)
                add(
                    -1,
                    [&, st, r]() {
                        std::vector<SOp> ops = greedy_ops(n, gates, S.dropped, S.n_applied, kmax, o.fuse_diag, nullptr,
                                                          dev_sets, 0, st, r);
                        if (ops.empty()) return Cand(std::vector<SOp>(), -1.0);  // no candidate of that rank
                        return priced(std::move(ops));
                    },
                    2);
    if (kmax > 1)
        add(kmax - 1,
            [&]() { return priced(greedy_ops(n, gates, S.dropped, S.n_applied, kmax, o.fuse_diag, &cost)); });
    // set families: kmax's are at hand; a narrower cap's are found inside
    // its tasks, one task per (cap, slack)
    if (o.cluster_sets)
        for (int kc = std::max(2, k_lo); kc <= kmax; ++kc)
            for (int slack = 0; slack < 2; ++slack) {
                if (kc == kmax) {
                    const std::vector<uint64_t>* fs = slack ? &sets1 : &sets0;
                    if (fs->empty()) continue;
                    add(
                        0,
                        [&, fs]() {
                            return priced(
                                greedy_ops(n, gates, S.dropped, S.n_applied, kmax, o.fuse_diag, nullptr, fs));
                        },
                        1);
                } else {
                    add(kc, [&, kc, slack]() {
                        std::vector<uint64_t> a, b;
                        dense_sets(n, gates, S.dropped, kc, a, b);
                        const std::vector<uint64_t>& sets = slack ? b : a;
                        if (sets.empty()) return Cand(std::vector<SOp>(), -1.0);  // no such family: not a candidate
                        return priced(greedy_ops(n, gates, S.dropped, S.n_applied, kc, o.fuse_diag, nullptr, &sets));
                    });
                }
            }
    // First every ungated candidate (in parallel: all of them at once, with
    // the gated ones too where narrower caps are expected to pay), then the
    // gated ones whose cap qualified (a second round only where some did)
    const size_t nplain = (size_t)(kmax - k_lo + 1);
    std::vector<char> want(fns.size(), 0);
    for (size_t i = 0; i < fns.size(); ++i) want[i] = o.parallel ? (gate[i] <= 0 || narrow_likely) : i < nplain;
    std::vector<Cand> res = run_tasks(o.parallel, fns, &want, &key);
    std::vector<char> use_cap(kmax + 1, 1);
    for (int kc = k_lo; kc < kmax; ++kc) use_cap[kc] = res[kc - k_lo].second < res[kmax - k_lo].second;
    std::vector<char> rest(fns.size(), 0);
    bool more_needed = false;
    for (size_t i = nplain; i < fns.size(); ++i) {
        const bool w = gate[i] <= 0 || use_cap[gate[i]];
        rest[i] = w && !want[i];
        more_needed |= rest[i] != 0;
        want[i] = w;
    }
    if (more_needed) {
        std::vector<Cand> more = run_tasks(o.parallel, fns, &rest, &key);
        for (size_t i = nplain; i < fns.size(); ++i)
            if (rest[i]) res[i] = std::move(more[i]);
    }
    double passes = 0.0;  // fewest passes of the other candidates
    bool any = false;
    for (size_t i = 0; i < fns.size(); ++i)
        if (want[i] && gate[i] >= 0 && res[i].second >= 0) {
            const double p = effective_passes(res[i].first, gates, fold);
            if (!any || p < passes) passes = p;
            any = true;
        }
    std::vector<Cand> cands;
    for (size_t i = 0; i < fns.size(); ++i) {
        if (!want[i]) continue;
        if (gate[i] < 0 && (res[i].second < 0 || (any && effective_passes(res[i].first, gates, fold) >= passes)))
            continue;
        cands.push_back(std::move(res[i]));
    }
    double best_cost = 0.0;
    bool have = false;
    for (Cand& cand : cands) {
        if (cand.second < 0) continue;
        if (!have || cand.second < best_cost) {
            best_cost = cand.second;
            S.ops = std::move(cand.first);
            have = true;
        }
    }
    return S;
}

}  // namespace qsim
