// Sanitizer driver for the library's host-only scheduling code (scheduler.cpp,
// stages.cpp; built with host -fsanitize=address,undefined by
// tests/test_sanitizers_cpu.py): random gate lists through every scheduling
// mode and option, and stage plans. Checks that every
// gate a schedule keeps is applied exactly once and that stage plans keep the
// per-qubit order; the sanitizers report memory errors and undefined
// behaviour themselves.
#include <algorithm>
#include <cstdio>
#include <random>
#include <vector>

#include "qsim.h"
#include "qsim_internal.h"
#include "scheduler.h"

using namespace qsim;

namespace {
std::mt19937_64 rng(7);
int below(int m) { return (int)(rng() % (uint64_t)m); }

std::vector<SGate> random_gates(int n, int count, bool leading_h) {
    std::vector<SGate> g;
    if (leading_h)
        for (int q = 0; q < n; ++q) g.push_back(SGate{G_H, 1, {q, 0, 0, 0, 0, 0}, false});
    static const int named[] = {G_H, G_T, G_SX, G_SY, G_X, G_Y, G_Z, G_TDG};
    for (int i = 0; i < count; ++i) {
        SGate s{};
        const int r = below(10);
        if (r < 5 || n < 2) {
            s.kind = named[below(8)];
            s.nq = 1;
            s.q[0] = below(n);
        } else if (r < 8) {
            s.kind = G_CZ;
            s.nq = 2;
            s.q[0] = below(n);
            do s.q[1] = below(n); while (s.q[1] == s.q[0]);
        } else {
            s.kind = G_DENSE;
            s.nq = 1 + below(std::min(n, 6));
            for (int j = 0; j < s.nq; ++j) {
                bool dup;
                do {
                    s.q[j] = below(n);
                    dup = false;
                    for (int t = 0; t < j; ++t) dup |= s.q[t] == s.q[j];
                } while (dup);
            }
        }
        s.diag = gate_is_diagonal(s.kind);
        g.push_back(s);
    }
    return g;
}

int check_schedule(const Schedule& S, const std::vector<SGate>& g, int n, int kmax) {
    std::vector<int> seen(g.size(), 0);
    for (const SOp& op : S.ops) {
        // a cluster holds at most kmax qubits, or one dense gate wider than that
        int widest = 0;
        for (int m : op.members) widest = std::max(widest, g.at(m).nq);
        if (op.kind == OP_CLUSTER && (op.k < 1 || op.k > std::max(kmax, widest) || op.k > kMaxK)) return 1;
        for (int j = 0; j < op.k && op.kind != OP_GATE; ++j)
            if (op.qubits[j] < 0 || op.qubits[j] >= n || (j && op.qubits[j] <= op.qubits[j - 1])) return 2;
        for (int m : op.members) seen.at(m)++;
        for (int m : op.epi) seen.at(m)++;
    }
    for (size_t i = 0; i < g.size(); ++i)
        if (seen[i] != (S.dropped[i] ? 0 : 1)) return 3;
    return 0;
}

int check_stages(const StagePlan& P, const std::vector<SGate>& g, int n) {
    if (!P.ok) return 0;
    std::vector<int> last(n, 0);
    for (size_t i = 0; i < g.size(); ++i) {
        const int s = P.gate_stage[i];
        if (s < 0) continue;
        if (s >= (int)P.loc.size()) return 4;
        for (int j = 0; j < g[i].nq; ++j) {
            if (s < last[g[i].q[j]]) return 5;
            last[g[i].q[j]] = s;
        }
    }
    return 0;
}
}  // namespace

int main() {
    int bad = 0;
    const OpCostFn cost = [](int k, const int* q, int n_epi) { return 1.0 + k * 0.3 + q[0] * 0.01 + n_epi * 0.05; };
    for (int trial = 0; trial < 120 && !bad; ++trial) {
        const int n = 2 + below(30);
        const std::vector<SGate> g = random_gates(n, 10 + below(150), trial % 2 == 0);
        for (int mode = 0; mode <= 2 && !bad; ++mode)
            for (int kmax = 1; kmax <= kMaxK && !bad; ++kmax) {
                SchedOpts o;
                o.mode = mode;
                o.kmax = kmax;
                o.fold_start = below(4);
                o.fuse_diag = below(2);
                o.skip_trailing_diag = below(2);
                o.skip_initial_h = below(2);
                o.cluster_sets = below(2);
                o.parallel = false;
                const Schedule S = make_schedule(n, g, o, mode == 2 ? cost : OpCostFn());
                if (int e = check_schedule(S, g, n, mode == 0 ? 6 : kmax)) {
                    std::fprintf(stderr, "trial %d mode %d kmax %d: schedule check %d\n", trial, mode, kmax, e);
                    bad = 1;
                }
            }
        for (int l = (n + 1) / 2; l <= n && !bad; l += 1 + below(3)) {
            StageOpts so;
            so.n_local = l;
            so.spec_cz = below(2);
            so.spec_diag1 = below(2);
            so.search = below(2);
            so.early_swaps = below(2);
            so.kmax = below(kMaxK + 1);
            so.skip_initial_h = below(2);
            so.skip_trailing_diag = below(2);
            const StagePlan P = make_stage_plan(n, g, so);
            if (int e = check_stages(P, g, n)) {
                std::fprintf(stderr, "trial %d: stage check %d\n", trial, e);
                bad = 1;
            }
        }
    }
    std::printf("scheduler driver done: %s\n", bad ? "FAILED" : "ok");
    return bad;
}
