// Gate scheduling: clustering of a gate list into k-qubit clusters
// (Haener & Steiger, Sec. 3.6.1, step 2) plus diagonal passes.
#pragma once

#include <cstdint>
#include <functional>
#include <vector>

namespace qsim {

struct SGate {
    int kind;
    int nq;
    int q[6];
    bool diag;
};

enum : int { OP_CLUSTER = 0, OP_DIAG = 1, OP_GATE = 2 };

constexpr int kSchedMaxK = 7;  // widest cluster (the library's kMaxK)

struct SOp {
    int kind = OP_CLUSTER;
    int k = 0;
    int qubits[kSchedMaxK] = {};  // sorted (clusters); the gate's qubits (per-gate ops)
    std::vector<int> members;            // gates folded into the matrix / the pass / the single gate
    std::vector<int> epi;                // diagonal gates applied while storing
};

// Predicted time (microseconds) of one cluster op on k qubits with the given
// sorted qubits; used by the cost-driven scheduler.
using OpCostFn = std::function<double(int k, const int* qubits, int n_epi)>;

struct SchedOpts {
    int kmax = 5;
    int mode = 1;  // 0 per-gate, 1 greedy, 2 cost-driven
    bool fuse_diag = false;
    bool skip_trailing_diag = false;
    bool skip_initial_h = false;
    bool cluster_sets = true;  // also offer closures of dense qubit sets (greedy and cost-driven)
    bool parallel = true;      // build candidate schedules on threads of their own
    bool deviations = true;    // also the one-deviation schedules (see kDevSteps), on large states
    // How a run from the uniform state (skip_initial_h) writes its start:
    // 0 an initialisation pass; 1 the first cluster with it, in one write-only
    // pass; 2 also a second cluster of 6 qubits, multiplied per column on the
    // matrix cores; 3 as 2, in the table form where it applies (the second
    // cluster shares at most 2 qubits with the first, and 2^(shared + rows the
    // first cluster's diagonal gates sign-flip) <= 128). Schedules are
    // compared with that pass priced as write-only, and with 2 or 3 and
    // kmax > 6 candidates whose first two clusters have at most 6 qubits are
    // offered as well.
    int fold_start = 0;
};

// Cost of the write-only start relative to the full passes it replaces:
// measured on the 30-qubit complex64 state, the uniform start with one cluster
// takes 0.41-0.49 of a cluster pass, with two clusters 0.69 of a 6-qubit pass
// on the matrix cores and 0.47 in the table form (1.63 ms, the write
// ceiling, against 3.48 ms).
constexpr double kFold1Share = 0.45;
constexpr double kFold2Share = 0.70;
constexpr double kFold2TableShare = 0.47;
// with a 7-qubit second cluster (table form only): the write-only pass
// against a 7-qubit pass
constexpr double kFold7TableShare = 0.45;
// Table form limits: at most 2 shared qubits and 2^(shared + sign-flipped
// rows) table rows of the second cluster's outputs: 128 rows of 64 outputs
// (k = 6) or 64 rows of 128 (k = 7), 64 KiB either way.
constexpr int kFoldTableBits6 = 7;
constexpr int kFoldTableBits7 = 6;
// The one-deviation search (schedules that take, at one of the first
// kDevSteps steps, one of the kDevRanks next-best clusters instead of the
// best, a limited-discrepancy search) costs about 0.7 ms of host time; it
// runs where a pass takes longer than that (states of at least
// kDevMinQubits qubits) and candidates are built in parallel.
constexpr int kDevSteps = 3;
constexpr int kDevRanks = 4;
constexpr int kDevMinQubits = 29;

// The folded start a schedule's first ops take (SchedOpts::fold_start): 0
// none, 1 the first cluster, 2 two clusters with the second (6 qubits) on the
// matrix cores, 3 the same in the table form, 4 two clusters with a 7-qubit
// second one in the table form.
int schedule_fold_kind(const std::vector<SOp>& ops, const std::vector<SGate>& gates, int fold_start);

struct Schedule {
    std::vector<SOp> ops;
    bool uniform_init = false;  // leading H layer replaced by uniform initialisation
    std::vector<char> dropped;  // per gate: removed by a skip option
    int n_applied = 0;
};

// Gates a run leaves out (Sec. 3.6): with skip_initial_h, the first gate of
// every qubit when all of them are H (the run starts from the uniform state
// instead; uniform_init is then set); with skip_trailing_diag, every diagonal
// gate that no non-diagonal gate follows on any of its qubits.
void mark_skips(int n, const std::vector<SGate>& gates, bool skip_initial_h, bool skip_trailing_diag,
                std::vector<char>& dropped, bool& uniform_init);

// Build the schedule. `cost` is used by mode 2 only: the greedy schedule of
// every cap k <= kmax is built and the cheapest by predicted total wins
// (empty cost: the greedy schedule with cap kmax).
Schedule make_schedule(int n, const std::vector<SGate>& gates, const SchedOpts& o, const OpCostFn& cost);

// Stage finding for a state spread over 2^(n - n_local) memories
// (Sec. 3.6.1 steps 1 and 3, Sec. 3.5); stages.cpp.
struct StageOpts {
    int n_local = 30;          // bit locations 0 .. n_local - 1 are local
    bool spec_cz = true;       // CZ on global qubits needs no communication
    bool spec_diag1 = false;   // nor do diagonal single-qubit gates
    bool search = true;        // cheap search for the qubits to swap (else the lowest locations)
    bool early_swaps = true;   // step 3
    int kmax = 5;              // clusters within each stage (0: none)
    bool fuse_diag = false;
    bool skip_initial_h = false;
    bool skip_trailing_diag = false;
};

struct StagePlan {
    bool ok = true;                        // false: a gate gathers more qubits than are local
    std::vector<int> gate_stage;           // per gate: its stage, -1 when skipped
    std::vector<std::vector<int>> loc;     // per stage: bit location of every qubit
    std::vector<int> n_clusters;           // per stage, with kmax > 0
    int n_moved = 0;                       // clusters moved across a swap by step 3
};

StagePlan make_stage_plan(int n, const std::vector<SGate>& gates, const StageOpts& o);

}  // namespace qsim
