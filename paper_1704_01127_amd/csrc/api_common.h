// Host-side helpers shared by the C ABI entry points (state and batch).
#pragma once

#include <string>
#include <vector>

#include "qsim.h"
#include "qsim_internal.h"
#include "scheduler.h"

namespace qsim {
namespace api {

// Set the thread's last-error message and return st.
qsim_status fail(qsim_status st, const std::string& msg);
qsim_status hip_fail(hipError_t e, const char* where);

#define HIP_TRY(expr, where)                                      \
    do {                                                          \
        hipError_t e_ = (expr);                                   \
        if (e_ != hipSuccess) return ::qsim::api::hip_fail(e_, where); \
    } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int gate_nq(const qsim_gate& g);
// Kind, arity, matrix pointer and qubit range / distinctness of gate idx on n qubits.
qsim_status check_gate(int n, const qsim_gate& g, int idx);
// Matrix-build record of gate g inside a cluster (pos_of: qubit -> position
// in the sorted cluster, -1 outside); dense matrices are appended to `dense`.
BuildGate to_build_gate(const qsim_gate& g, const int* pos_of, std::vector<double>& dense);
// Diagonal gates applied while a cluster's results are stored: terms on
// target qubits only join the matrix (appended to bgates), the others go to e.
qsim_status split_epilogue(const int* pos_of, const qsim_gate* gates, const std::vector<int>& epi_gates,
                           std::vector<BuildGate>& bgates, std::vector<double>& dense, EpiDesc& e);
std::vector<SGate> to_sgates(const qsim_gate* gates, int n_gates);
OpCostFn cost_fn(const qsim_run_opts* o, int n, bool dbl);
SchedOpts to_sched_opts(const qsim_run_opts* o);
// SchedOpts::fold_start of a run on a state of n qubits (complex128 if dbl).
int fold_start_for(bool dbl, int n);

}  // namespace api
}  // namespace qsim
