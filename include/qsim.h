/*
 * qsim.h - C ABI of a state-vector quantum circuit simulator for one AMD
 * Instinct MI355X (gfx950).
 *
 * The method is the one of Haener & Steiger, "0.5 Petabyte Simulation of a
 * 45-Qubit Quantum Circuit" (SC'17): an n-qubit state is a vector of 2^n
 * complex amplitudes (Sec. 2); gates are applied in place; many gates are
 * fused into one dense k-qubit gate by a clustering scheduler (Sec. 3.6.1,
 * step 2) and each such k-qubit gate is applied by gathering the 2^k
 * amplitudes that share all non-target bits, multiplying them by the 2^k x 2^k
 * matrix and scattering them back (Sec. 3.2). Diagonal gates (CZ, T, Z) need
 * no gather (Sec. 3.5) and are applied as one pass, or fused into the
 * neighbouring cluster's store.
 *
 * Conventions used by every call:
 *   - amplitude index i = sum_q b_q 2^q: qubit q is bit q of the index (Sec. 2);
 *   - a k-qubit matrix is 2^k x 2^k complex128, row-major, (re, im)
 *     interleaved; bit j of its row/column index belongs to qubits[j]
 *     (Sec. 3.2), the qubits may be listed in any order;
 *   - the state is interleaved complex: QSIM_C64 = (float re, float im),
 *     QSIM_C128 = (double re, double im), the layouts of torch.complex64 and
 *     torch.complex128.
 *
 * Ownership: the caller owns all device memory (state and workspace). The
 * library never allocates or frees device memory; it enqueues its work on the
 * caller's HIP stream and returns before the work is done. Host pointers are
 * read only during the call. A qsim_state handle holds metadata only.
 *
 * Errors: every call returns a qsim_status; QSIM_OK is 0, errors are
 * negative, and qsim_last_error() returns a message for the calling thread.
 * Argument errors are detected on the host before anything is enqueued.
 * Errors of enqueued GPU work surface at the next qsim_sync() or
 * qsim_probs()/qsim_compare() (which synchronise the stream).
 */
#ifndef QSIM_H
#define QSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qsim_state_s* qsim_state;

/* Widest cluster the scheduler forms (a fused k-qubit gate, Sec. 3.6.1) and
 * widest single gate a caller passes. 7-qubit clusters exist on complex64
 * states of at least 12 qubits while QSIM_OPT_K6_KERNEL is 2 (fp16 matrix
 * cores with operand halves); elsewhere the cap is 6. Per-op qubit lists
 * (qsim_op_timings, qsim_schedule) have QSIM_MAX_CLUSTER entries per op. */
#define QSIM_MAX_CLUSTER 7
#define QSIM_MAX_GATE_QUBITS 6

typedef enum { QSIM_C64 = 1, QSIM_C128 = 2 } qsim_dtype;

/* Initial contents of the state at qsim_create / qsim_init_state.
 * QSIM_INIT_ZERO    |0...0>
 * QSIM_INIT_UNIFORM every amplitude 2^{-n/2}: the state after the cycle-0
 *                   Hadamard layer, which a simulator may skip (Sec. 3.6)
 * QSIM_INIT_KEEP    leave the buffer as the caller filled it */
typedef enum { QSIM_INIT_ZERO = 0, QSIM_INIT_UNIFORM = 1, QSIM_INIT_KEEP = 2 } qsim_init;

typedef enum {
    QSIM_OK = 0,
    QSIM_E_INVALID = -1,     /* bad argument: qubit >= n or repeated, null pointer, buffer too small */
    QSIM_E_UNSUPPORTED = -2, /* a gate over 6 qubits, kmax over 7, n out of range, too many entries in a
                                diagonal layer */
    QSIM_E_DEVICE = -3       /* a HIP runtime error or a failed GPU launch */
} qsim_status;

/* Gate kinds. The named matrices are the ones printed in Sec. 2 (H, T, X^1/2,
 * Y^1/2, X, CZ), the Pauli Y and Z, the inverses of T, X^1/2 and Y^1/2 (for
 * mirrored circuits), a phase gate diag(1, e^{i theta}) and a dense k-qubit
 * matrix (k <= 6). */
typedef enum {
    QSIM_GATE_H = 0,
    QSIM_GATE_T = 1,
    QSIM_GATE_SQRT_X = 2,
    QSIM_GATE_SQRT_Y = 3,
    QSIM_GATE_X = 4,
    QSIM_GATE_Y = 5,
    QSIM_GATE_Z = 6,
    QSIM_GATE_CZ = 7,
    QSIM_GATE_TDG = 8,
    QSIM_GATE_SQRT_X_DG = 9,
    QSIM_GATE_SQRT_Y_DG = 10,
    QSIM_GATE_PHASE = 11, /* diag(1, e^{i theta}) */
    QSIM_GATE_DENSE = 12  /* k qubits, matrix in `mat` (host, 2^k x 2^k complex128) */
} qsim_gate_kind;

typedef struct {
    int32_t kind;       /* qsim_gate_kind */
    int32_t k;          /* number of qubits: 1, 2 for CZ, 1..6 for DENSE */
    int32_t qubits[6];  /* target qubits; bit j of a DENSE matrix index <-> qubits[j] */
    double theta;       /* angle of QSIM_GATE_PHASE */
    const double* mat;  /* DENSE only: host pointer, read during the call */
} qsim_gate;

/* How qsim_run_circuit executes a gate list. */
typedef enum {
    QSIM_SCHED_PER_GATE = 0, /* one launch per gate, no fusion (the plain method) */
    QSIM_SCHED_GREEDY = 1,   /* clusters of <= kmax qubits, most gates per cluster (Sec. 3.6.1, step 2) */
    QSIM_SCHED_ANALYTIC = 2, /* greedy schedules for every cap <= kmax, the cheapest under the
                                measured cost table (qsim_set_cost_table) wins */
    QSIM_SCHED_LEARNED = 3   /* as ANALYTIC with the MLP cost model loaded by qsim_set_cost_model;
                                falls back to GREEDY when none is loaded */
} qsim_scheduler;

typedef struct {
    int32_t kmax;               /* largest cluster, 1..7 (ignored by PER_GATE); runs and schedules
                                   cap it at 6 where no 7-qubit kernel applies (QSIM_MAX_CLUSTER) */
    int32_t scheduler;          /* qsim_scheduler */
    int32_t skip_trailing_diag; /* drop diagonal gates after the last non-diagonal gate on all
                                   their qubits: they change phases, not probabilities (Sec. 3.6) */
    int32_t fuse_diag;          /* let a cluster carry diagonal gates outside its qubits and apply
                                   them while storing (no extra pass over the state) */
    int32_t skip_initial_h;     /* the run starts from |0...0>. If every qubit's first gate is an
                                   H, that layer is replaced by writing the uniform state over
                                   the whole vector (its contents are not read; Sec. 3.6);
                                   otherwise the caller promises the state holds |0...0> */
    int32_t record_timings;     /* time every launched op with HIP events (slows the run) */
    int32_t schedule_dtype;     /* qsim_dtype the cost models assume in qsim_schedule
                                   (qsim_run_circuit uses the state's); 0 = C64 */
    int32_t fused_stats;        /* when the run's last op is a cluster on a complex64 state applied
                                   by a direct matrix-core kernel (k = 4..7) or, for k = 2, 3 on a
                                   state of at least k + 6 qubits, by the staged vector-ALU kernel,
                                   that kernel also sums
                                   the float64 norm, sum of p^2 and entropy of the amplitudes it
                                   stores, and the next qsim_probs with dev_out = NULL returns them
                                   without reading the state again. Any library call that changes
                                   the state or computes other reductions discards them; a caller
                                   that writes the amplitudes itself must not set this flag. */
} qsim_run_opts;

typedef struct {
    int32_t n_ops;              /* launches of cluster / diagonal / per-gate kernels */
    int32_t n_clusters_by_k[8]; /* clusters applied, by k (index 0 unused) */
    int32_t n_diag_ops;         /* standalone diagonal passes */
    int32_t n_gates_applied;    /* gates after trailing / initial skips */
    int32_t n_gates_fused_epilogue;
    double schedule_ms;         /* host time spent scheduling */
    double total_ms;            /* host wall time of the call (launches are asynchronous) */
} qsim_run_stats;

/* Workspace needed for a state of n qubits and dtype dt when clusters have
 * at most kmax qubits. The workspace holds cluster matrices, descriptors and
 * reduction partial sums. */
size_t qsim_workspace_bytes(int n_qubits, qsim_dtype dt, int kmax);

/* Create a handle for the state held in dev_amps: the 2^n complex amplitudes
 * of an n-qubit state, amplitude i belonging to the basis state whose bit q is
 * the value of qubit q (Sec. 2). dev_amps holds 2^n amplitudes of dt,
 * >= 256-byte aligned, amps_bytes >= 2^n * sizeof(amplitude), with the
 * workspace dev_workspace (>= qsim_workspace_bytes, 256-byte aligned). Both
 * buffers stay owned by the caller and must outlive the handle. hip_stream
 * is a hipStream_t (NULL = the default stream). n_qubits in [1, 34] for C64,
 * [1, 33] for C128. Enqueues the initialisation `init`. */
qsim_status qsim_create(int n_qubits, qsim_dtype dt, void* dev_amps, size_t amps_bytes,
                        void* dev_workspace, size_t ws_bytes, void* hip_stream, qsim_init init,
                        qsim_state* out);
qsim_status qsim_destroy(qsim_state s);
qsim_status qsim_init_state(qsim_state s, qsim_init init);

/* Apply one dense k-qubit gate (Sec. 3.2) in place: for every assignment c of
 * the n-k other bits, psi[c + dep(y)] <- sum_x mat[y][x] psi[c + dep(x)],
 * where dep(x) puts bit j of x at qubit qubits[j]. 1 <= k <= 6, qubits
 * distinct and < n. mat: host, 2^k x 2^k complex128 row-major. The matrix is
 * re-indexed to sorted qubit order (Sec. 3.2) and, for a C64 state, rounded
 * to float. */
qsim_status qsim_apply_cluster(qsim_state s, int k, const int32_t* qubits, const double* mat);

/* Apply a diagonal layer in place, with no gather (Sec. 3.5): every amplitude
 * is multiplied by prod_{pairs (a,b)} (-1)^{b_a b_b} * prod_j e^{i theta_j b_{q_j}}.
 * cz_pairs: 2*n_pairs qubit indices (host); phase_qubits / phase_theta:
 * n_phase entries (host). At most 64 pairs and 64 phases. */
qsim_status qsim_apply_diag(qsim_state s, int n_pairs, const int32_t* cz_pairs, int n_phase,
                            const int32_t* phase_qubits, const double* phase_theta);

/* Relabel bit locations in place (the local swap of Sec. 3.4, which moves
 * the qubits to be exchanged to chosen bit locations): for j < m the bit at
 * location from[j] moves to location to[j], i.e. the amplitude at index i
 * goes to the index whose bit to[j] is bit from[j] of i; other bits stay.
 * from and to list the same m <= 12 distinct locations (< n). One pass over
 * the state (read and write), in tiles of up to 2^12 amplitudes staged
 * through LDS. Errors: QSIM_E_UNSUPPORTED for m > 12, QSIM_E_INVALID for
 * locations out of range, repeated, or differing between from and to. */
qsim_status qsim_permute_qubits(qsim_state s, int m, const int32_t* from, const int32_t* to);

/* Apply one gate with the per-gate kernels (one launch; the plain method):
 * a 2x2 matrix on the index pairs (i, i + 2^q) (Sec. 2), a sign flip for CZ,
 * a phase on the amplitudes with bit q set for diagonal 1-qubit gates, and
 * the cluster kernel for DENSE. */
qsim_status qsim_apply_gate(qsim_state s, const qsim_gate* gate);

/* Run a gate list (in circuit order) on the state. With a fusing scheduler
 * the gates are clustered (Sec. 3.6.1, step 2), every cluster matrix is built
 * in float64 on the GPU and applied by the cluster kernel. stats may be
 * NULL. */
qsim_status qsim_run_circuit(qsim_state s, const qsim_gate* gates, int n_gates,
                             const qsim_run_opts* opts, qsim_run_stats* stats);

/* Output probabilities p_i = |a_i|^2 (Sec. 3.6) and float64 reductions on the
 * GPU: norm = sum p_i, sum_p2 = sum p_i^2, entropy = -sum p_i ln p_i (nats).
 * dev_out (nullable): 2^n reals of out_dt (QSIM_C64 -> float, QSIM_C128 ->
 * double). Scalar pointers are host pointers and may be NULL. Synchronises
 * the stream. */
qsim_status qsim_probs(qsim_state s, void* dev_out, qsim_dtype out_dt, double* norm,
                       double* sum_p2, double* entropy_nats);

/* Compare the state with a reference vector on the GPU, in float64:
 * fidelity = |<ref|psi>|^2 / (<ref|ref> <psi|psi>), max_abs_diff = max_i
 * |psi_i - ref_i|. dev_ref: 2^n amplitudes of ref_dt. Synchronises. */
qsim_status qsim_compare(qsim_state s, const void* dev_ref, qsim_dtype ref_dt, double* fidelity,
                         double* max_abs_diff);

/* Tell the library that the caller has written the amplitudes itself (a
 * copy into dev_amps): the float64 sums a fused_stats run left for the next
 * qsim_probs describe the old state and are dropped. No GPU work. */
qsim_status qsim_state_changed(qsim_state s);

/* qsim_probs for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results as qsim_probs on the 2^n amplitudes of dt at
 * dev_amps (amps_bytes >= 2^n * sizeof(amplitude)), with no state handle and
 * no workspace. The reduction's partial sums go to a fixed device array of
 * the library (qsim_noalloc_scratch_bytes(), about 128 KiB, one per GPU, held
 * until the process ends); nothing is allocated. Enqueued on hip_stream (a
 * hipStream_t, NULL = default) on the current device, then synchronised.
 * Calls that overlap on one GPU (other host threads, other streams) share the
 * array and race: the caller serialises them. n_qubits in [1, 34] for C64,
 * [1, 33] for C128; larger states are rejected with QSIM_E_UNSUPPORTED. */
qsim_status qsim_probs_noalloc(int n_qubits, qsim_dtype dt, const void* dev_amps, size_t amps_bytes,
                               void* hip_stream, void* dev_out, qsim_dtype out_dt, double* norm,
                               double* sum_p2, double* entropy_nats);
size_t qsim_noalloc_scratch_bytes(void);

/* Wait for the state's stream; reports errors of enqueued work. */
qsim_status qsim_sync(qsim_state s);

/* Message of the last error on the calling thread ("" if none). */
const char* qsim_last_error(void);

/* Per-launch GPU times of the last qsim_run_circuit that had record_timings
 * set, measured with HIP events on the state's stream. For each launch, in
 * order: op_kind (0 cluster, 1 diagonal pass, 2 single-qubit gate, 3
 * single-qubit phase, 4 CZ, 5 cluster-matrix build, 6 uniform initialisation
 * written together with the first cluster, 7 two clusters in one pass, 8 the
 * uniform initialisation and the first two clusters in one pass, 9 the
 * permutation pass of QSIM_OPT_MAP_QUBITS),
 * op_k (cluster size - 5 for a pair, 6 for kind 8; number of matrices for a build),
 * op_qubits[QSIM_MAX_CLUSTER*i ..] (sorted targets of a cluster - of the first for a pair,
 * of the second for kind 8 -
 * or the gate's qubits, -1 padded), op_epi (flags of a cluster: bit 0 = applies diagonal
 * gates while storing, bit 1 = LDS-staged kernel variant, bit 2 = matrix-core
 * kernel, bit 3 = also sums the reductions, bit 4 = kind 8 in its table form
 * (QSIM_OPT_FOLD_TABLE), bits 8-15 = the number of diagonal
 * gates the scheduler attached to it, capped at 255 - the epilogue size the
 * learned cost model is given) and ms (milliseconds). Arrays of cap entries (any may be NULL);
 * *n_ops receives the count. Synchronises the stream. */
qsim_status qsim_op_timings(qsim_state s, int32_t* op_kind, int32_t* op_k, int32_t* op_qubits,
                            int32_t* op_epi, float* ms, int cap, int* n_ops);

/* Process-wide tuning (the autotuner's controls).
 * The matrix-core cluster kernels (k <= 5; k = 6 on complex64 states; k = 7
 * has the direct form only) exist
 * in two variants: 0 gathers each lane's amplitudes straight from HBM into
 * registers, 1 moves the wave's tile as linear runs and re-orders it through
 * LDS. The variant is looked up per
 * (dtype, k, low_class = number of targets among qubits 0..5, capped at 3) in
 * a tune table, which qsim_set_tune_entry overwrites (the autotuner fills it
 * from measurements). QSIM_OPT_CLUSTER_VARIANT = 0 or 1 forces one variant
 * everywhere, -1 (default) uses the table. Batches: QSIM_OPT_BATCH_GRID is
 * the number of work-groups of the persistent launch (0, the default: one
 * 8-wave work-group per compute unit, the kernel's occupancy); QSIM_OPT_BATCH_PAD picks the
 * identity qubits that pad a cluster to 5 targets (0, default: the lowest
 * qubits outside it, which lengthens the contiguous runs of a tile; 1: the
 * highest); QSIM_OPT_BATCH_ITEM_TILES is the number of tiles (2^11
 * amplitudes each) of one work item, a power of two in [1, 4096] (default
 * 128), read when a batch is planned. QSIM_OPT_K6_KERNEL picks the kernel
 * of 6-qubit clusters on complex64 states: 0 the fp32 real-split product, 1
 * the fp32 three-multiplication complex product, 2 (default) fp16 matrix
 * cores on hi / lo halves of the operands (about 2^-21 relative error, the
 * size of fp32 rounding); only with 2 are 7-qubit clusters formed (the same
 * halves on the matrix's real and imaginary parts),
 * read when a cluster is enqueued. QSIM_OPT_FOLD_INIT (default 2): when a
 * run starts from the uniform state (skip_initial_h) with a cluster, 1
 * writes that state and the cluster - a product state again - in one pass
 * instead of an initialisation pass and a cluster pass; 2 also takes in the
 * second op when it is a 6-qubit cluster on a complex64 state: its inputs are
 * computed from that closed form instead of read, so one write-only pass
 * stands for three; 0 keeps them apart. QSIM_OPT_FOLD_TABLE (default 1):
 * with QSIM_OPT_FOLD_INIT 2, the second cluster's input column is w (the
 * first cluster applied to the uniform vector) at an index that varies over
 * the rows only through the qubits both clusters share, with the signs of the
 * first cluster's diagonal gates that couple a column qubit to a row. When at
 * most 2 qubits are shared and 2^(shared + sign-flipped rows) <= 128, the
 * second cluster's outputs for every such (shared pattern, sign mask) are
 * computed once, in float64, into a table of at most 64 KiB, and the
 * write-only pass combines at most 4 of its rows per column instead of
 * multiplying the column on the matrix cores; 0 always multiplies.
 * QSIM_OPT_PAIR
 * (default 0): on complex64 states of >= 11 qubits, two consecutive clusters
 * of <= 5 qubits are applied in one pass over the state (their qubits fit one
 * tile held in LDS; fp16 matrix cores on operand halves); 2 sends every such
 * cluster alone through that kernel. It is off by default because the paired
 * pass is limited by per-wave ALU and LDS work and takes longer than two
 * single passes. QSIM_OPT_PAIR_TILE is that tile's size in qubits, 11
 * (default) or 10 (12 waves per compute unit; a pair whose ten qubits leave
 * out qubit 0 uses the 11-qubit tile). QSIM_OPT_CLUSTER_SETS (default 1):
 * the clustering schedulers (greedy and cost-driven) also offer, at every
 * step, the closure of each dense connected qubit set of the circuit's
 * interaction graph (all ready gates inside the set) besides the clusters
 * grown gate by gate from a seed, and keep the schedule with fewer ops
 * (greedy) or the smaller predicted time (cost-driven); 0 grows from seeds
 * only (Sec. 3.6.1's greedy), read when a schedule is built.
 * QSIM_OPT_DEVIATIONS (default 1): on states of at least 29 qubits, runs that
 * build their candidate schedules in parallel (qsim_run_circuit,
 * qsim_schedule) also build the schedules that differ from the greedy choice
 * at one of the first 3 steps, taking one of the 4 next-best clusters there
 * (with the larger family of dense qubit sets), and keep one only if it
 * needs fewer passes than every other candidate (a limited-discrepancy
 * search, about 0.3 ms of host time); 0 skips them. Read when a schedule is
 * built.
 * QSIM_OPT_BATCH_ORDER: the order in which a batch's work items are handed
 * out, read when a batch is planned: 0 (default) level order (the j-th op
 * of every circuit before any (j+1)-th), 1 critical path first (a list
 * schedule simulated on the host: an op's items become available when the
 * circuit's previous op is done, circuits with the longest remaining chain
 * go first; it shortens the end of the launch, where only the deepest
 * circuits are left, but costs more planning than it saves on the
 * 512-circuit workload), 2 diagonal order (op j of circuit i gets key i + j,
 * so only about as many circuits as they have ops are in flight: for circuits
 * that are pieces of one large state, which then stay in the Infinity Cache
 * between their ops). Every order is free of deadlock.
 * QSIM_OPT_CHECK_UNITARY (default 0; a debugging aid): 1 makes every call
 * that takes a dense matrix (qsim_apply_cluster, DENSE gates of runs,
 * schedules and batches) check on the host that max_ij |(M M^+ - I)_ij| <=
 * 1e-10 (the gates of Sec. 2 are unitary) and return QSIM_E_INVALID
 * otherwise, before anything is enqueued.
 * QSIM_OPT_MAP_QUBITS (default 0; the GPU form of the qubit mapping of
 * Sec. 3.6.2): 1 lets a fusing run that starts from the uniform state
 * (skip_initial_h) place the qubits its clusters use least on the bit
 * locations where the cluster kernels are slowest (the lowest six and the top
 * three) - free at the start, since every relabelling of the uniform state is
 * the same state - and restore the caller's order with one permutation pass
 * at the end (at most twelve moving locations). Read when a run is
 * scheduled. Errors:
 * QSIM_E_INVALID for an unknown option or an out-of-range value. */
typedef enum {
    QSIM_OPT_CLUSTER_VARIANT = 1,
    QSIM_OPT_BATCH_GRID = 2,
    QSIM_OPT_BATCH_PAD = 3,
    QSIM_OPT_BATCH_ITEM_TILES = 4,
    QSIM_OPT_K6_KERNEL = 5,
    QSIM_OPT_FOLD_INIT = 6,
    QSIM_OPT_PAIR = 7,
    QSIM_OPT_PAIR_TILE = 8,
    QSIM_OPT_CLUSTER_SETS = 9,
    QSIM_OPT_BATCH_ORDER = 10,
    QSIM_OPT_CHECK_UNITARY = 11,
    QSIM_OPT_MAP_QUBITS = 12,
    QSIM_OPT_FOLD_TABLE = 13,
    QSIM_OPT_DEVIATIONS = 14
} qsim_option;
qsim_status qsim_set_option(int option, int value);
int qsim_get_option(int option);
qsim_status qsim_set_tune_entry(qsim_dtype dt, int k, int low_class, int variant);
int qsim_get_tune_entry(qsim_dtype dt, int k, int low_class);

/* Cost table of QSIM_SCHED_ANALYTIC: us_by_k[k] = measured microseconds of one
 * op on a state of n_ref qubits (index 0: a diagonal pass, 1..7: a k-qubit
 * cluster); costs scale as 2^(n - n_ref) because every op streams the whole
 * state (Sec. 3.1: the kernels are memory bound; a compute-bound k shows up as
 * a larger entry). The cost-driven schedulers build the greedy schedule for
 * every cap k <= kmax and keep the one with the smallest predicted total time.
 * The autotuner measures the table. */
qsim_status qsim_set_cost_table(qsim_dtype dt, const double* us_by_k, int n_ref);

/* ------------------------------------------------------------------------
 * Learned cost model (QSIM_SCHED_LEARNED). Not in the paper: the paper picks
 * k_max per machine by benchmarks (Sec. 3.3, 3.6.1); here a small MLP trained
 * on the simulator's own recorded kernel times predicts the time of a
 * candidate op, and the scheduler keeps the candidate schedule with the
 * smallest predicted total.
 *
 * Features of an op (k = 0: a standalone diagonal pass; qubits sorted): a
 * vector of qsim_cost_feature_count() floats, computed the same way for
 * training data and for scheduling. */
int qsim_cost_feature_count(void);
qsim_status qsim_cost_features(int n_qubits, qsim_dtype dt, int k, const int32_t* qubits, int n_epi,
                               float* out);

/* MLP in -> H -> H -> 1, ReLU, float32. Parameters in one array:
 * W1[H][in], b1[H], W2[H][H], b2[H], W3[H], b3[1] (qsim_mlp_param_count).
 * The prediction y of normalised features x = (f - feat_mean) / feat_std is
 * ln(microseconds per 2^30 amplitudes) = y * y_std + y_mean. Host copies are
 * taken; params = NULL unloads the model (LEARNED then falls back to the
 * fixed-k greedy scheduler). in must equal qsim_cost_feature_count(), H <= 64
 * for the GPU kernels (256 on the host). */
size_t qsim_mlp_param_count(int n_in, int n_hidden);
qsim_status qsim_set_cost_model(const float* params, int n_in, int n_hidden, const float* feat_mean,
                                const float* feat_std, double y_mean, double y_std);
/* Predicted microseconds of one op under the loaded model (1.0 if none; -1.0
 * for k outside 0..QSIM_MAX_CLUSTER or a null qubit list with k > 0). */
double qsim_cost_model_predict_us(int n_qubits, qsim_dtype dt, int k, const int32_t* qubits, int n_epi);
/* Host forward pass (float32, fused multiply-adds in index order): y[b] for x[batch][in]. */
qsim_status qsim_mlp_predict_host(const float* params, int n_in, int n_hidden, const float* x, int batch,
                                  float* y);

/* GPU training kernels (device pointers, enqueued on `stream`, n_in <= 32,
 * n_hidden <= 64). Forward: y[b] for x[batch][in], the same arithmetic as the
 * host pass. Backward: gradient of the mean squared error
 * L = (1/batch) sum_b (y_b - target_b)^2 with respect to every parameter, and
 * L itself (dev_loss, nullable); dev_scratch holds
 * qsim_mlp_scratch_floats(n_in, n_hidden, batch) floats. Adam: one step of
 * Kingma & Ba's update with bias correction at step `step` (>= 1). */
size_t qsim_mlp_scratch_floats(int n_in, int n_hidden, int batch);
qsim_status qsim_mlp_forward(int n_in, int n_hidden, const float* dev_params, const float* dev_x, int batch,
                             float* dev_y, void* stream);
qsim_status qsim_mlp_backward(int n_in, int n_hidden, const float* dev_params, const float* dev_x,
                              const float* dev_target, int batch, float* dev_grad, float* dev_loss,
                              float* dev_scratch, void* stream);
qsim_status qsim_mlp_adam(int n_params, float* dev_params, const float* dev_grad, float* dev_m, float* dev_v,
                          int step, float lr, float beta1, float beta2, float eps, void* stream);

/* Host-only: the schedule qsim_run_circuit would use (no GPU work). For each
 * gate: gate_op[g] = index of the op applying it (-1 if skipped) and
 * gate_role[g] = 0 (folded into the op's matrix), 1 (applied while storing,
 * diagonal) or 2 (the op is a standalone diagonal pass). For each op:
 * op_kind[o] (0 cluster, 1 diagonal pass, 2 per-gate), op_k[o] and its sorted
 * qubits op_qubits[QSIM_MAX_CLUSTER*o ..]. Arrays of op_cap entries; *n_ops receives the
 * count. Returns QSIM_E_INVALID if op_cap is too small. */
qsim_status qsim_schedule(int n_qubits, const qsim_gate* gates, int n_gates,
                          const qsim_run_opts* opts, int32_t* gate_op, int32_t* gate_role,
                          int32_t* op_kind, int32_t* op_k, int32_t* op_qubits, int op_cap,
                          int* n_ops);

/* ------------------------------------------------------------------ stages
 * Stage finding for a state spread over 2^g memories (host only, no GPU
 * work). Qubits sit at bit locations 0..n-1 of the amplitude index; locations
 * below n_local are local, the g = n - n_local above them global. A gate runs
 * without communication when every qubit it gathers is local (Sec. 3.4).
 * Step 1 (Sec. 3.6.1): gates on different qubits commute, so the largest
 * first stage - every gate that can run before a global qubit is needed - is
 * taken; then all g global qubits are swapped with g local qubits (one
 * all-to-all, Sec. 3.4) and the next stage is grown, until the circuit ends.
 * The local qubits that go global are those at the lowest locations
 * (search = 0, the paper's upper bound) or the result of a cheap search
 * (search = 1: candidate sets led by the qubits whose next gather lies
 * furthest ahead, each played out to the end; fewest swaps wins; the first
 * layout, free because no state exists yet, is searched too). Sec. 3.5's
 * specialisation: a CZ on global qubits is a conditional phase or local Z and
 * needs no swap (specialize bit 0); diagonal single-qubit gates are phases
 * (bit 1; the paper's stage finding assumes the random gates dense, i.e. bit 1
 * off). Step 2: each stage's gates are clustered (kmax > 0; only local qubits
 * count, Table 1). Step 3 (early_swaps): a stage's last cluster moves past the
 * following swap when its gates can run there and the two stages then need
 * fewer clusters; the number of swaps does not change. */
typedef struct {
    int32_t n_local;            /* n/2 <= n_local <= n */
    int32_t specialize;         /* bit 0: CZ on global qubits; bit 1: diagonal 1-qubit gates */
    int32_t search;
    int32_t early_swaps;
    int32_t kmax;               /* 0..7; 0 = no clustering (stage_clusters reads -1) */
    int32_t fuse_diag;          /* clustering option, as in qsim_run_opts */
    int32_t skip_initial_h;     /* as in qsim_run_opts */
    int32_t skip_trailing_diag; /* as in qsim_run_opts */
} qsim_stage_opts;

/* gate_stage (n_gates, nullable): stage of each gate, -1 when skipped.
 * stage_loc (max_stages * n_qubits, nullable): bit location of qubit q in
 * stage s at [s * n_qubits + q]; consecutive stages differ by one swap.
 * stage_clusters (max_stages, nullable): clusters of each stage. *n_stages
 * receives the number of stages (swaps + 1), also when max_stages is too
 * small (then QSIM_E_INVALID and nothing else is written). */
qsim_status qsim_stage_schedule(int n_qubits, const qsim_gate* gates, int n_gates, const qsim_stage_opts* opts,
                                int32_t* gate_stage, int32_t* stage_loc, int32_t* stage_clusters, int max_stages,
                                int* n_stages);

/* ------------------------------------------------------------------ batches
 * Many independent circuits in one persistent launch (complex64 states).
 * Every circuit is scheduled as by qsim_run_circuit (greedy clusters of at
 * most opts->kmax <= 6 qubits, Sec. 3.6; diagonal gates fused or in
 * diagonal passes). A 6-qubit cluster is applied on fp16 matrix cores with
 * operand halves; smaller clusters are padded with identity qubits to 5
 * targets (fp32 real-split product), and each diagonal pass becomes an
 * identity 5-qubit cluster with a diagonal epilogue, so that one persistent
 * kernel applies every op. Matrices are built in float64 on the GPU. Work
 * items (one op, QSIM_OPT_BATCH_ITEM_TILES tiles of 2^11 amplitudes) are
 * taken from an atomic counter in dependency order; an item waits until
 * every earlier op of its circuit is complete. */
typedef struct qsim_batch_s* qsim_batch;

typedef struct {
    int32_t n_qubits;        /* 11 .. 30 */
    int32_t n_gates;
    const qsim_gate* gates;  /* host; read by qsim_batch_plan only */
    void* dev_amps;          /* 2^n complex64, 256-byte aligned, caller-owned, one per circuit */
} qsim_batch_circuit;

typedef struct {
    int32_t n_circuits;
    int32_t n_ops;           /* initialisations + cluster ops, all circuits */
    int32_t n_clusters;      /* cluster ops (padded clusters and diagonal passes) */
    int32_t n_items;         /* work items of the persistent launch */
    int32_t grid;            /* work-groups of the last run */
    int32_t n_gates_applied; /* after the skips of opts */
    double plan_ms;          /* host time of qsim_batch_plan */
    double run_ms;           /* host wall time of the last qsim_batch_run */
    size_t workspace_bytes;
} qsim_batch_stats;

/* Schedule and pack n_circuits circuits (host only; no GPU work). opts:
 * kmax in [1, 6], scheduler GREEDY, ANALYTIC or LEARNED (PER_GATE is
 * QSIM_E_UNSUPPORTED), fuse_diag, skip_trailing_diag, skip_initial_h.
 * *workspace_bytes receives the device workspace qsim_batch_run needs. The
 * circuit descriptors' amplitude pointers are kept; the gate lists are not. */
qsim_status qsim_batch_plan(const qsim_batch_circuit* circuits, int n_circuits, const qsim_run_opts* opts,
                            qsim_batch* out, size_t* workspace_bytes);

/* Run a planned batch: initialise every state, apply every op, then wait
 * for the stream (synchronous). dev_workspace: >= the planned bytes,
 * 256-byte aligned, caller-owned; its contents are overwritten.
 * wait_limit_us: longest time (device wall clock, microseconds) a work-group
 * waits for an earlier op of its circuit (0 = 10 s); a wait that gives up
 * sets an error flag, the launch still runs to its end, and the call returns
 * QSIM_E_DEVICE (the states are then undefined). Runs of batches sharing
 * states or a workspace must not overlap. stats (nullable) is filled. */
qsim_status qsim_batch_run(qsim_batch b, void* dev_workspace, size_t ws_bytes, void* hip_stream,
                           uint32_t wait_limit_us, qsim_batch_stats* stats);
qsim_status qsim_batch_destroy(qsim_batch b);

#ifdef __cplusplus
}
#endif
#endif /* QSIM_H */
