// Internal declarations of the qsim library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qsim {

constexpr int kMaxK = 7;     // largest cluster (7: complex64 on the fp16-halves kernel only)
constexpr int kMaxGateQ = 6; // widest single gate (a dense matrix)
constexpr int kEpiMax = 64;  // entries of each list of a diagonal descriptor

// Named 2x2 gate matrices, row-major, (re, im) interleaved. Sec. 2 prints H,
// T, X^1/2, Y^1/2 and X; Y and Z are the Pauli matrices; the *_DG entries are
// conjugate transposes; PHASE is diag(1, e^{i theta}).
__host__ __device__ inline void gate2x2(int kind, double theta, double m[8]) {
    const double r = 0.70710678118654752440;  // 1/sqrt(2) = cos(pi/4) = sin(pi/4)
    for (int i = 0; i < 8; ++i) m[i] = 0.0;
    switch (kind) {
        case 0:  // H
            m[0] = r; m[2] = r; m[4] = r; m[6] = -r; break;
        case 1:  // T
            m[0] = 1; m[6] = r; m[7] = r; break;
        case 2:  // X^1/2
            m[0] = .5; m[1] = .5; m[2] = .5; m[3] = -.5; m[4] = .5; m[5] = -.5; m[6] = .5; m[7] = .5; break;
        case 3:  // Y^1/2
            m[0] = .5; m[1] = .5; m[2] = -.5; m[3] = -.5; m[4] = .5; m[5] = .5; m[6] = .5; m[7] = .5; break;
        case 4:  // X
            m[2] = 1; m[4] = 1; break;
        case 5:  // Y
            m[3] = -1; m[5] = 1; break;
        case 6:  // Z
            m[0] = 1; m[6] = -1; break;
        case 8:  // T^dagger
            m[0] = 1; m[6] = r; m[7] = -r; break;
        case 9:  // (X^1/2)^dagger
            m[0] = .5; m[1] = -.5; m[2] = .5; m[3] = .5; m[4] = .5; m[5] = .5; m[6] = .5; m[7] = -.5; break;
        case 10:  // (Y^1/2)^dagger
            m[0] = .5; m[1] = -.5; m[2] = .5; m[3] = -.5; m[4] = -.5; m[5] = .5; m[6] = .5; m[7] = -.5; break;
        case 11:  // PHASE
            m[0] = 1; m[6] = cos(theta); m[7] = sin(theta); break;
        default:
            break;
    }
}

// Gate kinds (values of qsim_gate_kind).
enum : int32_t {
    G_H = 0, G_T = 1, G_SX = 2, G_SY = 3, G_X = 4, G_Y = 5, G_Z = 6, G_CZ = 7,
    G_TDG = 8, G_SXDG = 9, G_SYDG = 10, G_PHASE = 11, G_DENSE = 12
};

__host__ __device__ inline bool gate_is_diagonal(int kind) {
    return kind == G_T || kind == G_Z || kind == G_CZ || kind == G_TDG || kind == G_PHASE;
}

// Phase e^{i theta} a diagonal single-qubit gate puts on |1>.
__host__ __device__ inline double gate_phase_angle(int kind, double theta) {
    const double pi = 3.14159265358979323846;
    switch (kind) {
        case G_T: return pi / 4;
        case G_TDG: return -pi / 4;
        case G_Z: return pi;
        case G_PHASE: return theta;
        default: return 0.0;
    }
}

// Diagonal factors of a state index, split by which bits they read:
//   cc   : CZ pairs whose two qubits are both outside the target set
//   mix  : CZ pairs with one qubit among the targets: (bit j of the target
//          index x, state bit b)
//   ph   : phase gates on qubits outside the target set (cos, sin)
// Terms that read target bits only are folded into the cluster matrix. A
// standalone diagonal pass lists all its pairs in cc and phases in ph.
struct EpiDesc {
    int32_t n_cc, n_mix, n_ph, pad;
    int32_t cc[kEpiMax][2];
    int32_t mix[kEpiMax][2];
    int32_t ph_q[kEpiMax];
    double ph[kEpiMax][2];
};

// Cluster-matrix build: one op per work-group of the builder kernel.
struct BuildGate {
    int32_t kind;
    int32_t nq;
    int32_t pos[6];     // positions inside the cluster's sorted qubit list
    int32_t dense_off;  // DENSE: offset (in doubles) of its matrix in the dense pool
    int32_t pad;
    double theta;
};

enum : int32_t {
    LAYOUT_PLAIN = 0,     // complex matrix M[y][x] (T re, T im), for the VALU kernel
    LAYOUT_MFMA32F = 1,   // real-split, permuted for v_mfma_f32_32x32x2_f32
    LAYOUT_MFMA16D = 2,   // real-split, permuted for v_mfma_f64_16x16x4_f64
    LAYOUT_GAUSS32F = 3,  // k = 6 float: Re M, Im M, Re M + Im M (three-product complex matrix)
    LAYOUT_SPLIT16F = 4,  // k = 6 float: fp16 hi / lo halves of 16 x the real-split matrix
    LAYOUT_SPLIT7 = 5     // k = 7 float: fp16 hi / lo halves of 16 x Re M and 16 x Im M
};

// A 7-qubit matrix is built by kBuildParts7 work-groups, each owning 32 of
// its 128 columns (part p: columns 32 p .. 32 p + 31); smaller ones by one.
constexpr int kBuildParts7 = 4;
struct BuildOp {
    int32_t k;
    int32_t n_gates;
    int32_t gate0;      // first BuildGate of this op
    int32_t layout;
    int32_t is_double;  // element type of the output
    int32_t part;       // k = 7: which quarter of the columns this work-group builds
    int64_t out_off;    // byte offset of the output inside the matrix region
};

// Geometry of one cluster application.
struct ClusterGeom {
    int32_t t[kMaxK];   // sorted target qubits
    int32_t n;          // qubits of the state
    int32_t k;
    uint64_t ncols;     // 2^(n-k)
};

// Geometry of the LDS-staged cluster kernels. A wave tile is the set of
// amplitudes whose "tile bits" (the k targets and the C lowest non-target
// bits, the columns) vary while all other bits are fixed; tau is the index of
// an amplitude inside its tile (the tile bits in ascending order). The tile is
// read and written as linear runs of tau (coalesced) and re-ordered through LDS.
struct StageGeom {
    int32_t nt;          // tile bits (k + C)
    int32_t tb[16];      // their state-bit positions, ascending
    int32_t tpos[6];     // tau bit of target m
    int32_t cpos[6];     // tau bit of column bit b
    int32_t swz[6];      // 6-qubit staged loop: LDS slot of tau = tau ^ (XOR of swz[i] over set bits 5 + i)
    uint64_t ioff[32];   // state offset of linear chunk i (tau = i << lane_bits ...)
};

// Batched persistent launch: every op is a 6-qubit float cluster (fp16 matrix
// halves, staged half tiles), a 5-qubit one (smaller clusters padded with
// identity qubits; fp32 real-split, staged tiles), or the initialisation of a
// state. Device pointers are filled in at run time.
struct BatchOp {
    float2* psi;           // the circuit's state
    const float* A;        // permuted real-split matrix (clusters)
    const EpiDesc* epi;    // diagonal epilogue or null
    StageGeom sg;          // tile geometry (clusters)
    uint64_t tiles;        // wave tiles of 2^11 amplitudes
    int32_t kind;          // 0 5-qubit cluster, 1 |0..0>, 2 uniform, 3 6-qubit cluster,
                           // 4 uniform start with the first cluster (write-only; A: plain complex128)
    int32_t circuit;
    int32_t lowt;          // target 0 is a cluster qubit
    int32_t n;             // qubits of the state
    uint32_t dep;          // items of this circuit that must be complete first
    uint32_t k;            // kind 4: the cluster's targets (5 or 6)
};
struct BatchItem {
    uint32_t op;
    uint32_t tile0;        // tiles [tile0, tile0 + item_tiles) of the op
};
extern int g_batch_grid;        // work-groups of the batch launch, 0 = one per CU (its occupancy)
extern int g_batch_pad;         // padding qubits: 0 lowest outside the cluster, 1 highest
extern int g_batch_item_tiles;  // tiles of 2^11 amplitudes per work item
extern int g_k6_kernel;         // float k = 6 clusters: 0 fp32 real-split, 1 fp32 three-product, 2 fp16 halves
extern int g_fold_init;         // fold the uniform initialisation into the first cluster
extern int g_pair;              // apply consecutive clusters of <= 5 qubits (complex64) two per pass
extern int g_pair_tile;         // tile bits of the pair kernel: 11 (8 waves) or 10 (12 waves)
extern int g_cluster_sets;  // scheduler: candidate qubit sets on (1) or off (0)
extern int g_batch_order;   // batch ticket order: 0 level order (default), 1 critical path first

// Bytes of a cluster matrix in each layout.
inline int64_t matrix_bytes(int k, int layout, bool dbl) {
    const int64_t d = int64_t(1) << k;
    const int64_t es = dbl ? 8 : 4;
    if (layout == LAYOUT_PLAIN) return d * d * 2 * es;
    if (layout == LAYOUT_GAUSS32F) return 3 * d * d * es;
    if (layout == LAYOUT_SPLIT16F) return 2 * (2 * d) * (2 * d) * 2;
    if (layout == LAYOUT_SPLIT7) return 4 * d * d * 2;
    return (2 * d) * (2 * d) * es;
}

// Largest cluster a state can take: 7 qubits on complex64 states of at least
// 12 qubits (a wave tile is 32 columns of 2^7 amplitudes) while 6-qubit
// clusters use the fp16-halves kernel; 6 otherwise.
inline int max_cluster_k(bool dbl, int n) { return (!dbl && g_k6_kernel == 2 && n >= 12) ? 7 : 6; }

// ------------------------------------------------------------ launchers
// All launchers enqueue on `st` and return hipSuccess or the launch error.
hipError_t launch_init(void* psi, int n, bool dbl, int mode, hipStream_t st);
// m (1 or 2) five-qubit clusters on a complex64 state of n >= 11 qubits in one
// pass, in order; targets sorted; matrices in LAYOUT_SPLIT16F (k = 5).
hipError_t launch_multi(void* psi, int n, int m, const int32_t (*targets)[5], const void* const* mats,
                        const EpiDesc* const* epis, hipStream_t st);
// The uniform start, a first cluster (g1: plain complex128 matrix mat1) with
// its epilogue expressed relative to the second cluster's targets (epi1), and
// a second cluster of 6 or 7 qubits (g2, its own epilogue epi2; the first has
// at most as many), in one write-only pass over a complex64 state of n >= 11
// (k2 = 6) or 12 (k2 = 7) qubits. omask < 0 (k2 = 6 only): mat2 in
// LAYOUT_SPLIT16F, the second cluster multiplied per column on the matrix
// cores. Otherwise mat2 is plain complex128, omask marks the second cluster's
// target bits that are also the first cluster's (at most 2) and rmask those
// epi1's mixed terms sign-flip; the second cluster's outputs for every
// (pattern of the omask rows, sign mask over the rmask rows) are first put in
// `table` (2^(|omask| + |rmask|) <= kFoldTabRows rows of 64 complex64, or
// kFoldTab7Rows rows of 128 for k2 = 7) and the pass combines them per column.
constexpr int kFoldTabRows = 128;
constexpr int kFoldTab7Rows = 64;  // with a 7-qubit second cluster: rows of 128 outputs
hipError_t launch_fold2(void* psi, const ClusterGeom& g2, const void* mat2, const EpiDesc* epi2, const EpiDesc* epi1,
                        const ClusterGeom& g1, const void* mat1, int omask, int rmask, void* table,
                        hipStream_t st);
// The uniform state followed by one cluster (matrix: plain complex128 layout)
// and its diagonal epilogue, written in one pass.
hipError_t launch_init_cluster(void* psi, bool dbl, const ClusterGeom& g, const void* mat, const EpiDesc* epi,
                               hipStream_t st);
hipError_t launch_build(const BuildOp* ops, int n_ops, const BuildGate* gates, const double* dense,
                        char* mat_base, hipStream_t st);
// Variant of the cluster kernel chosen for (dtype, k, n, targets).
int cluster_layout(bool dbl, int k, int n);
// variant (matrix-core layouts, k <= 5): 0 = direct register gather, 1 = LDS-staged.
// stats_part: also sum p, p^2 and -p ln p of the stored amplitudes into
// stats_part (per work-group, 8 doubles each; *stats_blocks receives their
// number); the direct float matrix-core kernels (k = 4..7) and the staged
// vector-ALU kernel (float, k = 2, 3) do this, other cases return
// hipErrorInvalidValue.
hipError_t launch_cluster(void* psi, bool dbl, const ClusterGeom& g, const void* mat, int layout,
                          const EpiDesc* epi, int variant, hipStream_t st, double* stats_part = nullptr,
                          unsigned* stats_blocks = nullptr);
// Can a cluster launch also produce the sums (see launch_cluster)?
inline bool cluster_stats_supported(bool dbl, int n, int k, int layout, int variant) {
    return !dbl && variant == 0 &&
           ((layout == LAYOUT_SPLIT7 && k == 7) || (layout == LAYOUT_SPLIT16F && k == 6) ||
            (layout == LAYOUT_MFMA32F && k >= 4) || (layout == LAYOUT_PLAIN && (k == 2 || k == 3) && n - k >= 6));
}
// Kernel variant of the matrix-core cluster path: 0 = direct register
// gather, 1 = LDS-staged linear loads. Chosen per (dtype, k, low_class) from a
// process-wide tune table; a forced variant (>= 0) overrides the table.
// Class of a target set for the variant choice: how many targets sit on the
// lowest 6 state bits (0 | 1 | 2 | 3 or more): those bits would otherwise be
// the contiguous column bits of a direct gather.
constexpr int kLowClasses = 4;
inline int low_class(const int32_t* t, int k) {
    int c = 0;
    for (int j = 0; j < k; ++j) c += t[j] < 6;
    return c < 3 ? c : 3;
}
void set_cluster_variant(int v);  // -1 = use the tune table
int get_cluster_variant();
void set_tune_entry(bool dbl, int k, int cls, int variant);
int get_tune_entry(bool dbl, int k, int cls);
int cluster_variant_for(bool dbl, const ClusterGeom& g, int layout);
// The op can run with either matrix-core kernel variant (direct or staged).
inline bool variant_choice(bool dbl, int k, int layout) {
    return layout != LAYOUT_PLAIN && (k <= 5 || (!dbl && layout == LAYOUT_SPLIT16F));
}
int get_cluster_variant();
// Learned cost model: features of an op (variant_override >= 0 replaces the
// kernel variant the library would pick, where the op has both).
void op_features(int n, bool dbl, int k, const int* q, int n_epi, float* f, int variant_override);
hipError_t launch_diag(void* psi, bool dbl, int n, const EpiDesc* epi, hipStream_t st);
StageGeom make_stage_geom(const ClusterGeom& g, int C, int unit);
hipError_t launch_batch(const BatchOp* ops, const BatchItem* items, uint32_t n_items, uint32_t* counters,
                        uint32_t n_circuits, uint32_t item_tiles, uint64_t wait_ticks, unsigned grid,
                        hipStream_t st);
hipError_t launch_gate1q(void* psi, bool dbl, int n, int q, const double m[8], hipStream_t st);
hipError_t launch_phase1q(void* psi, bool dbl, int n, int q, double cs, double sn, hipStream_t st);
hipError_t launch_cz(void* psi, bool dbl, int n, int a, int b, hipStream_t st);
// Bit permutation of the amplitude index (a relabelling of bit locations,
// Sec. 3.4's local swap). Tiles are the 2^nt amplitudes whose tile bits
// tb[0..nt) (ascending state bit positions) vary; tau is the index inside a
// tile (bit j of tau at state bit tb[j]). The amplitude at tile index tau
// moves to the tile index whose bit to[j] is bit j of tau.
constexpr int kPermMaxBits = 12;
struct PermGeom {
    int32_t nt;
    int32_t tb[kPermMaxBits];
    int32_t to[kPermMaxBits];
};
hipError_t launch_permute(void* psi, bool dbl, int n, const PermGeom& pg, hipStream_t st);

// Reductions: partial sums go to `part` (kReduceBlocks * 8 doubles), the
// final values to `res` (4 doubles).
constexpr int kReduceBlocks = 2048;
hipError_t launch_stats(const void* psi, bool dbl, int n, void* probs, bool probs_dbl, double* part,
                        double* res, hipStream_t st);
// Final reduction of per-work-group sums written by a cluster launch (stats_part).
hipError_t launch_reduce_stats(const double* part, unsigned nblocks, double* res, hipStream_t st);
hipError_t launch_compare(const void* psi, bool dbl, int n, const void* ref, bool ref_dbl,
                          double* part, double* res, hipStream_t st);

}  // namespace qsim
