// GPU kernels of the state-vector simulator (gfx950 / MI355X).
//
// State: 2^n interleaved complex amplitudes (float2 or double2), amplitude
// index i = sum_q b_q 2^q (Haener & Steiger, Sec. 2).
//
// Cluster kernels apply one dense k-qubit gate in place (Sec. 3.2): with the
// targets sorted (t_0 < ... < t_{k-1}), a "column" c is an assignment of the
// n-k other bits, deposited into the non-target positions; the 2^k amplitudes
// of a column are gathered, multiplied by the 2^k x 2^k matrix and scattered
// back. Consecutive columns differ in the lowest non-target bits, so a wave's
// columns are contiguous runs of memory.
//
// For k >= 4 (float) / k >= 3 (double) the product is a real GEMM on the
// matrix cores: with the state's (re, im) interleaving the complex matrix
// becomes the real 2^(k+1) x 2^(k+1) matrix [[Re m, -Im m], [Im m, Re m]] per
// entry - the (m_R, m_R) / (-m_I, m_I) pairing of Sec. 3.2, Eqs. (1)-(3) -
// and one MFMA block multiplies it by 32 (float) or 16 (double) columns. The
// rows and inner index of that matrix are permuted once, when it is built,
// so that every lane's MFMA operands and results are exactly the amplitudes
// it loads and stores: lane (p, h) of a float wave owns the amplitudes whose
// highest target bit is h in column p, with no LDS round trip for the state.
#include "qsim_internal.h"

#include <cmath>
#include <cstring>
#include <type_traits>

namespace qsim {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };

// Insert a zero bit at position t.
__device__ __forceinline__ uint64_t insert_zero(uint64_t c, int t) {
    const uint64_t low = (uint64_t(1) << t) - 1;
    return ((c & ~low) << 1) | (c & low);
}

// Deposit column index c into the non-target bit positions.
template <int K>
__device__ __forceinline__ uint64_t deposit_cols(uint64_t c, const ClusterGeom& g) {
#pragma unroll
    for (int j = 0; j < K; ++j) c = insert_zero(c, g.t[j]);
    return c;
}

// Offset of target index x: bit j of x at state bit t[j], j < NB.
template <int NB>
__device__ __forceinline__ uint64_t target_off(int x, const ClusterGeom& g) {
    uint64_t o = 0;
#pragma unroll
    for (int j = 0; j < NB; ++j)
        if ((x >> j) & 1) o |= uint64_t(1) << g.t[j];
    return o;
}

// ------------------------------------------------------------ diagonal factors
// Factor of the diagonal gates that depends on the non-target bits of a
// column (sign parity, sign mask over target bits, complex phase).
template <typename T>
struct ColFactor {
    uint32_t sgn, w;
    T cr, ci;
};

template <typename T, typename E>
__device__ __forceinline__ ColFactor<T> col_factor(E* __restrict__ e, uint64_t base) {
    ColFactor<T> f{0u, 0u, T(1), T(0)};
    const int ncc = e->n_cc;
    for (int i = 0; i < ncc; ++i)
        f.sgn ^= (uint32_t)((base >> e->cc[i][0]) & (base >> e->cc[i][1]) & 1);
    const int nm = e->n_mix;
    for (int i = 0; i < nm; ++i) f.w ^= (uint32_t)((base >> e->mix[i][1]) & 1) << e->mix[i][0];
    const int np = e->n_ph;
    if (np) {
        double cr = 1.0, ci = 0.0;
        for (int i = 0; i < np; ++i) {
            if ((base >> e->ph_q[i]) & 1) {
                const double a = e->ph[i][0], b = e->ph[i][1];
                const double t = cr * a - ci * b;
                ci = cr * b + ci * a;
                cr = t;
            }
        }
        f.cr = (T)cr;
        f.ci = (T)ci;
    }
    return f;
}

template <typename T>
__device__ __forceinline__ void apply_factor(T& re, T& im, const ColFactor<T>& f, uint32_t y, bool ph) {
    if (ph) {
        const T r = re * f.cr - im * f.ci;
        const T i = re * f.ci + im * f.cr;
        re = r;
        im = i;
    }
    const bool neg = ((f.sgn ^ (uint32_t)__popc(y & f.w)) & 1u) != 0;
    re = neg ? -re : re;
    im = neg ? -im : im;
}

// Work-groups of a launch are dealt to the 8 XCDs round-robin (work-group b
// runs on XCD b % 8). Renumbered so that the work-groups of one XCD are
// consecutive, the tiles a persistent grid has in flight form one contiguous
// stretch per XCD (each XCD has its own L2). A bijection of the work-group
// numbers when the grid is a multiple of 8, else the identity.
__device__ __forceinline__ uint32_t xcd_block() {
    const uint32_t b = blockIdx.x, g = gridDim.x;
    return (g & 7) == 0 ? (b & 7) * (g >> 3) + (b >> 3) : b;
}

// Float64 sums of p = |a|^2 (slot 0), p^2 (slot 1) and -p ln p (slot 2) over
// float amplitudes. ln p = e ln 2 + ln m with p = m 2^e split exactly and
// ln m (m in [1/2, 1)) in float, within ~1.4e-7 absolute - far below what a
// float state resolves; a double log costs as much ALU time as reading the
// state.
__device__ __forceinline__ void stats_acc_f(double (&v)[8], float x, float y) {
    const double pr = (double)x * (double)x + (double)y * (double)y;
    v[0] += pr;
    v[1] += pr * pr;
    if (pr > 0.0) {
        int e;
        const double m = frexp(pr, &e);
        v[2] -= pr * ((double)e * 0.6931471805599453 + (double)logf((float)m));
    }
}

// Block reduction of up to 8 values into out (defined with the reductions).
__device__ void block_reduce_store(double (&vals)[8], int nv, unsigned maxmask, double* out);

// Lane l's value of x, in every lane (l uniform).
__device__ __forceinline__ double readlane_f64(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Row sums of a plain complex128 d x d matrix, times amp, into LDS: eight
// threads per row, each summing every eighth entry (so all loads are in
// flight at once), combined by shuffles within the eight. Every thread of the
// block takes part (the shuffles); the caller synchronises afterwards.
template <typename V2>
__device__ __forceinline__ void row_sums(const double2* __restrict__ M, int d, double amp, V2* out) {
    const int sub = (int)threadIdx.x & 7;
    for (int r0 = 0; r0 < d; r0 += (int)blockDim.x / 8) {
        const int r = r0 + (int)threadIdx.x / 8;
        double re = 0.0, im = 0.0;
        if (r < d)
            for (int x = sub; x < d; x += 8) {
                const double2 m = M[r * d + x];
                re += m.x;
                im += m.y;
            }
#pragma unroll
        for (int o = 4; o > 0; o >>= 1) {
            re += __shfl_xor(re, o);
            im += __shfl_xor(im, o);
        }
        if (r < d && sub == 0) {
            out[r].x = (decltype(out[r].x))(re * amp);
            out[r].y = (decltype(out[r].y))(im * amp);
        }
    }
}

typedef float vf4 __attribute__((ext_vector_type(4)));
typedef double vd2 __attribute__((ext_vector_type(2)));
// Explicitly global pointers for code that also runs on pointers read from a
// descriptor (the compiler would otherwise use flat memory instructions,
// whose outstanding loads also hold up every LDS wait).
#define QSIM_GLOBAL __attribute__((address_space(1)))
typedef QSIM_GLOBAL float2 g_float2;
typedef QSIM_GLOBAL vf4 g_vf4;
typedef const QSIM_GLOBAL EpiDesc g_epi;
// Diagonal descriptors read through the constant address space: uniform,
// read-only data the compiler then loads with scalar instructions. (Vector
// loads of them would share the vector-memory counter with a tile's prefetch,
// and waiting for them would wait for the whole prefetch.)
typedef const __attribute__((address_space(4))) EpiDesc c_epi;

// Copy a cluster matrix of N elements into LDS: 16-byte loads, all in flight
// before the first LDS store (a loop of single loads would wait for each).
template <int N, int THREADS, typename T, typename V4>
__device__ __forceinline__ void load_matrix(T* __restrict__ dst, const V4* __restrict__ src) {
    typedef vf4 v4;
    constexpr int CHUNKS = N * (int)sizeof(T) / 16;
    static_assert(N * sizeof(T) % 16 == 0, "matrix is a whole number of 16-byte chunks");
    constexpr int PER = CHUNKS / THREADS;
    constexpr int REST = CHUNKS % THREADS;
    v4 r[PER > 0 ? PER : 1];
#pragma unroll
    for (int i = 0; i < PER; ++i) r[i] = src[threadIdx.x + i * THREADS];
    v4 t{0.0f, 0.0f, 0.0f, 0.0f};
    if (REST && threadIdx.x < REST) t = src[PER * THREADS + threadIdx.x];
#pragma unroll
    for (int i = 0; i < PER; ++i) reinterpret_cast<v4*>(dst)[threadIdx.x + i * THREADS] = r[i];
    if (REST && threadIdx.x < REST) reinterpret_cast<v4*>(dst)[PER * THREADS + threadIdx.x] = t;
}

// ------------------------------------------------------------ cluster: MFMA, float
// Wave tile: all 2^K target combinations x 32*NB columns. Lane l: p = l%32,
// h = l/32 owns target indices x = j | h << (K-1), j < 2^(K-1), of its
// column(s). Without a target at bit 0 (LOWT = false) and NB = 2 a lane's two
// columns are adjacent in memory (one 16-byte load per amplitude pair); with
// t_0 = 0 (LOWT) the amplitudes j, j+1 of one column are adjacent instead.
template <int K, int NB, bool LOWT>
struct TileF32 {
    static constexpr int HX = (1 << K) / 2;
    static constexpr int COLS = 32 * NB;

    __device__ __forceinline__ static void bases(uint64_t tile, int p, const ClusterGeom& g, uint64_t (&base)[NB]) {
        if (LOWT || NB == 1) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) base[nb] = deposit_cols<K>(tile * COLS + p + 32 * nb, g);
        } else {
            base[0] = deposit_cols<K>(tile * COLS + 2 * p, g);
            base[NB - 1] = base[0] | 1;
        }
    }
    __device__ __forceinline__ static void load(const float2* __restrict__ psi, const uint64_t (&base)[NB],
                                                uint64_t hoff, const ClusterGeom& g, float (&B)[NB][2 * HX]) {
        if (!LOWT && NB == 2) {
#pragma unroll
            for (int j = 0; j < HX; ++j) {
                const float4 v = *reinterpret_cast<const float4*>(psi + (base[0] | hoff | target_off<K - 1>(j, g)));
                B[0][2 * j] = v.x; B[0][2 * j + 1] = v.y;
                B[NB - 1][2 * j] = v.z; B[NB - 1][2 * j + 1] = v.w;
            }
        } else if (LOWT) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int j = 0; j < HX; j += 2) {
                    const float4 v =
                        *reinterpret_cast<const float4*>(psi + (base[nb] | hoff | target_off<K - 1>(j, g)));
                    B[nb][2 * j] = v.x; B[nb][2 * j + 1] = v.y;
                    B[nb][2 * j + 2] = v.z; B[nb][2 * j + 3] = v.w;
                }
        } else {
#pragma unroll
            for (int j = 0; j < HX; ++j) {
                const float2 v = psi[base[0] | hoff | target_off<K - 1>(j, g)];
                B[0][2 * j] = v.x; B[0][2 * j + 1] = v.y;
            }
        }
    }
    __device__ __forceinline__ static void store(float2* __restrict__ psi, const uint64_t (&base)[NB], uint64_t hoff,
                                                 const ClusterGeom& g, const float (&O)[NB][2 * HX]) {
        if (!LOWT && NB == 2) {
#pragma unroll
            for (int j = 0; j < HX; ++j)
                *reinterpret_cast<float4*>(psi + (base[0] | hoff | target_off<K - 1>(j, g))) =
                    make_float4(O[0][2 * j], O[0][2 * j + 1], O[NB - 1][2 * j], O[NB - 1][2 * j + 1]);
        } else if (LOWT) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int j = 0; j < HX; j += 2)
                    *reinterpret_cast<float4*>(psi + (base[nb] | hoff | target_off<K - 1>(j, g))) =
                        make_float4(O[nb][2 * j], O[nb][2 * j + 1], O[nb][2 * j + 2], O[nb][2 * j + 3]);
        } else {
#pragma unroll
            for (int j = 0; j < HX; ++j)
                psi[base[0] | hoff | target_off<K - 1>(j, g)] = make_float2(O[0][2 * j], O[0][2 * j + 1]);
        }
    }
};

// Persistent: each wave walks tiles with a stride of the whole grid and
// prefetches the next tile's amplitudes into registers before it runs the
// current tile's MFMA chain, so loads stay in flight under the matrix work.
//
// STATS: the launch is the last op of a run; the kernel also sums p = |a|^2,
// p^2 and -p ln p of the amplitudes it stores (float64, per work-group into
// part[blockIdx.x * 8 + 0..2]), so the state need not be read again for them.
template <int K, int NB, bool LOWT, bool STATS = false>
__global__ __launch_bounds__(256, 2) void k_cluster_f32_mfma(float2* __restrict__ psi,
                                                             const float* __restrict__ Ap,
                                                             const EpiDesc* __restrict__ epi,
                                                             ClusterGeom g, double* __restrict__ part) {
    using T = TileF32<K, NB, LOWT>;
    constexpr int D = 1 << K;
    constexpr int HX = D / 2;       // amplitudes per lane and column
    constexpr int RB = 2 * D / 32;  // 32-row blocks of the real-split matrix
    constexpr int S = D;            // MFMA steps (inner dimension 2^(K+1), 2 per step)
    __shared__ float As[RB * S * 64];
    load_matrix<RB * S * 64, 256>(As, reinterpret_cast<const vf4*>(Ap));
    __syncthreads();

    const int lane = threadIdx.x & 63, p = lane & 31, h = lane >> 5;
    const uint64_t hoff = h ? (uint64_t(1) << g.t[K - 1]) : 0;
    const uint64_t ntiles = g.ncols / T::COLS;
    const uint64_t stride = (uint64_t)gridDim.x * 4;
    const bool has_epi = epi != nullptr;
    const bool has_ph = has_epi && epi->n_ph > 0;

    // The prefetch is unconditional (the last tile is re-read instead of
    // reading past the end) so the load count per iteration is fixed and the
    // waits the compiler places for the amplitudes cover only their own loads.
    uint64_t tile = (uint64_t)xcd_block() * 4 + (threadIdx.x >> 6);
    double sv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (tile >= ntiles) {  // uniform in the wave: every wave reaches one reduction
        if constexpr (STATS) block_reduce_store(sv, 3, 0u, part + blockIdx.x * 8);
        return;
    }
    const uint64_t last = ntiles - 1;
    float B[NB][2 * HX];
    uint64_t base[NB];
    T::bases(tile, p, g, base);
    T::load(psi, base, hoff, g, B);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_sched_barrier(0);
    do {
        const uint64_t nxt = tile + stride < last ? tile + stride : last;
        float Bn[NB][2 * HX];
        uint64_t basen[NB];
        T::bases(nxt, p, g, basen);
        T::load(psi, basen, hoff, g, Bn);
        __builtin_amdgcn_sched_barrier(0);

        floatx16 acc[NB][RB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[nb][rb][i] = 0.0f;
        int aoff = lane;
        asm volatile("" : "+v"(aoff));  // keep the matrix reads inside the loop (not in registers)
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const float a = As[(rb * S + s) * 64 + aoff];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[nb][rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, B[nb][s], acc[nb][rb], 0, 0, 0);
            }
        }
        // acc[nb][j / 8][2 (j % 8) + {0, 1}] is output amplitude j of the lane
        float O[NB][2 * HX];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int j = 0; j < 2 * HX; ++j) O[nb][j] = acc[nb][j / 16][j % 16];
        if (has_epi) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const ColFactor<float> f = col_factor<float>(epi, base[nb]);
#pragma unroll
                for (int j = 0; j < HX; ++j)
                    apply_factor(O[nb][2 * j], O[nb][2 * j + 1], f, (uint32_t)(j | (h << (K - 1))), has_ph);
            }
        }
        if constexpr (STATS) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int j = 0; j < HX; ++j) stats_acc_f(sv, O[nb][2 * j], O[nb][2 * j + 1]);
        }
        T::store(psi, base, hoff, g, O);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            base[nb] = basen[nb];
#pragma unroll
            for (int j = 0; j < 2 * HX; ++j) B[nb][j] = Bn[nb][j];
        }
        tile += stride;
    } while (tile < ntiles);
    if constexpr (STATS) block_reduce_store(sv, 3, 0u, part + blockIdx.x * 8);
}

// ------------------------------------------------------------ cluster: MFMA, float, k = 6
// Three-multiplication complex product: with M = Mr + i Mi and x = xr + i xi,
//   Re(M x) = Mr xr - Mi xi,   Im(M x) = (Mr + Mi)(xr + xi) - Mr xr - Mi xi,
// three real 64 x 64 products instead of the four blocks of the real-split
// matrix: 25% fewer matrix-core operations, which is what bounds k = 6.
// v_mfma_f32_16x16x4_f32: operand lane l holds row / column l % 16 at inner
// index l / 16; result register r of lane l holds row 4 (l / 16) + r. Wave
// tile: 16 columns; lane (p, q) = (l % 16, l / 16) owns amplitudes j | q << 4,
// j < 16, of column p. At step s the lane supplies inner index s | q << 4,
// its own amplitude j = s; result register r of row block rb lands on its
// amplitude (4 rb + r) | q << 4 (the builder permutes the matrix rows so).
template <bool LOWT>
__global__ __launch_bounds__(256, 2) void k_cluster_f32_gauss6(float2* __restrict__ psi,
                                                               const float* __restrict__ Ap,
                                                               const EpiDesc* __restrict__ epi,
                                                               ClusterGeom g) {
    constexpr int K = 6, HX = 16;
    __shared__ float As[3 * 4 * 16 * 64];
    load_matrix<3 * 4 * 16 * 64, 256>(As, reinterpret_cast<const vf4*>(Ap));
    __syncthreads();

    const int lane = threadIdx.x & 63, p = lane & 15, q = lane >> 4;
    const uint64_t qoff = ((q & 1) ? uint64_t(1) << g.t[4] : 0) | ((q >> 1) ? uint64_t(1) << g.t[5] : 0);
    const uint64_t ntiles = g.ncols / 16;
    const uint64_t stride = (uint64_t)gridDim.x * 4;
    const bool has_epi = epi != nullptr;
    const bool has_ph = has_epi && epi->n_ph > 0;

    uint64_t tile = (uint64_t)xcd_block() * 4 + (threadIdx.x >> 6);
    if (tile >= ntiles) return;
    const uint64_t last = ntiles - 1;
    auto load = [&](uint64_t b, float (&X)[2 * HX]) {
        if (LOWT) {
#pragma unroll
            for (int j = 0; j < HX; j += 2) {
                const float4 v = *reinterpret_cast<const float4*>(psi + (b | target_off<4>(j, g)));
                X[2 * j] = v.x; X[2 * j + 1] = v.y; X[2 * j + 2] = v.z; X[2 * j + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int j = 0; j < HX; ++j) {
                const float2 v = psi[b | target_off<4>(j, g)];
                X[2 * j] = v.x; X[2 * j + 1] = v.y;
            }
        }
    };
    uint64_t base = deposit_cols<K>(tile * 16 + p, g);
    float B[2 * HX];
    load(base | qoff, B);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_sched_barrier(0);
    do {
        const uint64_t nxt = tile + stride < last ? tile + stride : last;
        const uint64_t basen = deposit_cols<K>(nxt * 16 + p, g);
        float Bn[2 * HX];
        load(basen | qoff, Bn);
        __builtin_amdgcn_sched_barrier(0);

        ColFactor<float> f{0u, 0u, 1.0f, 0.0f};
        if (has_epi) f = col_factor<float>(epi, base);
        vf4 a1[4], a2[4], a3[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) a1[rb][i] = a2[rb][i] = a3[rb][i] = 0.0f;
        int aoff = lane;
        asm volatile("" : "+v"(aoff));  // keep the matrix reads inside the loop (not in registers)
#pragma unroll
        for (int st = 0; st < 16; ++st) {
            const float xr = B[2 * st], xi = B[2 * st + 1], xs = xr + xi;
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                a1[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(As[((0 * 4 + rb) * 16 + st) * 64 + aoff], xr, a1[rb], 0,
                                                             0, 0);
                a2[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(As[((1 * 4 + rb) * 16 + st) * 64 + aoff], xi, a2[rb], 0,
                                                             0, 0);
                a3[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(As[((2 * 4 + rb) * 16 + st) * 64 + aoff], xs, a3[rb], 0,
                                                             0, 0);
            }
        }
        // amplitude j = 4 rb + r of the lane
        float O[2 * HX];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                O[2 * (4 * rb + r)] = a1[rb][r] - a2[rb][r];
                O[2 * (4 * rb + r) + 1] = a3[rb][r] - a1[rb][r] - a2[rb][r];
            }
        if (has_epi) {
#pragma unroll
            for (int j = 0; j < HX; ++j)
                apply_factor(O[2 * j], O[2 * j + 1], f, (uint32_t)(j | (q << 4)), has_ph);
        }
        const uint64_t b0 = base | qoff;
        if (LOWT) {
#pragma unroll
            for (int j = 0; j < HX; j += 2)
                *reinterpret_cast<float4*>(psi + (b0 | target_off<4>(j, g))) =
                    make_float4(O[2 * j], O[2 * j + 1], O[2 * j + 2], O[2 * j + 3]);
        } else {
#pragma unroll
            for (int j = 0; j < HX; ++j) psi[b0 | target_off<4>(j, g)] = make_float2(O[2 * j], O[2 * j + 1]);
        }
        base = basen;
#pragma unroll
        for (int j = 0; j < 2 * HX; ++j) B[j] = Bn[j];
        tile += stride;
    } while (tile < ntiles);
}

// ------------------------------------------------------------ cluster: float state, k = 6, fp16 matrix cores
// The real-split product of a 6-qubit cluster needs 32 flop per byte of state,
// beyond what the fp32 matrix cores sustain at HBM speed. The fp16 matrix
// cores are 16 times faster, so the product runs on them with each operand
// split into two halves, v = hi + lo (hi = fp16(v), lo = fp16(v - hi)):
//   A x ~= A_hi x_hi + A_hi x_lo + A_lo x_hi,
// accumulated in fp32 (the dropped A_lo x_lo and the split residuals are
// ~2^-22 relative, the size of fp32 rounding). The matrix is stored as
// 16 M, split by the builder. Each column of the state tile is scaled by a
// power of two that puts its largest magnitude just below 2^14 (exact, and no
// fp16 overflow for any input), and its results are scaled back.
// v_mfma_f32_32x32x16_f16: operand lane l, element i holds row / column l % 32
// at inner index 8 (l / 32) + i; result register r of lane l holds row
// 8 (r / 4) + 4 (l / 32) + r % 4 (as for the fp32 32x32 instruction). Lane
// (p, h) owns amplitudes j | h << 5 of column p; at step s it supplies its
// floats 8 s .. 8 s + 7 (amplitudes 4 s .. 4 s + 3, re / im interleaved).
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

// fp16 halves of two scaled floats, packed: H = (f16(x0 sc), f16(x1 sc)),
// L = (f16(x0 sc - H.lo), f16(x1 sc - H.hi)), rounded to nearest even - the
// arithmetic of (_Float16)(x * sc) and (_Float16)(x * sc - hi), four
// mixed-precision FMAs per pair (checked bit for bit against that form; the
// compiler's own code computed the high halves twice to pack them).
__device__ __forceinline__ void split_pair_f16(float x0, float x1, float sc, uint32_t& H, uint32_t& L) {
    __asm__("v_fma_mixlo_f16 %0, %2, %4, 0\n\t"
            "v_fma_mixhi_f16 %0, %3, %4, 0\n\t"
            "v_fma_mixlo_f16 %1, %2, %4, -%0 op_sel_hi:[0,0,1]\n\t"
            "v_fma_mixhi_f16 %1, %3, %4, -%0 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
            : "=&v"(H), "=&v"(L)
            : "v"(x0), "v"(x1), "v"(sc));
}

// The fp16 halves (hi, lo) of a lane's N floats of one column, scaled by the
// power of two that puts the column's largest magnitude (over this lane and
// its partner lane, lane ^ 32) just below 2^14: exact scaling, no fp16
// overflow for any input, zero columns stay zero. Returns the exponent se
// of that scale (the results are scaled back by 2^(-se) times the matrix's
// own 2^-4). Float i of the lane is element i % 8 of xh / xl[i / 8].
template <int N>
__device__ __forceinline__ int split_halves(const float (&X)[N], half8 (&xh)[N / 8], half8 (&xl)[N / 8]) {
    float mx = 0.0f;  // |x| is a free operand modifier of the max
#pragma unroll
    for (int i = 0; i < N; ++i) mx = fmaxf(mx, fabsf(X[i]));
    const uint32_t mb = max(__float_as_uint(mx), (uint32_t)__shfl_xor((int)__float_as_uint(mx), 32));
    const int e = (int)(mb >> 23) - 126;  // largest magnitude < 2^e
    const int se = min(max(14 - e, -100), 100);
    const float sc = __builtin_ldexpf(1.0f, se);
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int st = 0; st < N / 8; ++st) {
        u32x4 h, l;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t a, b;
            split_pair_f16(X[8 * st + 2 * q], X[8 * st + 2 * q + 1], sc, a, b);
            h[q] = a;
            l[q] = b;
        }
        xh[st] = __builtin_bit_cast(half8, h);
        xl[st] = __builtin_bit_cast(half8, l);
    }
    return se;
}


// STATS: as in k_cluster_f32_mfma (sums of the stored amplitudes' p, p^2,
// -p ln p into part, per work-group).
template <bool LOWT, bool STATS = false>
__global__ __launch_bounds__(256, 2) void k_cluster_f32_split6(float2* __restrict__ psi,
                                                               const half8* __restrict__ Ap,
                                                               const EpiDesc* __restrict__ epi,
                                                               ClusterGeom g, double* __restrict__ part) {
    constexpr int K = 6, HX = 32, RB = 4, S = 8;
    using T = TileF32<K, 1, LOWT>;
    __shared__ half8 Ah[RB * S * 64];
    __shared__ half8 Al[RB * S * 64];
    load_matrix<RB * S * 64 * 8, 256>(reinterpret_cast<_Float16*>(Ah), reinterpret_cast<const vf4*>(Ap));
    load_matrix<RB * S * 64 * 8, 256>(reinterpret_cast<_Float16*>(Al),
                                      reinterpret_cast<const vf4*>(Ap + RB * S * 64));
    __syncthreads();

    const int lane = threadIdx.x & 63, p = lane & 31, h = lane >> 5;
    const uint64_t hoff = h ? (uint64_t(1) << g.t[K - 1]) : 0;
    const uint64_t ntiles = g.ncols / 32;
    const uint64_t stride = (uint64_t)gridDim.x * 4;
    const bool has_epi = epi != nullptr;
    const bool has_ph = has_epi && epi->n_ph > 0;

    uint64_t tile = (uint64_t)xcd_block() * 4 + (threadIdx.x >> 6);
    double sv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (tile >= ntiles) {  // uniform in the wave: every wave reaches one reduction
        if constexpr (STATS) block_reduce_store(sv, 3, 0u, part + blockIdx.x * 8);
        return;
    }
    const uint64_t last = ntiles - 1;

    // split the column's amplitudes (scaled) into fp16 halves; returns the
    // factor that undoes the column and matrix scaling
    auto split = [&](const float (&X)[2 * HX], half8 (&xh)[S], half8 (&xl)[S]) -> float {
        return __builtin_ldexpf(1.0f, -split_halves<2 * HX>(X, xh, xl) - 4);
    };

    float B[1][2 * HX];
    uint64_t base[1];
    T::bases(tile, p, g, base);
    T::load(psi, base, hoff, g, B);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_sched_barrier(0);
    half8 xh[S], xl[S];
    float unscale = split(B[0], xh, xl);
    do {
        const uint64_t nxt = tile + stride < last ? tile + stride : last;
        float Bn[1][2 * HX];
        uint64_t basen[1];
        T::bases(nxt, p, g, basen);
        T::load(psi, basen, hoff, g, Bn);
        __builtin_amdgcn_sched_barrier(0);

        floatx16 acc[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[rb][i] = 0.0f;
        int aoff = lane;
        asm volatile("" : "+v"(aoff));  // keep the matrix reads inside the loop (not in registers)
#pragma unroll
        for (int st = 0; st < S; ++st) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const half8 ah = Ah[(rb * S + st) * 64 + aoff];
                const half8 al = Al[(rb * S + st) * 64 + aoff];
                acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, xl[st], acc[rb], 0, 0, 0);
                acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, xh[st], acc[rb], 0, 0, 0);
                acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, xh[st], acc[rb], 0, 0, 0);
            }
        }
        float O[1][2 * HX];
#pragma unroll
        for (int j = 0; j < 2 * HX; ++j) O[0][j] = acc[j / 16][j % 16] * unscale;
        if (has_epi) {
            const ColFactor<float> f = col_factor<float>(epi, base[0]);
#pragma unroll
            for (int j = 0; j < HX; ++j)
                apply_factor(O[0][2 * j], O[0][2 * j + 1], f, (uint32_t)(j | (h << (K - 1))), has_ph);
        }
        if constexpr (STATS) {
#pragma unroll
            for (int j = 0; j < HX; ++j) stats_acc_f(sv, O[0][2 * j], O[0][2 * j + 1]);
        }
        T::store(psi, base, hoff, g, O);
        base[0] = basen[0];
        unscale = split(Bn[0], xh, xl);
        tile += stride;
    } while (tile < ntiles);
    if constexpr (STATS) block_reduce_store(sv, 3, 0u, part + blockIdx.x * 8);
}

// A column's diagonal-epilogue factor (col_factor), split for a wave that
// walks many tiles: terms on the state bits above the tile (uniform in the
// wave, new each tile) and terms on the column bits (fixed per lane) are
// separate, and a CZ pair with one qubit of each kind is a mask over the
// column index, set per tile. Target bits take no part (the host moved such
// terms into the matrix or the mask over rows).
// Tile part of base (tile bits zero) for a K-qubit cluster: bit 0 the sign,
// bits 1..K the mask over rows, the 5 bits above them the mask over the
// column index; the phase in (cr, ci).
template <int K = 6>
__device__ __forceinline__ uint32_t epi_tile_part(c_epi* __restrict__ e, uint64_t base, uint64_t colmask,
                                                  double& cr, double& ci) {
    uint32_t sgn = 0, w = 0, cross = 0;
    const int ncc = e->n_cc;
    for (int i = 0; i < ncc; ++i) {
        const int a = e->cc[i][0], b = e->cc[i][1];
        const bool ca = (colmask >> a) & 1, cb = (colmask >> b) & 1;
        if (!ca && !cb)
            sgn ^= (uint32_t)((base >> a) & (base >> b) & 1);
        else if (ca && !cb)
            cross ^= (uint32_t)((base >> b) & 1) << __popcll(colmask & ((uint64_t(1) << a) - 1));
        else if (!ca && cb)
            cross ^= (uint32_t)((base >> a) & 1) << __popcll(colmask & ((uint64_t(1) << b) - 1));
    }
    const int nm = e->n_mix;
    for (int i = 0; i < nm; ++i) {
        const int b = e->mix[i][1];
        if (!((colmask >> b) & 1)) w ^= (uint32_t)((base >> b) & 1) << e->mix[i][0];
    }
    cr = 1.0;
    ci = 0.0;
    const int np = e->n_ph;
    for (int i = 0; i < np; ++i) {
        const int q = e->ph_q[i];
        if (!((colmask >> q) & 1) && ((base >> q) & 1)) {
            const double a = e->ph[i][0], b = e->ph[i][1];
            const double t = cr * a - ci * b;
            ci = cr * b + ci * a;
            cr = t;
        }
    }
    return sgn | (w << 1) | (cross << (K + 1));
}

// Column part of the same factor (cbits: the column's state bits).
__device__ __forceinline__ void epi_lane_part(c_epi* __restrict__ e, uint64_t cbits, uint64_t colmask, uint32_t& sgn,
                                              uint32_t& w, double& cr, double& ci) {
    sgn = 0;
    w = 0;
    const int ncc = e->n_cc;
    for (int i = 0; i < ncc; ++i) {
        const int a = e->cc[i][0], b = e->cc[i][1];
        if (((colmask >> a) & 1) && ((colmask >> b) & 1)) sgn ^= (uint32_t)((cbits >> a) & (cbits >> b) & 1);
    }
    const int nm = e->n_mix;
    for (int i = 0; i < nm; ++i) {
        const int b = e->mix[i][1];
        if ((colmask >> b) & 1) w ^= (uint32_t)((cbits >> b) & 1) << e->mix[i][0];
    }
    cr = 1.0;
    ci = 0.0;
    const int np = e->n_ph;
    for (int i = 0; i < np; ++i) {
        const int q = e->ph_q[i];
        if (((colmask >> q) & 1) && ((cbits >> q) & 1)) {
            const double a = e->ph[i][0], b = e->ph[i][1];
            const double t = cr * a - ci * b;
            ci = cr * b + ci * a;
            cr = t;
        }
    }
}

// Combine the two parts for column index p (tile part read from its lane).
template <int K = 6>
__device__ __forceinline__ ColFactor<float> epi_combine(uint32_t tb, double tr, double ti, uint32_t ls, uint32_t lw,
                                                        double lr, double li, int p) {
    ColFactor<float> f;
    f.sgn = ls ^ (tb & 1u) ^ ((uint32_t)__popc((uint32_t)p & (tb >> (K + 1)) & 31u) & 1u);
    f.w = lw ^ ((tb >> 1) & ((1u << K) - 1u));
    f.cr = (float)(tr * lr - ti * li);
    f.ci = (float)(tr * li + ti * lr);
    return f;
}

// Swap a (in the odd 16-lane rows of the wave) with b (in the even rows):
// afterwards lane l of an even row holds in b what lane l + 16 held in a, and
// lane l + 16 holds in a what lane l held in b.
__device__ __forceinline__ void lane_swap16(float& a, float& b) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}

// ------------------------------------------------------------ cluster: float state, k = 7, fp16 matrix cores
// A 7-qubit cluster doubles the matrix work per byte of state of a 6-qubit
// one and still stays below the HBM time on the fp16 matrix cores, so it
// takes the same operand halves (A x ~= A_hi x_hi + A_hi x_lo + A_lo x_hi,
// fp32 accumulation). Its real-split matrix (2^8 x 2^8 entries) would not fit
// in LDS, so the complex product is written with the real and imaginary
// parts of M instead (Sec. 3.2, Eqs. (1)-(3)):
//   Re y = Re M Re x - Im M Im x,   Im y = Im M Re x + Re M Im x,
// four real products on two matrices (their halves: 128 KiB of LDS; the
// minus sign goes onto the halves of Im x, an exact sign flip). One
// work-group of 4 waves per compute unit.
// Wave tile: 32 columns x 2^7 targets. Lane l: p = l % 32 (column), h = l / 32
// owns the amplitudes j | h << 6 (j < 64) of its column, for its loads and
// its stores. v_mfma_f32_32x32x16_f16: at step s the lane supplies the halves
// of its amplitudes j = 8 s .. 8 s + 7 (inner index 16 s + 8 h + i <->
// amplitude (8 s + i) | h << 6); result register r of row block rb holds its
// amplitude j = 16 rb + r (physical row 8 (r / 4) + 4 h + r % 4). The builder
// permutes M once to match (LAYOUT_SPLIT7).
template <bool LOWT, bool STATS = false>
__global__ __launch_bounds__(256, 1) void k_cluster_f32_split7(float2* __restrict__ psi,
                                                               const half8* __restrict__ Ap,
                                                               const EpiDesc* __restrict__ epi,
                                                               ClusterGeom g, double* __restrict__ part) {
    constexpr int K = 7, HX = 64, RB = 4, S = 8, NP = RB * S * 64;
    // parts: 16 Re M hi, lo, 16 Im M hi, lo; entry (rb, s, lane) of each
    __shared__ half8 L[4 * NP];
    load_matrix<4 * NP * 8, 256>(reinterpret_cast<_Float16*>(L), reinterpret_cast<const vf4*>(Ap));
    __syncthreads();

    const int lane = threadIdx.x & 63, p = lane & 31, h = lane >> 5;
    const uint64_t hoff = h ? (uint64_t(1) << g.t[K - 1]) : 0;
    // Without a target on qubit 0 the tile's columns are neighbouring
    // amplitudes. Lanes p and p + 16 (p < 16 within each half-wave) then hold
    // columns 2 p and 2 p + 1: each accesses both columns of every other row
    // (even rows in the lower lane, odd ones in the upper) as one 16 byte
    // access, and one lane swap per 32-bit value (v_permlane16_swap, between
    // the two 16-lane rows) gives each lane its own column after a load and
    // the pair of columns before a store. Half the memory instructions of
    // 8-byte accesses, for the same 256-byte runs: 2 % off the pass. Not in
    // the STATS form, whose store phase is bound by its float64 sums (the
    // swaps made it 3 % slower). With a target on qubit 0 the 16 byte
    // accesses are two rows of the lane's own column.
    constexpr bool PAIR = !LOWT && !STATS;
    const int cpair = PAIR ? 2 * (p & 15) : p;                  // first column of the lane's accesses
    const uint64_t cown = PAIR ? (uint64_t)((p >> 4) & 1) : 0;  // the lane's own column: cpair + cown
    const uint64_t roff = cown ? (uint64_t(1) << g.t[0]) : 0;   // odd rows
    const uint64_t ntiles = g.ncols / 32;
    const uint64_t stride = (uint64_t)gridDim.x * 4;
    const bool has_epi = epi != nullptr;
    const bool has_ph = has_epi && epi->n_ph > 0;
    // state offset of the lane's amplitude j = 8 a + i: olo[i] | ohi[a] (bits of
    // j on targets 0..2 and 3..5; target 6 is h)
    uint64_t olo[8], ohi[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        olo[i] = target_off<3>(i, g);
        ohi[i] = ((i & 1) ? uint64_t(1) << g.t[3] : 0) | ((i & 2) ? uint64_t(1) << g.t[4] : 0) |
                 ((i & 4) ? uint64_t(1) << g.t[5] : 0);
    }

    uint64_t tile = (uint64_t)xcd_block() * 4 + (threadIdx.x >> 6);
    double sv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (tile >= ntiles) {  // uniform in the wave: every wave reaches one reduction
        if constexpr (STATS) block_reduce_store(sv, 3, 0u, part + blockIdx.x * 8);
        return;
    }
    const uint64_t last = ntiles - 1;
    // amplitudes 8 a .. 8 a + 7 of the lane for a in [A0, A1)
    // (the bits are disjoint, so the OR is a sum: one pointer per group a,
    // then the low offsets added to it)
    // (b: the lane's access base, odd-row offset included)
    auto load = [&](uint64_t b, float (&X)[2 * HX], int a0, int a1) {
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            if (a < a0 || a >= a1) continue;
            const float2* pa = psi + (b | ohi[a]);
            if (LOWT || PAIR) {
#pragma unroll
                for (int i = 0; i < 8; i += 2) {
                    const float4 v = *reinterpret_cast<const float4*>(pa + olo[i]);
                    const int j = 8 * a + i;
                    X[2 * j] = v.x; X[2 * j + 1] = v.y; X[2 * j + 2] = v.z; X[2 * j + 3] = v.w;
                }
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const float2 v = pa[olo[i]];
                    const int j = 8 * a + i;
                    X[2 * j] = v.x; X[2 * j + 1] = v.y;
                }
            }
        }
    };
    // real and imaginary parts of amplitudes 8 s + i, scaled, into fp16
    // halves; returns the factor that undoes the column and matrix scaling
    half8 rh[S], rl[S], ih[S], il[S];
    auto split = [&](float (&X)[2 * HX]) -> float {
        if constexpr (PAIR) {  // rows j, j + 1 of the lane's own column
#pragma unroll
            for (int j = 0; j < HX; j += 2) {
                lane_swap16(X[2 * j], X[2 * j + 2]);
                lane_swap16(X[2 * j + 1], X[2 * j + 3]);
            }
        }
        float mx = 0.0f;  // largest magnitude (|x| is a free operand modifier of the max)
#pragma unroll
        for (int i = 0; i < 2 * HX; ++i) mx = fmaxf(mx, fabsf(X[i]));
        uint32_t mb = __float_as_uint(mx);
        mb = max(mb, (uint32_t)__shfl_xor((int)mb, 32));  // the other half of the column
        const int e = (int)(mb >> 23) - 126;               // largest magnitude < 2^e
        const int se = min(max(14 - e, -100), 100);
        const float sc = __builtin_ldexpf(1.0f, se);
        typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int s = 0; s < S; ++s) {
            u32x4 hr, lr, hi4, li4;
#pragma unroll
            for (int q = 0; q < 4; ++q) {  // amplitudes j, j + 1: halves q of the registers
                const int j = 8 * s + 2 * q;
                uint32_t a, b, c, d;
                split_pair_f16(X[2 * j], X[2 * j + 2], sc, a, b);
                split_pair_f16(X[2 * j + 1], X[2 * j + 3], sc, c, d);
                hr[q] = a;
                lr[q] = b;
                hi4[q] = c;
                li4[q] = d;
            }
            rh[s] = __builtin_bit_cast(half8, hr);
            rl[s] = __builtin_bit_cast(half8, lr);
            ih[s] = __builtin_bit_cast(half8, hi4);
            il[s] = __builtin_bit_cast(half8, li4);
        }
        return __builtin_ldexpf(1.0f, -se - 4);
    };
    floatx16 ar[RB], ai[RB];
    // the products of steps s0 .. s1 - 1
    auto mma = [&](int s0, int s1) {
        int aoff = lane;
        asm volatile("" : "+v"(aoff));  // keep the matrix reads inside the loop (not in registers)
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (s < s0 || s >= s1) continue;
            // -Im x: the sign bits of both packed halves flipped by one XOR per register
            typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
            const u32x4 sbit = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
            const half8 nh = __builtin_bit_cast(half8, __builtin_bit_cast(u32x4, ih[s]) ^ sbit);
            const half8 nl = __builtin_bit_cast(half8, __builtin_bit_cast(u32x4, il[s]) ^ sbit);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const int at = (rb * S + s) * 64 + aoff;
                const half8 Rh = L[at], Rl = L[NP + at], Ih = L[2 * NP + at], Il = L[3 * NP + at];
                ar[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Rh, rl[s], ar[rb], 0, 0, 0);
                ai[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ih, rl[s], ai[rb], 0, 0, 0);
                ar[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Rl, rh[s], ar[rb], 0, 0, 0);
                ai[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Il, rh[s], ai[rb], 0, 0, 0);
                ar[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Rh, rh[s], ar[rb], 0, 0, 0);
                ai[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ih, rh[s], ai[rb], 0, 0, 0);
                ar[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ih, nl, ar[rb], 0, 0, 0);
                ai[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Rh, il[s], ai[rb], 0, 0, 0);
                ar[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Il, nh, ar[rb], 0, 0, 0);
                ai[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Rl, ih[s], ai[rb], 0, 0, 0);
                ar[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ih, nh, ar[rb], 0, 0, 0);
                ai[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Rh, ih[s], ai[rb], 0, 0, 0);
            }
        }
    };

    uint64_t base = deposit_cols<K>(tile * 32 + cpair, g);
    float unscale;
    {
        float B[2 * HX];
        load(base | hoff | roff, B, 0, 8);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_sched_barrier(0);
        unscale = split(B);
    }
    do {
        const uint64_t nxt = tile + stride < last ? tile + stride : last;
        const uint64_t basen = deposit_cols<K>(nxt * 32 + cpair, g);
        // the next tile's loads go out in two halves: the second once the
        // first four steps have freed their operand registers
        float Bn[2 * HX];
        load(basen | hoff | roff, Bn, 0, 4);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int i = 0; i < 16; ++i) ar[rb][i] = ai[rb][i] = 0.0f;
        mma(0, 4);
        __builtin_amdgcn_sched_barrier(0);
        load(basen | hoff | roff, Bn, 4, 8);
        __builtin_amdgcn_sched_barrier(0);
        mma(4, 8);
        // Diagonal epilogue: the column's sign parity and phase are one complex
        // factor for all its amplitudes, so they join the scale (ucr, uci);
        // the sign mask over the target index becomes bit j of msk for the
        // lane's amplitude j (target 6 is the lane's h: its term is the
        // column's). The store loop is specialised on which parts are present.
        float ucr = unscale, uci = 0.0f;
        uint32_t mlo = 0, mhi = 0;  // bit j of mhi:mlo: amplitude j changes sign
        bool ph = false, sg = false;
        if (has_epi) {
            const ColFactor<float> f = col_factor<float>(epi, base | cown);
            if ((f.sgn ^ ((uint32_t)h & (f.w >> (K - 1)))) & 1u) ucr = -ucr;
            if (has_ph) {
                uci = ucr * f.ci;
                ucr = ucr * f.cr;
                ph = true;
            }
            const uint32_t pat[5] = {0xaaaaaaaau, 0xccccccccu, 0xf0f0f0f0u, 0xff00ff00u, 0xffff0000u};
#pragma unroll
            for (int b = 0; b < 5; ++b)
                if ((f.w >> b) & 1u) {
                    mlo ^= pat[b];
                    mhi ^= pat[b];
                }
            if ((f.w >> 5) & 1u) mhi = ~mhi;
            sg = epi->n_mix > 0;  // uniform: the descriptor has sign-mask terms
        }
        const uint64_t b0 = base | hoff | roff;
        auto store_all = [&](auto PH, auto SG) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int r = 0; r < 16; r += 2) {
                    const int j = 16 * rb + r;
                    float v[4];
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const float xr = ar[rb][r + u], xi = ai[rb][r + u];
                        if constexpr (decltype(PH)::value) {  // one fixed contraction in every variant
                            v[2 * u] = fmaf(xr, ucr, -(xi * uci));
                            v[2 * u + 1] = fmaf(xr, uci, xi * ucr);
                        } else {
                            v[2 * u] = xr * ucr;
                            v[2 * u + 1] = xi * ucr;
                        }
                        if constexpr (decltype(SG)::value) {
                            const int jj = j + u;
                            const uint32_t m = jj < 32 ? mlo : mhi;
                            const uint32_t sb = (m << (31 - (jj & 31))) & 0x80000000u;
                            v[2 * u] = __uint_as_float(__float_as_uint(v[2 * u]) ^ sb);
                            v[2 * u + 1] = __uint_as_float(__float_as_uint(v[2 * u + 1]) ^ sb);
                        }
                    }
                    if constexpr (STATS) {
                        stats_acc_f(sv, v[0], v[1]);
                        stats_acc_f(sv, v[2], v[3]);
                    }
                    if constexpr (PAIR) {  // row j of both columns (lower lane), row j + 1 (upper)
                        lane_swap16(v[0], v[2]);
                        lane_swap16(v[1], v[3]);
                    }
                    float2* pa = psi + (b0 | ohi[j >> 3]);
                    if (LOWT || PAIR) {
                        *reinterpret_cast<float4*>(pa + olo[j & 7]) = make_float4(v[0], v[1], v[2], v[3]);
                    } else {
                        pa[olo[j & 7]] = make_float2(v[0], v[1]);
                        pa[olo[(j + 1) & 7]] = make_float2(v[2], v[3]);
                    }
                }
        };
        using T_ = std::true_type;
        using F_ = std::false_type;
        if constexpr (STATS) {  // once per run: one general path (uci = 0, no mask bits when absent)
            store_all(T_(), T_());
        } else if (ph) {
            if (sg) store_all(T_(), T_()); else store_all(T_(), F_());
        } else {
            if (sg) store_all(F_(), T_()); else store_all(F_(), F_());
        }
        base = basen;
        unscale = split(Bn);
        tile += stride;
    } while (tile < ntiles);
    if constexpr (STATS) block_reduce_store(sv, 3, 0u, part + blockIdx.x * 8);
}

// ------------------------------------------------------------ cluster: MFMA, double
// v_mfma_f64_16x16x4_f64: lane l: p = l%16 (column), q = l/16 owns target
// indices x = j | q << (K-2), j < 2^(K-2), of its column(s). Operand A/B: lane
// l holds row / column l%16 at inner index l/16; result register r of lane l
// holds row 4 r + l/16, column l%16. Same prefetching loop as the float kernel.
template <int K, int NB, int THREADS>
__global__ __launch_bounds__(THREADS, 512 / THREADS) void k_cluster_f64_mfma(double2* __restrict__ psi,
                                                                           const double* __restrict__ Ap,
                                                                           const EpiDesc* __restrict__ epi,
                                                                           ClusterGeom g) {
    constexpr int D = 1 << K;
    constexpr int HX = D / 4;
    constexpr int RB = 2 * D / 16;
    constexpr int S = 2 * D / 4;
    constexpr int COLS = 16 * NB;
    constexpr int WAVES = THREADS / 64;
    __shared__ double As[RB * S * 64];
    load_matrix<RB * S * 64, THREADS>(As, reinterpret_cast<const vf4*>(Ap));
    __syncthreads();

    const int lane = threadIdx.x & 63, p = lane & 15, q = lane >> 4;
    const uint64_t qoff = ((q & 1) ? (uint64_t(1) << g.t[K - 2]) : 0) | ((q & 2) ? (uint64_t(1) << g.t[K - 1]) : 0);
    const uint64_t ntiles = g.ncols / COLS;
    const uint64_t stride = (uint64_t)gridDim.x * WAVES;
    const bool has_epi = epi != nullptr;
    const bool has_ph = has_epi && epi->n_ph > 0;

    auto load = [&](uint64_t t, uint64_t (&bs)[NB], double (&B)[NB][2 * HX]) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) bs[nb] = deposit_cols<K>(t * COLS + p + 16 * nb, g);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int j = 0; j < HX; ++j) {
                const double2 v = psi[bs[nb] | qoff | target_off<K - 2>(j, g)];
                B[nb][2 * j] = v.x;
                B[nb][2 * j + 1] = v.y;
            }
    };

    uint64_t tile = (uint64_t)xcd_block() * WAVES + (threadIdx.x >> 6);
    if (tile >= ntiles) return;
    const uint64_t last = ntiles - 1;
    double B[NB][2 * HX];
    uint64_t base[NB];
    load(tile, base, B);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_sched_barrier(0);
    do {
        const uint64_t nxt = tile + stride < last ? tile + stride : last;
        double Bn[NB][2 * HX];
        uint64_t basen[NB];
        load(nxt, basen, Bn);
        __builtin_amdgcn_sched_barrier(0);

        doublex4 acc[NB][RB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[nb][rb][i] = 0.0;
        int aoff = lane;
        asm volatile("" : "+v"(aoff));
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const double a = As[(rb * S + s) * 64 + aoff];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[nb][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, B[nb][s], acc[nb][rb], 0, 0, 0);
            }
        }
        // acc[nb][j / 2][2 (j % 2) + {0, 1}] is output amplitude j of the lane
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            ColFactor<double> f{0u, 0u, 1.0, 0.0};
            if (has_epi) f = col_factor<double>(epi, base[nb]);
#pragma unroll
            for (int j = 0; j < HX; ++j) {
                double re = acc[nb][j / 2][2 * (j % 2)], im = acc[nb][j / 2][2 * (j % 2) + 1];
                if (has_epi) apply_factor(re, im, f, (uint32_t)(j | (q << (K - 2))), has_ph);
                psi[base[nb] | qoff | target_off<K - 2>(j, g)] = make_double2(re, im);
            }
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            base[nb] = basen[nb];
#pragma unroll
            for (int j = 0; j < 2 * HX; ++j) B[nb][j] = Bn[nb][j];
        }
        tile += stride;
    } while (tile < ntiles);
}

// ------------------------------------------------------------ cluster: MFMA, LDS-staged
// The same MFMA products, but the wave tile (targets x 2^C columns) is moved
// between HBM and registers as linear runs of its tile index tau: lane l reads
// and writes 16 consecutive bytes, so each load / store instruction covers
// runs of at least 2^C amplitudes whatever the target bits are (targets on
// the lowest bits scatter a direct register gather across many cache lines).
// The re-ordering into the MFMA operand layout goes through a private LDS
// buffer of the wave; the next tile's linear loads are in flight while the
// current tile's MFMA chain runs.



// LDS exchange between lanes of one wave: LDS operations of a wave execute in
// order, so only the compiler must be kept from reordering them.
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// State offset of tile t: t deposited into the non-tile bit positions.
template <int NT>
__device__ __forceinline__ uint64_t tile_base(uint64_t t, const StageGeom& sg) {
#pragma unroll
    for (int i = 0; i < NT; ++i) t = insert_zero(t, sg.tb[i]);
    return t;
}

// tau of target index x (bits m0 <= m < m1 of x).
template <int M0, int M1>
__device__ __forceinline__ int tau_of_targets(int x, const StageGeom& sg) {
    int t = 0;
#pragma unroll
    for (int m = M0; m < M1; ++m)
        if ((x >> m) & 1) t |= 1 << sg.tpos[m];
    return t;
}

template <int C>
__device__ __forceinline__ int tau_of_column(int c, const StageGeom& sg) {
    int t = 0;
#pragma unroll
    for (int b = 0; b < C; ++b)
        if ((c >> b) & 1) t |= 1 << sg.cpos[b];
    return t;
}

template <int C>
__device__ __forceinline__ uint64_t state_bits_of_column(int c, const StageGeom& sg) {
    uint64_t o = 0;
#pragma unroll
    for (int b = 0; b < C; ++b)
        if ((c >> b) & 1) o |= uint64_t(1) << sg.tb[sg.cpos[b]];
    return o;
}

// Linear loads and the LDS re-ordering of the float staged kernel.
template <int K, int C, bool LOWT>
struct StageF32 {
    static constexpr int HX = (1 << K) / 2;
    static constexpr int NB = (1 << C) / 32;
    static constexpr int NL = (1 << (K + C)) / 128;
    // t0: the tile's base (uniform in the wave); lane_off: the lane's bits
    __device__ __forceinline__ static void load_lin(const g_float2* __restrict__ psi, uint64_t t0,
                                                    uint64_t lane_off, const StageGeom& sg, vf4 (&R)[NL]) {
#pragma unroll
        for (int i = 0; i < NL; ++i) R[i] = *reinterpret_cast<const g_vf4*>(psi + ((t0 | sg.ioff[i]) | lane_off));
    }
    __device__ __forceinline__ static void stage_in(vf4* L4, int lane, const int (&tc)[NB], int th,
                                                    const StageGeom& sg, const vf4 (&R)[NL],
                                                    float (&B)[NB][2 * HX]) {
#pragma unroll
        for (int i = 0; i < NL; ++i) L4[i * 64 + lane] = R[i];
        wave_lds_fence();
        if (!LOWT) {
#pragma unroll
            for (int j = 0; j < HX; ++j) {
                const vf4 v = L4[(tc[0] | th | tau_of_targets<0, K - 1>(j, sg)) >> 1];
                B[0][2 * j] = v.x; B[0][2 * j + 1] = v.y;
                B[1][2 * j] = v.z; B[1][2 * j + 1] = v.w;
            }
        } else {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int j = 0; j < HX; j += 2) {
                    const vf4 v = L4[(tc[nb] | th | tau_of_targets<0, K - 1>(j, sg)) >> 1];
                    B[nb][2 * j] = v.x; B[nb][2 * j + 1] = v.y;
                    B[nb][2 * j + 2] = v.z; B[nb][2 * j + 3] = v.w;
                }
        }
        wave_lds_fence();
    }
};

// float: lane l covers tau = 2 (i * 64 + l) + {0, 1} in linear order. In MFMA
// order lane (p, h) owns target indices j | h << (K-1) of columns 2p, 2p+1
// (tau bit 0 is a column bit) or p, p+32 (tau bit 0 is target 0, LOWT).
//
// One wave applies the cluster whose matrix is in LDS (As) to tiles
// tile, tile + stride, ... < tile_end, staging through its LDS buffer L4.
template <int K, int C, bool LOWT>
__device__ __forceinline__ void staged_f32_tiles(g_float2* __restrict__ psi, const float* As, vf4* L4,
                                                 c_epi* __restrict__ epi, const StageGeom& sg,
                                                 uint64_t tile, uint64_t tile_end, uint64_t stride) {
    constexpr int D = 1 << K;
    constexpr int HX = D / 2;
    constexpr int RB = 2 * D / 32;
    constexpr int S = D;
    constexpr int NB = (1 << C) / 32;
    constexpr int NT = K + C;
    constexpr int TILE = 1 << NT;
    constexpr int NL = TILE / 128;
    static_assert(NB == 2, "two column blocks per lane");
    // an opaque lane: what is derived from it is computed per call, not hoisted
    // into a caller's loop (the batch kernel's item loop) and kept live there
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    const int p = lane & 31, h = lane >> 5;
    uint64_t lane_off = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b)
        if ((lane >> b) & 1) lane_off |= uint64_t(1) << sg.tb[b + 1];
    int tc[NB];
    uint64_t cbits[NB];
    if (!LOWT) {
        tc[0] = tau_of_column<C>(2 * p, sg);
        tc[1] = tc[0] | 1;
        cbits[0] = state_bits_of_column<C>(2 * p, sg);
        cbits[1] = state_bits_of_column<C>(2 * p + 1, sg);
    } else {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            tc[nb] = tau_of_column<C>(p + 32 * nb, sg);
            cbits[nb] = state_bits_of_column<C>(p + 32 * nb, sg);
        }
    }
    const int th = h << sg.tpos[K - 1];
    const uint64_t ntiles = tile_end;
    const bool has_epi = epi != nullptr;
    const bool has_ph = has_epi && epi->n_ph > 0;

    if (tile >= ntiles) return;
    const uint64_t last = ntiles - 1;
    vf4 R[NL];
    StageF32<K, C, LOWT>::load_lin(psi, tile_base<NT>(tile, sg), lane_off, sg, R);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_sched_barrier(0);
    float B[NB][2 * HX];
    StageF32<K, C, LOWT>::stage_in(L4, lane, tc, th, sg, R, B);
    do {
        // the lane offset stays one value: the 16 chunk addresses built from it
        // are recomputed (an OR each) instead of held across the loop
        asm volatile("" : "+v"(lane_off));
        const uint64_t nxt = tile + stride < last ? tile + stride : last;
        StageF32<K, C, LOWT>::load_lin(psi, tile_base<NT>(nxt, sg), lane_off, sg, R);
        __builtin_amdgcn_sched_barrier(0);

        floatx16 acc[NB][RB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[nb][rb][i] = 0.0f;
        int aoff = lane;
        asm volatile("" : "+v"(aoff));
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const float a = As[(rb * S + s) * 64 + aoff];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[nb][rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, B[nb][s], acc[nb][rb], 0, 0, 0);
            }
        }
        float O[NB][2 * HX];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int j = 0; j < 2 * HX; ++j) O[nb][j] = acc[nb][j / 16][j % 16];
        const uint64_t tb0 = tile_base<NT>(tile, sg);
        if (has_epi) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const ColFactor<float> f = col_factor<float>(epi, tb0 | cbits[nb]);
#pragma unroll
                for (int j = 0; j < HX; ++j)
                    apply_factor(O[nb][2 * j], O[nb][2 * j + 1], f, (uint32_t)(j | (h << (K - 1))), has_ph);
            }
        }
        // MFMA order -> LDS -> linear order -> HBM
        if (!LOWT) {
#pragma unroll
            for (int j = 0; j < HX; ++j)
                L4[(tc[0] | th | tau_of_targets<0, K - 1>(j, sg)) >> 1] =
                    vf4{O[0][2 * j], O[0][2 * j + 1], O[1][2 * j], O[1][2 * j + 1]};
        } else {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                for (int j = 0; j < HX; j += 2)
                    L4[(tc[nb] | th | tau_of_targets<0, K - 1>(j, sg)) >> 1] =
                        vf4{O[nb][2 * j], O[nb][2 * j + 1], O[nb][2 * j + 2], O[nb][2 * j + 3]};
        }
        wave_lds_fence();
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const vf4 v = L4[i * 64 + lane];
            *reinterpret_cast<g_vf4*>(psi + ((tb0 | sg.ioff[i]) | lane_off)) = v;
        }
        wave_lds_fence();
        StageF32<K, C, LOWT>::stage_in(L4, lane, tc, th, sg, R, B);
        tile += stride;
    } while (tile < ntiles);
}



template <int K, int C, bool LOWT>
__global__ __launch_bounds__(256, 2) void k_cluster_f32_stage(float2* __restrict__ psi,
                                                              const float* __restrict__ Ap,
                                                              const EpiDesc* __restrict__ epi, ClusterGeom g,
                                                              StageGeom sg) {
    constexpr int D = 1 << K;
    constexpr int RB = 2 * D / 32;
    constexpr int S = D;
    constexpr int TILE = 1 << (K + C);
    __shared__ float As[RB * S * 64];
    __shared__ vf4 Ls[4][TILE / 2];
    load_matrix<RB * S * 64, 256>(As, reinterpret_cast<const vf4*>(Ap));
    __syncthreads();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: tile bases are scalar
    staged_f32_tiles<K, C, LOWT>((g_float2*)psi, As, Ls[w], (c_epi*)epi, sg, (uint64_t)xcd_block() * 4 + w,
                                 g.ncols >> C, (uint64_t)gridDim.x * 4);
}

template <int K, int C>
struct StageF64 {
    static constexpr int HX = (1 << K) / 4;
    static constexpr int NB = (1 << C) / 16;
    static constexpr int NL = (1 << (K + C)) / 64;
    // t0: the tile's base (uniform in the wave); lane_off: the lane's bits
    __device__ __forceinline__ static void load_lin(const vd2* __restrict__ psi, uint64_t t0, uint64_t lane_off,
                                                    const StageGeom& sg, vd2 (&R)[NL]) {
#pragma unroll
        for (int i = 0; i < NL; ++i) R[i] = *reinterpret_cast<const vd2*>(psi + ((t0 | sg.ioff[i]) | lane_off));
    }
    __device__ __forceinline__ static void stage_in(vd2* L, int lane, const int (&tc)[NB], int tq,
                                                    const StageGeom& sg, const vd2 (&R)[NL],
                                                    double (&B)[NB][2 * HX]) {
#pragma unroll
        for (int i = 0; i < NL; ++i) L[i * 64 + lane] = R[i];
        wave_lds_fence();
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int j = 0; j < HX; ++j) {
                const vd2 v = L[tc[nb] | tq | tau_of_targets<0, K - 2>(j, sg)];
                B[nb][2 * j] = v.x;
                B[nb][2 * j + 1] = v.y;
            }
        wave_lds_fence();
    }
};

// double: lane l covers tau = i * 64 + l in linear order; in MFMA order lane
// (p, q) owns target indices j | q << (K-2) of columns p and p + 16.
template <int K, int C, int THREADS>
__global__ __launch_bounds__(THREADS, 512 / THREADS) void k_cluster_f64_stage(vd2* __restrict__ psi,
                                                                            const double* __restrict__ Ap,
                                                                            const EpiDesc* __restrict__ epi,
                                                                            ClusterGeom g, StageGeom sg) {
    constexpr int D = 1 << K;
    constexpr int HX = D / 4;
    constexpr int RB = 2 * D / 16;
    constexpr int S = 2 * D / 4;
    constexpr int NB = (1 << C) / 16;
    constexpr int NT = K + C;
    constexpr int TILE = 1 << NT;
    constexpr int NL = TILE / 64;
    constexpr int WAVES = THREADS / 64;
    __shared__ double As[RB * S * 64];
    __shared__ vd2 Ls[WAVES][TILE];
    load_matrix<RB * S * 64, THREADS>(As, reinterpret_cast<const vf4*>(Ap));
    __syncthreads();

    const int lane = threadIdx.x & 63, p = lane & 15, q = lane >> 4,
              w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: tile bases are scalar
    vd2* L = Ls[w];
    uint64_t lane_off = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b)
        if ((lane >> b) & 1) lane_off |= uint64_t(1) << sg.tb[b];
    int tc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) tc[nb] = tau_of_column<C>(p + 16 * nb, sg);
    const int tq = ((q & 1) << sg.tpos[K - 2]) | ((q >> 1) << sg.tpos[K - 1]);
    const uint64_t ntiles = g.ncols >> C;
    const uint64_t stride = (uint64_t)gridDim.x * WAVES;
    const bool has_epi = epi != nullptr;
    const bool has_ph = has_epi && epi->n_ph > 0;

    uint64_t tile = (uint64_t)xcd_block() * WAVES + w;
    if (tile >= ntiles) return;
    const uint64_t last = ntiles - 1;
    vd2 R[NL];
    StageF64<K, C>::load_lin(psi, tile_base<NT>(tile, sg), lane_off, sg, R);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_sched_barrier(0);
    double B[NB][2 * HX];
    StageF64<K, C>::stage_in(L, lane, tc, tq, sg, R, B);
    do {
        asm volatile("" : "+v"(lane_off));  // chunk addresses recomputed, not held across the loop
        const uint64_t nxt = tile + stride < last ? tile + stride : last;
        StageF64<K, C>::load_lin(psi, tile_base<NT>(nxt, sg), lane_off, sg, R);
        __builtin_amdgcn_sched_barrier(0);

        doublex4 acc[NB][RB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[nb][rb][i] = 0.0;
        int aoff = lane;
        asm volatile("" : "+v"(aoff));
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const double a = As[(rb * S + s) * 64 + aoff];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    acc[nb][rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, B[nb][s], acc[nb][rb], 0, 0, 0);
            }
        }
        const uint64_t tb0 = tile_base<NT>(tile, sg);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            ColFactor<double> f{0u, 0u, 1.0, 0.0};
            // the column's state bits are rebuilt here (a few scalar-indexed
            // ORs) rather than held across the loop, where they were spilled
            if (has_epi) f = col_factor<double>(epi, tb0 | state_bits_of_column<C>(p + 16 * nb, sg));
#pragma unroll
            for (int j = 0; j < HX; ++j) {
                double re = acc[nb][j / 2][2 * (j % 2)], im = acc[nb][j / 2][2 * (j % 2) + 1];
                if (has_epi) apply_factor(re, im, f, (uint32_t)(j | (q << (K - 2))), has_ph);
                L[tc[nb] | tq | tau_of_targets<0, K - 2>(j, sg)] = vd2{re, im};
            }
        }
        wave_lds_fence();
        {
#pragma unroll
            for (int i = 0; i < NL; ++i) *reinterpret_cast<vd2*>(psi + ((tb0 | sg.ioff[i]) | lane_off)) = L[i * 64 + lane];
        }
        wave_lds_fence();
        StageF64<K, C>::stage_in(L, lane, tc, tq, sg, R, B);
        tile += stride;
    } while (tile < ntiles);
}

// ------------------------------------------------------------ several 5-qubit clusters per pass
// Any two 5-qubit clusters touch at most 10 qubits, so both fit in one tile of
// 2^11 amplitudes (their qubits plus the lowest other ones): the tile is read
// from HBM once, each cluster is applied to it in LDS, and it is written back
// once - one pass for M clusters (the GPU form of applying several gates while
// a block sits in fast memory, Fig. 2). Each cluster's product runs on the fp16
// matrix cores with operand halves (as for k = 6), which keeps M = 2 within the
// matrix-core time of one pass. The tile is kept in LDS in tile order tau; for
// cluster m the lanes read their two columns (the tile bits that are not m's
// targets) in MFMA order, and write the results back to the same places.
// sg[m]: the common tile bits (tb, ioff) and cluster m's target / column
// positions (tpos, cpos); tile bit 0 is either a column bit of m (lane (p, h)
// owns columns 2p, 2p + 1) or m's target 0 (columns p, p + 32).
struct MultiArgs {
    StageGeom sg[2];
    const half8* A[2];        // fp16-halves matrices (LAYOUT_SPLIT16F, k = 5)
    const EpiDesc* epi[2];
    int32_t lowt[2];
};

// LDS slot of amplitude v (tile order) in the multi-cluster kernel. With SWZ
// the higher index bits are folded into bits 1..3 by XOR, so lanes whose
// amplitudes differ only in high bits - a cluster's columns can sit on any
// tile bits - use different banks. The map is linear over XOR, hence
// slot(a | b) = slot(a) ^ slot(b) for disjoint a, b: column and target parts
// of an address are mapped once, outside the tile loop.
template <bool SWZ>
__device__ __forceinline__ int lds_slot(int v) {
    return SWZ ? v ^ ((((v >> 4) ^ (v >> 7) ^ (v >> 10)) & 7) << 1) : v;
}

template <int M, int WAVES, bool SWZ>
__global__ __launch_bounds__(WAVES * 64, 8 / WAVES) void k_cluster_f32_multi(float2* __restrict__ psi, MultiArgs a,
                                                                           uint64_t ntiles) {
    constexpr int K = 5, C = 6, HX = 16, RB = 2, S = 4, NL = 16;
    __shared__ half8 As[M][2][RB * S * 64];  // [cluster][hi, lo]
    __shared__ float2 Ls[WAVES][1 << (K + C)];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        load_matrix<RB * S * 64 * 8, WAVES * 64>(reinterpret_cast<_Float16*>(As[m][0]),
                                                reinterpret_cast<const vf4*>(a.A[m]));
        load_matrix<RB * S * 64 * 8, WAVES * 64>(reinterpret_cast<_Float16*>(As[m][1]),
                                                reinterpret_cast<const vf4*>(a.A[m] + RB * S * 64));
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, p = lane & 31, h = lane >> 5;
    float2* L = Ls[w];
    g_float2* gpsi = (g_float2*)psi;
    const StageGeom& sg0 = a.sg[0];
    uint64_t lane_off = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b)
        if ((lane >> b) & 1) lane_off |= uint64_t(1) << sg0.tb[b + 1];
    // Uniform state kept small (scalar registers are scarce here, and a
    // scalar reload waits on the LDS counter too): the tile chunks' state
    // offsets and each cluster's target offsets are linear in the index bits,
    // so four masks each stand for the sixteen values.
    uint64_t imask[4];  // state bit of tile bit 7 + b
#pragma unroll
    for (int b = 0; b < 4; ++b) imask[b] = uint64_t(1) << sg0.tb[7 + b];
    int tmask[M][4];    // mapped LDS offset of target b (b < 4) of cluster m
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
        for (int b = 0; b < 4; ++b) tmask[m][b] = lds_slot<SWZ>(1 << a.sg[m].tpos[b]);
    auto chunk_off = [&](int i) {
        uint64_t o = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if ((i >> b) & 1) o |= imask[b];
        return o;
    };
    auto load_tile = [&](uint64_t b0, vf4 (&R)[NL]) {
#pragma unroll
        for (int i = 0; i < NL; ++i) R[i] = *reinterpret_cast<const g_vf4*>(gpsi + (b0 | chunk_off(i)));
    };

    uint64_t tile = (uint64_t)xcd_block() * WAVES + w;
    if (tile >= ntiles) return;
    const uint64_t stride = (uint64_t)gridDim.x * WAVES;
    const uint64_t last = ntiles - 1;
    vf4 R[NL];
    load_tile(tile_base<K + C>(tile, sg0) | lane_off, R);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_sched_barrier(0);
    do {
        // the tile to LDS (tile order: lane l holds amplitudes 2 (i 64 + l) + {0, 1}),
        // then prefetch the next one
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int v = lds_slot<SWZ>(2 * (i * 64 + lane));  // bit 0 is 0 and not swizzled
            L[v] = make_float2(R[i].x, R[i].y);
            L[v | 1] = make_float2(R[i].z, R[i].w);
        }
        wave_lds_fence();
        const uint64_t nxt = tile + stride < last ? tile + stride : last;
        load_tile(tile_base<K + C>(nxt, sg0) | lane_off, R);
        __builtin_amdgcn_sched_barrier(0);
        const uint64_t tb0 = tile_base<K + C>(tile, sg0);

#pragma unroll
        for (int m = 0; m < M; ++m) {
            const StageGeom& sg = a.sg[m];
            c_epi* epi = (c_epi*)a.epi[m];
            const bool has_ph = epi != nullptr && epi->n_ph > 0;
            // the lane's two columns one after the other: amplitudes j | h << 4
#pragma unroll 1
            for (int nb = 0; nb < 2; ++nb) {
                const int col = a.lowt[m] ? p + 32 * nb : 2 * p + nb;
                const int coff = lds_slot<SWZ>(tau_of_column<C>(col, sg) | (h << sg.tpos[K - 1]));
                float X[2 * HX];
                auto toff = [&](int j) {
                    int o = 0;
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        if ((j >> b) & 1) o ^= tmask[m][b];
                    return o;
                };
#pragma unroll
                for (int j = 0; j < HX; ++j) {
                    const float2 v = L[coff ^ toff(j)];
                    X[2 * j] = v.x;
                    X[2 * j + 1] = v.y;
                }
                // fp16 halves, the column scaled by a power of two (shared by lanes p, p + 32)
                half8 xh[S], xl[S];
                const float unscale = __builtin_ldexpf(1.0f, -split_halves<2 * HX>(X, xh, xl) - 4);
                floatx16 acc[RB];
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int i = 0; i < 16; ++i) acc[rb][i] = 0.0f;
                int aoff = lane;
                asm volatile("" : "+v"(aoff));  // keep the matrix reads inside the loop (not in registers)
#pragma unroll
                for (int st = 0; st < S; ++st)
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
                        const half8 ah = As[m][0][(rb * S + st) * 64 + aoff];
                        const half8 al = As[m][1][(rb * S + st) * 64 + aoff];
                        acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, xl[st], acc[rb], 0, 0, 0);
                        acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, xh[st], acc[rb], 0, 0, 0);
                        acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, xh[st], acc[rb], 0, 0, 0);
                    }
#pragma unroll
                for (int j = 0; j < 2 * HX; ++j) X[j] = acc[j / 16][j % 16] * unscale;
                if (epi != nullptr) {
                    const ColFactor<float> f = col_factor<float>(epi, tb0 | state_bits_of_column<C>(col, sg));
#pragma unroll
                    for (int j = 0; j < HX; ++j)
                        apply_factor(X[2 * j], X[2 * j + 1], f, (uint32_t)(j | (h << (K - 1))), has_ph);
                }
                // every lane reads its column before any writes it (the lanes of a
                // column pair, p and p + 32, read disjoint amplitudes)
#pragma unroll
                for (int j = 0; j < HX; ++j) L[coff ^ toff(j)] = make_float2(X[2 * j], X[2 * j + 1]);
                __builtin_amdgcn_sched_barrier(0);
            }
            wave_lds_fence();
        }
        // tile order -> HBM
        {
            const uint64_t b0 = tb0 | lane_off;
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                const int v = lds_slot<SWZ>(2 * (i * 64 + lane));
                const float2 u = L[v], x = L[v | 1];
                *reinterpret_cast<g_vf4*>(gpsi + (b0 | chunk_off(i))) = vf4{u.x, u.y, x.x, x.y};
            }
        }
        wave_lds_fence();
        tile += stride;
    } while (tile < ntiles);
}

// Two 5-qubit clusters per pass on a tile of 2^10 amplitudes: the 10 tile bits
// hold both clusters' targets; each cluster's columns are the other 5 tile
// bits, one per lane pair (lane (p, h): column p, amplitudes j | h << 4). The
// smaller tile (8 KiB per wave) and the smaller register set let 12 waves
// share a CU, which hides more of each wave's serial chain (LDS, split,
// matrix cores, epilogue) under the other waves.
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64, 1) void k_cluster_f32_pair10(float2* __restrict__ psi, MultiArgs a,
                                                                   uint64_t ntiles) {
    constexpr int K = 5, NT = 10, HX = 16, RB = 2, S = 4, NL = 8;
    __shared__ half8 As[2][2][RB * S * 64];  // [cluster][hi, lo]
    __shared__ float2 Ls[WAVES][1 << NT];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        load_matrix<RB * S * 64 * 8, WAVES * 64>(reinterpret_cast<_Float16*>(As[m][0]),
                                                reinterpret_cast<const vf4*>(a.A[m]));
        load_matrix<RB * S * 64 * 8, WAVES * 64>(reinterpret_cast<_Float16*>(As[m][1]),
                                                reinterpret_cast<const vf4*>(a.A[m] + RB * S * 64));
    }
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, p = lane & 31, h = lane >> 5;
    float2* L = Ls[w];
    g_float2* gpsi = (g_float2*)psi;
    const StageGeom& sg0 = a.sg[0];
    uint64_t lane_off = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b)
        if ((lane >> b) & 1) lane_off |= uint64_t(1) << sg0.tb[b + 1];
    uint64_t imask[3];  // state bit of tile bit 7 + b
#pragma unroll
    for (int b = 0; b < 3; ++b) imask[b] = uint64_t(1) << sg0.tb[7 + b];
    auto chunk_off = [&](int i) {
        uint64_t o = 0;
#pragma unroll
        for (int b = 0; b < 3; ++b)
            if ((i >> b) & 1) o |= imask[b];
        return o;
    };
    // per cluster: mapped target offsets (linear in j) and the lane's column
    int tmask[2][4], coff[2];
    uint64_t cbits[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const StageGeom& sg = a.sg[m];
#pragma unroll
        for (int b = 0; b < 4; ++b) tmask[m][b] = lds_slot<true>(1 << sg.tpos[b]);
        coff[m] = lds_slot<true>(tau_of_column<5>(p, sg) | (h << sg.tpos[K - 1]));
        cbits[m] = state_bits_of_column<5>(p, sg);
    }

    uint64_t tile = (uint64_t)xcd_block() * WAVES + w;
    if (tile >= ntiles) return;
    const uint64_t stride = (uint64_t)gridDim.x * WAVES;
    const uint64_t last = ntiles - 1;
    vf4 R[NL];
    auto load_tile = [&](uint64_t b0) {
#pragma unroll
        for (int i = 0; i < NL; ++i) R[i] = *reinterpret_cast<const g_vf4*>(gpsi + (b0 | chunk_off(i)));
    };
    load_tile(tile_base<NT>(tile, sg0) | lane_off);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_sched_barrier(0);
    do {
#pragma unroll
        for (int i = 0; i < NL; ++i) {
            const int v = lds_slot<true>(2 * (i * 64 + lane));
            L[v] = make_float2(R[i].x, R[i].y);
            L[v | 1] = make_float2(R[i].z, R[i].w);
        }
        wave_lds_fence();
        const uint64_t nxt = tile + stride < last ? tile + stride : last;
        load_tile(tile_base<NT>(nxt, sg0) | lane_off);
        __builtin_amdgcn_sched_barrier(0);
        const uint64_t tb0 = tile_base<NT>(tile, sg0);
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            auto toff = [&](int j) {
                int o = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if ((j >> b) & 1) o ^= tmask[m][b];
                return o;
            };
            float X[2 * HX];
#pragma unroll
            for (int j = 0; j < HX; ++j) {
                const float2 v = L[coff[m] ^ toff(j)];
                X[2 * j] = v.x;
                X[2 * j + 1] = v.y;
            }
            half8 xh[S], xl[S];
            const int se = split_halves<2 * HX>(X, xh, xl);
            floatx16 acc[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[rb][i] = 0.0f;
            int aoff = lane;
            asm volatile("" : "+v"(aoff));  // keep the matrix reads inside the loop (not in registers)
#pragma unroll
            for (int st = 0; st < S; ++st)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    const half8 ah = As[m][0][(rb * S + st) * 64 + aoff];
                    const half8 al = As[m][1][(rb * S + st) * 64 + aoff];
                    acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, xl[st], acc[rb], 0, 0, 0);
                    acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, xh[st], acc[rb], 0, 0, 0);
                    acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, xh[st], acc[rb], 0, 0, 0);
                }
            // undo the scaling, with the column's diagonal phase folded in
            float ur = __builtin_ldexpf(1.0f, -se - 4), ui = 0.0f;
            uint32_t sgn = 0, wm = 0;
            c_epi* epi = (c_epi*)a.epi[m];
            if (epi != nullptr) {
                const ColFactor<float> f = col_factor<float>(epi, tb0 | cbits[m]);
                sgn = f.sgn;
                wm = f.w;
                ui = ur * f.ci;
                ur = ur * f.cr;
            }
#pragma unroll
            for (int j = 0; j < HX; ++j) {
                const float re = acc[j / 8][2 * (j % 8)], im = acc[j / 8][2 * (j % 8) + 1];
                float orr = re * ur - im * ui, oi = re * ui + im * ur;
                const bool neg = ((sgn ^ (uint32_t)__popc((uint32_t)(j | (h << (K - 1))) & wm)) & 1u) != 0;
                orr = neg ? -orr : orr;
                oi = neg ? -oi : oi;
                L[coff[m] ^ toff(j)] = make_float2(orr, oi);
            }
            wave_lds_fence();
        }
        {
            const uint64_t b0 = tb0 | lane_off;
#pragma unroll
            for (int i = 0; i < NL; ++i) {
                const int v = lds_slot<true>(2 * (i * 64 + lane));
                const float2 u = L[v], x = L[v | 1];
                *reinterpret_cast<g_vf4*>(gpsi + (b0 | chunk_off(i))) = vf4{u.x, u.y, x.x, x.y};
            }
        }
        wave_lds_fence();
        tile += stride;
    } while (tile < ntiles);
}

// ------------------------------------------------------------ cluster: float state, k = 6, LDS-staged
// The direct kernel above reads lane p's column with one load per amplitude;
// when several targets sit on the lowest state bits the 32 columns of a load
// are spread over up to 64 cache lines (8 - 16 bytes used of each), and the
// vector L1 becomes the bottleneck. This variant reads a tile of 2^11
// amplitudes (the 6 targets and the 5 lowest other bits) with linear 16-byte
// loads - 1 KiB runs - and re-orders it through LDS. Per wave the LDS holds
// half a tile (8 KiB): tile bit 10 is either target 5 (h) or column bit 4,
// so each lane's whole column lies in one half and the halves are staged one
// after the other. Eight waves and the matrix halves (64 KiB) fill 128 KiB.
// Core (fp16 halves on matrix cores, column scaling, epilogue) as above.
// Addresses: slot(tau) = swizzle(tau) & 1023 (StageGeom::swz, chosen per
// geometry so that the columns of a read pass fall on distinct banks), linear
// over XOR, so the lane's column part and the row part are mapped separately.
//
// One wave applies the cluster whose fp16 matrix halves are in LDS (Ah, Al)
// to tiles tile, tile + stride, ... < tile_end (tile numbers uniform in the
// wave), staging through its 8 KiB LDS buffer L.
//
// FOLD: the input is not loaded but computed - the state after the uniform
// start, a first cluster and its diagonal epilogue (see k_fold2_f32).
struct FoldIn {
    const float2* W;  // LDS: w over the first cluster's qubits (bit m of the index: its qubit m)
    int ymask[6];     // per row bit (this cluster's target m): the w-index bit it sets, 0 if none
    int t1[6];        // the first cluster's qubits
    int k1;
    c_epi* epi1;      // the first epilogue relative to this cluster's targets, or null
    // table form (FOLD 2): the second cluster's outputs split by the row bits
    // it shares with the first cluster (sigma: their pattern) and by the
    // first epilogue's row signs w. Row sigma + Wc[w] of Y (kFoldRow float2
    // each, in LDS) holds M2 applied to the sign vector of w restricted to
    // the rows of pattern sigma; a column's outputs are the sum over sigma of
    // W[ic | iys[sigma]] times that row.
    const float2* Y;
    const int* Wc;  // per row-sign mask w: its compressed index << (shared bits)
    int no;         // patterns sigma: 2^(shared row bits), at most 4
    int iys[4];     // w index of each pattern's shared rows
};
// LDS row of one table pattern: 64 outputs and a 16-byte pad, so that the
// rows of different patterns start on different banks
constexpr int kFoldRow = 66;

// FOLD: 0 the tile is loaded; 1 the column's inputs are computed from the
// first cluster's closed form and multiplied on the matrix cores; 2 the
// column's outputs are combined from the table of FoldIn::Y.
template <bool LOWT, int FOLD = 0>
__device__ __forceinline__ void split6s_tiles(g_float2* __restrict__ gpsi, const half8* Ah, const half8* Al, float2* L,
                                              c_epi* __restrict__ epi, const StageGeom& sg, uint64_t tile,
                                              uint64_t tile_end, uint64_t stride, const FoldIn* fin = nullptr) {
    constexpr int K = 6, C = 5, NT = K + C, HX = 32, RB = 4, S = 8, NL = 16;
    // an opaque lane: what is derived from it is computed per call, not hoisted
    // into a caller's loop (the batch kernel's item loop) and kept live there
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    const int p = lane & 31, h = lane >> 5;
    vf4* L4 = reinterpret_cast<vf4*>(L);
    bool has_epi = epi != nullptr;
    bool has_ph = has_epi && epi->n_ph > 0;
    if constexpr (FOLD != 0) {
        has_epi = has_epi || fin->epi1 != nullptr;
        has_ph = has_ph || (fin->epi1 != nullptr && fin->epi1->n_ph > 0);
    }
    uint64_t lane_off = 0;  // state offset of tile bits 1..6 (the lane of a linear load)
#pragma unroll
    for (int b = 0; b < 6; ++b)
        if ((lane >> b) & 1) lane_off |= uint64_t(1) << sg.tb[b + 1];
    // LDS slot of tau (the geometry's swizzle; linear over XOR)
    auto sslot = [&](int v) {
        int o = v;
#pragma unroll
        for (int i = 0; i < 6; ++i)
            if ((v >> (5 + i)) & 1) o ^= sg.swz[i];
        return o;
    };
    // the lane's column (tile order, then LDS slot), its half of the targets
    const int ctau = tau_of_column<C>(p, sg) | (h << sg.tpos[K - 1]);
    int lslot = sslot(ctau);
    uint32_t h5 = (uint32_t)h << (K - 1);
    const uint64_t cbits = state_bits_of_column<C>(p, sg);
    const int lph = (ctau >> 10) & 1;  // the half of the tile holding the column
    int lin = sslot(2 * lane);  // slot of linear chunk 0; chunk i adds slot(128 i) by XOR
    // row j's slot and linear chunk i's state offset, rebuilt from 5 and 4
    // uniform masks at each use (cheap scalar work) rather than 32 + 16 values
    // held across the loop
    int rmask[K - 1];
#pragma unroll
    for (int m = 0; m < K - 1; ++m) rmask[m] = sslot(1 << sg.tpos[m]);
    int cmask[4];  // slots of the linear chunks' bits (tau bits 7..10)
#pragma unroll
    for (int b = 0; b < 4; ++b) cmask[b] = sslot(128 << b);
    uint64_t imask[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) imask[b] = uint64_t(1) << sg.tb[7 + b];
    auto rslot = [&](int j) {
        int o = 0;
#pragma unroll
        for (int m = 0; m < K - 1; ++m)
            if ((j >> m) & 1) o ^= rmask[m];
        return o;
    };
    auto ioff = [&](int i) {
        uint64_t o = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if ((i >> b) & 1) o |= imask[b];
        return o;
    };
    auto cslot = [&](int i) {  // slot offset of linear chunk i (tau = 128 i)
        int o = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if ((i >> b) & 1) o ^= cmask[b];
        return o;
    };

    if (tile >= tile_end) return;
    const uint64_t last = tile_end - 1;
    // FOLD: the epilogue factors of both clusters and the w index, split into
    // column parts (here, once) and tile parts (lane j forms those of the
    // wave's tile it + j once per 64 tiles; each tile reads them from its lane)
    uint64_t colmask = 0;
    uint32_t l1s = 0, l1w = 0, l2s = 0, l2w = 0, t1b = 0, t2b = 0;
    double l1r = 1.0, l1i = 0.0, l2r = 1.0, l2i = 0.0, t1r = 1.0, t1i = 0.0, t2r = 1.0, t2i = 0.0;
    int icl = 0, it = 0;
    if constexpr (FOLD != 0) {
#pragma unroll
        for (int b = 0; b < C; ++b) colmask |= uint64_t(1) << sg.tb[sg.cpos[b]];
        if (fin->epi1 != nullptr) epi_lane_part(fin->epi1, cbits, colmask, l1s, l1w, l1r, l1i);
        if (epi != nullptr) epi_lane_part(epi, cbits, colmask, l2s, l2w, l2r, l2i);
#pragma unroll
        for (int m = 0; m < 6; ++m)
            if (m < fin->k1) icl |= (int)((cbits >> fin->t1[m]) & 1) << m;
    }
    vf4 R[NL];
    auto load_tile = [&](uint64_t t0) {  // t0: the tile's base (uniform)
#pragma unroll
        for (int i = 0; i < NL; ++i) R[i] = *reinterpret_cast<const g_vf4*>(gpsi + ((t0 | ioff(i)) | lane_off));
    };
    if constexpr (FOLD == 0) {
        load_tile(tile_base<NT>(tile, sg));
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_sched_barrier(0);
    }
    do {
        // per-lane bases stay in place: the 16 chunk addresses derived from them
        // are recomputed (one OR / XOR each) instead of held across the loop
        asm volatile("" : "+v"(lane_off), "+v"(lin), "+v"(lslot), "+v"(h5));
        asm volatile("" : "+s"(rmask[0]), "+s"(rmask[1]), "+s"(rmask[2]), "+s"(rmask[3]), "+s"(rmask[4]));
        asm volatile("" : "+s"(imask[0]), "+s"(imask[1]), "+s"(imask[2]), "+s"(imask[3]));
        asm volatile("" : "+s"(cmask[0]), "+s"(cmask[1]), "+s"(cmask[2]), "+s"(cmask[3]));
        float X[2 * HX];
        ColFactor<float> f1{0u, 0u, 1.0f, 0.0f}, f2{0u, 0u, 1.0f, 0.0f};
        if constexpr (FOLD != 0) {
            // the column's inputs from the closed form: w at the first cluster's
            // index (its qubits among the column bits, then among the row bits),
            // negated where a gate of the first epilogue couples a row bit with
            // a column bit; the column-only factor of that epilogue joins the
            // output factor
            if ((it & 63) == 0) {
                const uint64_t bj = tile_base<NT>(tile + (uint64_t)lane * stride, sg);  // past the end: unused
                t1b = 0;
                t2b = 0;
                if (fin->epi1 != nullptr) t1b = epi_tile_part(fin->epi1, bj, colmask, t1r, t1i);
                if (epi != nullptr) t2b = epi_tile_part(epi, bj, colmask, t2r, t2i);
                int ict = 0;
#pragma unroll
                for (int m = 0; m < 6; ++m)
                    if (m < fin->k1) ict |= (int)((bj >> fin->t1[m]) & 1) << m;
                t1b |= (uint32_t)ict << 12;
            }
            const int sl = it & 63;
            const uint32_t b1 = (uint32_t)__builtin_amdgcn_readlane((int)t1b, sl);
            const int ic = icl | (int)((b1 >> 12) & 63u);
            if (fin->epi1 != nullptr)
                f1 = epi_combine(b1, readlane_f64(t1r, sl), readlane_f64(t1i, sl), l1s, l1w, l1r, l1i, p);
            if (epi != nullptr)
                f2 = epi_combine((uint32_t)__builtin_amdgcn_readlane((int)t2b, sl), readlane_f64(t2r, sl),
                                 readlane_f64(t2i, sl), l2s, l2w, l2r, l2i, p);
            ++it;
            if constexpr (FOLD == 1) {
                const int yh = h ? fin->ymask[K - 1] : 0;
#pragma unroll
                for (int j = 0; j < HX; ++j) {
                    int iy = yh;
#pragma unroll
                    for (int b = 0; b < K - 1; ++b)
                        if ((j >> b) & 1) iy |= fin->ymask[b];
                    const float2 v = fin->W[ic | iy];
                    const bool neg = (__popc(((uint32_t)j | h5) & f1.w) & 1u) != 0;
                    X[2 * j] = neg ? -v.x : v.x;
                    X[2 * j + 1] = neg ? -v.y : v.y;
                }
            } else {
                // its half of the outputs (rows j | h << 5): the table rows of
                // its row-sign mask, weighted by w at its shared-row patterns
                const int pb = fin->Wc[f1.w & 63u];
#pragma unroll
                for (int j = 0; j < 2 * HX; ++j) X[j] = 0.0f;
#pragma unroll
                for (int sp = 0; sp < 4; ++sp) {
                    if (sp < fin->no) {
                        const float2 a = fin->W[ic | fin->iys[sp]];
                        const vf4* row = reinterpret_cast<const vf4*>(fin->Y + (pb + sp) * kFoldRow + h * HX);
#pragma unroll
                        for (int q = 0; q < HX / 2; ++q) {
                            const vf4 v = row[q];
                            X[4 * q] = fmaf(a.x, v.x, fmaf(-a.y, v.y, X[4 * q]));
                            X[4 * q + 1] = fmaf(a.x, v.y, fmaf(a.y, v.x, X[4 * q + 1]));
                            X[4 * q + 2] = fmaf(a.x, v.z, fmaf(-a.y, v.w, X[4 * q + 2]));
                            X[4 * q + 3] = fmaf(a.x, v.w, fmaf(a.y, v.z, X[4 * q + 3]));
                        }
                    }
                }
            }
        } else {
        // tile -> LDS, half by half; each lane reads its column in its half
#pragma unroll
        for (int ph = 0; ph < 2; ++ph) {
#pragma unroll
            for (int ii = 0; ii < NL / 2; ++ii) {
                const int i = ph * (NL / 2) + ii;
                L4[((lin ^ cslot(i)) & 1023) >> 1] = R[i];
            }
            wave_lds_fence();
            if (lph == ph) {
                if (LOWT) {
#pragma unroll
                    for (int j = 0; j < HX; j += 2) {
                        const vf4 v = L4[((lslot ^ rslot(j)) & 1023) >> 1];
                        X[2 * j] = v.x; X[2 * j + 1] = v.y; X[2 * j + 2] = v.z; X[2 * j + 3] = v.w;
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < HX; ++j) {
                        const float2 v = L[(lslot ^ rslot(j)) & 1023];
                        X[2 * j] = v.x; X[2 * j + 1] = v.y;
                    }
                }
            }
            wave_lds_fence();
        }
        }
        if constexpr (FOLD != 2) {
            // fp16 halves of the scaled column (shared scale with lane p + 32)
            half8 xh[S], xl[S];
            const int se = split_halves<2 * HX>(X, xh, xl);
            // the column is in registers: prefetch the next tile (issued here, the
            // peak register use is the halves + accumulators + the tile in flight)
            if constexpr (FOLD == 0) {
                const uint64_t nxt = tile + stride < last ? tile + stride : last;
                __builtin_amdgcn_sched_barrier(0);
                load_tile(tile_base<NT>(nxt, sg));
                __builtin_amdgcn_sched_barrier(0);
            }
            floatx16 acc[RB];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[rb][i] = 0.0f;
            int aoff = lane;
            asm volatile("" : "+v"(aoff));  // keep the matrix reads inside the loop (not in registers)
#pragma unroll
            for (int st = 0; st < S; ++st)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    const half8 ah = Ah[(rb * S + st) * 64 + aoff];
                    const half8 al = Al[(rb * S + st) * 64 + aoff];
                    acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, xl[st], acc[rb], 0, 0, 0);
                    acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, xh[st], acc[rb], 0, 0, 0);
                    acc[rb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, xh[st], acc[rb], 0, 0, 0);
                }
            const float unscale = __builtin_ldexpf(1.0f, -se - 4);
#pragma unroll
            for (int j = 0; j < 2 * HX; ++j) X[j] = acc[j / 16][j % 16] * unscale;
        }
        const uint64_t tb0 = tile_base<NT>(tile, sg);
        if (has_epi) {
            ColFactor<float> f{0u, 0u, 1.0f, 0.0f};
            if constexpr (FOLD != 0) {
                f = f2;
            } else {
                if (epi != nullptr) f = col_factor<float>(epi, tb0 | cbits);
            }
            if constexpr (FOLD != 0) {  // the first epilogue's column-only sign and phase
                f.sgn ^= f1.sgn;
                const float r = f.cr * f1.cr - f.ci * f1.ci;
                f.ci = f.cr * f1.ci + f.ci * f1.cr;
                f.cr = r;
            }
#pragma unroll
            for (int j = 0; j < HX; ++j)
                apply_factor(X[2 * j], X[2 * j + 1], f, (uint32_t)j | h5, has_ph);
        }
        // results -> LDS -> HBM, half by half
#pragma unroll
        for (int ph = 0; ph < 2; ++ph) {
            if (lph == ph) {
                if (LOWT) {
#pragma unroll
                    for (int j = 0; j < HX; j += 2)
                        L4[((lslot ^ rslot(j)) & 1023) >> 1] = vf4{X[2 * j], X[2 * j + 1], X[2 * j + 2], X[2 * j + 3]};
                } else {
#pragma unroll
                    for (int j = 0; j < HX; ++j) L[(lslot ^ rslot(j)) & 1023] = make_float2(X[2 * j], X[2 * j + 1]);
                }
            }
            wave_lds_fence();
#pragma unroll
            for (int ii = 0; ii < NL / 2; ++ii) {
                const int i = ph * (NL / 2) + ii;
                *reinterpret_cast<g_vf4*>(gpsi + ((tb0 | ioff(i)) | lane_off)) =
                    L4[((lin ^ cslot(i)) & 1023) >> 1];
            }
            wave_lds_fence();
        }
        tile += stride;
    } while (tile < tile_end);
}

template <bool LOWT>
__global__ __launch_bounds__(512, 1) void k_cluster_f32_split6s(float2* __restrict__ psi,
                                                                const half8* __restrict__ Ap,
                                                                const EpiDesc* __restrict__ epi, StageGeom sg,
                                                                uint64_t ntiles) {
    constexpr int RB = 4, S = 8, WAVES = 8;
    __shared__ half8 Ah[RB * S * 64];
    __shared__ half8 Al[RB * S * 64];
    __shared__ float2 Ls[WAVES][1024];
    load_matrix<RB * S * 64 * 8, WAVES * 64>(reinterpret_cast<_Float16*>(Ah), reinterpret_cast<const vf4*>(Ap));
    load_matrix<RB * S * 64 * 8, WAVES * 64>(reinterpret_cast<_Float16*>(Al),
                                            reinterpret_cast<const vf4*>(Ap + RB * S * 64));
    __syncthreads();
    // the wave index is uniform in the wave: tile numbers and bases are scalar
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    split6s_tiles<LOWT>((g_float2*)psi, Ah, Al, Ls[w], (c_epi*)epi, sg, (uint64_t)xcd_block() * WAVES + w, ntiles,
                        (uint64_t)gridDim.x * WAVES);
}

// ------------------------------------------------------------ uniform start + two clusters, one write-only pass
// From the uniform start, after a first cluster (qubits T1, matrix M1) and its
// diagonal epilogue E1 the state is a closed form: psi(x) = w[x on T1] E1(x),
// w = 2^(-n/2) times the row sums of M1. Relative to the second cluster's
// targets T2, E1 splits into terms on T2 alone (folded into the second matrix,
// before its gates, when it is built), terms coupling one T2 qubit with one
// column bit (a sign mask over the row index, per column) and terms on column
// bits alone (a sign and a phase per column, which commute with the product
// and join the second epilogue). The second cluster is then applied to inputs
// computed from w instead of loaded: one write-only pass stands for the
// initialisation and two cluster passes. The second cluster has 6 qubits; its
// core and write-back are those of the staged 6-qubit kernel.
struct Fold2Args {
    const double2* M1;  // first cluster: plain complex128 2^k1 x 2^k1, row-major
    double amp;         // 2^(-n/2)
    int32_t k1;
    int32_t t1[7];      // its qubits (sorted)
};

template <bool LOWT>
__global__ __launch_bounds__(512, 1) void k_fold2_f32(float2* __restrict__ psi, const half8* __restrict__ Ap,
                                                      const EpiDesc* __restrict__ epi2, const EpiDesc* __restrict__ epi1,
                                                      StageGeom sg, Fold2Args f, uint64_t ntiles) {
    constexpr int RB = 4, S = 8, WAVES = 8;
    __shared__ half8 Ah[RB * S * 64];
    __shared__ half8 Al[RB * S * 64];
    __shared__ float2 Ls[WAVES][1024];
    __shared__ float2 W[64];
    load_matrix<RB * S * 64 * 8, WAVES * 64>(reinterpret_cast<_Float16*>(Ah), reinterpret_cast<const vf4*>(Ap));
    load_matrix<RB * S * 64 * 8, WAVES * 64>(reinterpret_cast<_Float16*>(Al),
                                            reinterpret_cast<const vf4*>(Ap + RB * S * 64));
    const int d1 = 1 << f.k1;
    if ((int)threadIdx.x < 64) W[threadIdx.x] = make_float2(0.0f, 0.0f);
    __syncthreads();
    row_sums(f.M1, d1, f.amp, W);  // w: the first cluster applied to the uniform vector
    __syncthreads();
    FoldIn fin;
    fin.W = W;
    fin.k1 = f.k1;
    fin.epi1 = (c_epi*)epi1;
#pragma unroll
    for (int m = 0; m < 6; ++m) fin.t1[m] = f.t1[m];
#pragma unroll
    for (int m2 = 0; m2 < 6; ++m2) {
        const int q = sg.tb[sg.tpos[m2]];
        int b = 0;
#pragma unroll
        for (int m1 = 0; m1 < 6; ++m1)
            if (m1 < f.k1 && f.t1[m1] == q) b = 1 << m1;
        fin.ymask[m2] = b;
    }
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    split6s_tiles<LOWT, 1>((g_float2*)psi, Ah, Al, Ls[w], (c_epi*)epi2, sg, (uint64_t)xcd_block() * WAVES + w,
                              ntiles, (uint64_t)gridDim.x * WAVES, &fin);
}

// Table form: the second cluster's inputs are x[r] = w[ic | iy(r)] s(r) -
// w at the first cluster's index (ic from the column bits, iy from the rows
// the two clusters share), s the first epilogue's row signs. Split by the
// pattern sigma of the shared rows, M2 x = sum over sigma of
// w[ic | iy(sigma)] M2 (s restricted to the rows of pattern sigma), and s is
// fixed by the mask of its sign-flipped rows. One work-group per (sigma,
// compressed mask) forms M2 times that signed indicator in float64; the pass
// below weights and sums its rows per column.
struct FoldTabArgs {
    const double2* M2;  // second cluster: plain complex128 2^k2 x 2^k2, row-major
    int32_t omask;      // rows (second cluster's target bits) shared with the first cluster
    int32_t rmask;      // rows the first epilogue's mixed terms sign-flip
};

// bits of v at the set bits of mask (B bits), packed low; and back
template <int B>
__device__ __forceinline__ int pext_bits(int v, int mask) {
    int o = 0, k = 0;
#pragma unroll
    for (int b = 0; b < B; ++b)
        if ((mask >> b) & 1) o |= ((v >> b) & 1) << k++;
    return o;
}
template <int B>
__device__ __forceinline__ int pdep_bits(int v, int mask) {
    int o = 0, k = 0;
#pragma unroll
    for (int b = 0; b < B; ++b)
        if ((mask >> b) & 1) o |= ((v >> k++) & 1) << b;
    return o;
}

// one work-group of 2^K2 threads (one per output row) per table row
template <int K2>
__global__ __launch_bounds__(1 << K2) void k_fold2_table(float2* __restrict__ Y, FoldTabArgs a) {
    constexpr int D2 = 1 << K2;
    __shared__ double x[D2];
    const int t = threadIdx.x;
    const int no = __popc(a.omask);
    const int P = blockIdx.x;
    const int sigma = P & ((1 << no) - 1);
    const int w = pdep_bits<K2>(P >> no, a.rmask);
    x[t] = pext_bits<K2>(t, a.omask) != sigma ? 0.0 : ((__popc(t & w) & 1) ? -1.0 : 1.0);
    __syncthreads();
    double re = 0.0, im = 0.0;
    for (int s = 0; s < D2; ++s) {
        const double2 m = a.M2[t * D2 + s];
        re = fma(m.x, x[s], re);
        im = fma(m.y, x[s], im);
    }
    Y[P * D2 + t] = make_float2((float)re, (float)im);
}

template <bool LOWT>
__global__ __launch_bounds__(512, 1) void k_fold2t_f32(float2* __restrict__ psi, const float2* __restrict__ Yg,
                                                       const EpiDesc* __restrict__ epi2,
                                                       const EpiDesc* __restrict__ epi1, StageGeom sg, Fold2Args f,
                                                       FoldTabArgs a, uint64_t ntiles) {
    constexpr int WAVES = 8;
    __shared__ float2 Y[kFoldTabRows * kFoldRow];
    __shared__ float2 Ls[WAVES][1024];
    __shared__ float2 W[64];
    __shared__ int Wc[64];
    const int no = __popc(a.omask);
    // the table into LDS, rows padded to kFoldRow
    const int nq = 32 << (no + __popc(a.rmask));  // 16-byte pieces
    for (int i = (int)threadIdx.x; i < nq; i += (int)blockDim.x)
        reinterpret_cast<vf4*>(Y + (i >> 5) * kFoldRow)[i & 31] = reinterpret_cast<const vf4*>(Yg)[i];
    if ((int)threadIdx.x < 64) {
        W[threadIdx.x] = make_float2(0.0f, 0.0f);
        Wc[threadIdx.x] = pext_bits<6>((int)threadIdx.x, a.rmask) << no;
    }
    __syncthreads();
    row_sums(f.M1, 1 << f.k1, f.amp, W);  // w: the first cluster applied to the uniform vector
    __syncthreads();
    FoldIn fin;
    fin.W = W;
    fin.k1 = f.k1;
    fin.epi1 = (c_epi*)epi1;
#pragma unroll
    for (int m = 0; m < 6; ++m) fin.t1[m] = f.t1[m];
    int ymask[6];
#pragma unroll
    for (int m2 = 0; m2 < 6; ++m2) {
        const int q = sg.tb[sg.tpos[m2]];
        int b = 0;
#pragma unroll
        for (int m1 = 0; m1 < 6; ++m1)
            if (m1 < f.k1 && f.t1[m1] == q) b = 1 << m1;
        ymask[m2] = b;
        fin.ymask[m2] = b;
    }
    fin.Y = Y;
    fin.Wc = Wc;
    fin.no = 1 << no;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int rows = pdep_bits<6>(s, a.omask);
        int iy = 0;
#pragma unroll
        for (int m = 0; m < 6; ++m)
            if ((rows >> m) & 1) iy |= ymask[m];
        fin.iys[s] = iy;
    }
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    split6s_tiles<LOWT, 2>((g_float2*)psi, nullptr, nullptr, Ls[w], (c_epi*)epi2, sg, (uint64_t)xcd_block() * WAVES + w,
                           ntiles, (uint64_t)gridDim.x * WAVES, &fin);
}

// Table form with a 7-qubit second cluster (the first has at most 7 qubits):
// the write-only pass has no matrix in LDS, only the table (rows of 128
// outputs), so two work-groups fit per compute unit. The lanes own the
// amplitudes the 7-qubit cluster kernel's lanes do - lane (p, h) the
// amplitudes j | h << 6 of column p - and store them the same way; each
// output is summed from at most 4 table rows, weighted by w at the first
// cluster's index, then takes both epilogues' column factors and the second
// one's row signs.
constexpr int kFold7Row = 130;  // LDS row: 128 outputs and a 16-byte pad

template <bool LOWT>
__global__ __launch_bounds__(256, 2) void k_fold2t7_f32(float2* __restrict__ psi, const float2* __restrict__ Yg,
                                                        const EpiDesc* __restrict__ epi2,
                                                        const EpiDesc* __restrict__ epi1, ClusterGeom g, Fold2Args f,
                                                        FoldTabArgs a) {
    constexpr int K = 7, HX = 64;
    __shared__ float2 Y[kFoldTab7Rows * kFold7Row];
    __shared__ float2 W[128];
    __shared__ int Wc[128];
    const int no = __popc(a.omask);
    const int nq = 64 << (no + __popc(a.rmask));  // 16-byte pieces of the table
    for (int i = (int)threadIdx.x; i < nq; i += (int)blockDim.x)
        reinterpret_cast<vf4*>(Y + (i >> 6) * kFold7Row)[i & 63] = reinterpret_cast<const vf4*>(Yg)[i];
    if ((int)threadIdx.x < 128) {
        W[threadIdx.x] = make_float2(0.0f, 0.0f);
        Wc[threadIdx.x] = pext_bits<7>((int)threadIdx.x, a.rmask) << no;
    }
    __syncthreads();
    row_sums(f.M1, 1 << f.k1, f.amp, W);  // w: the first cluster applied to the uniform vector
    __syncthreads();
    // w-index bits of the rows both clusters hold, per shared-row pattern
    int iys[4];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
        const int rows = pdep_bits<7>(sp, a.omask);
        int iy = 0;
#pragma unroll
        for (int m = 0; m < K; ++m)
            if ((rows >> m) & 1)
#pragma unroll
                for (int m1 = 0; m1 < 7; ++m1)
                    if (m1 < f.k1 && f.t1[m1] == g.t[m]) iy |= 1 << m1;
        iys[sp] = iy;
    }
    const int nsp = 1 << no;

    const int lane = threadIdx.x & 63, p = lane & 31, h = lane >> 5;
    const uint64_t hoff = h ? (uint64_t(1) << g.t[K - 1]) : 0;
    const uint64_t ntiles = g.ncols / 32;
    const uint64_t stride = (uint64_t)gridDim.x * 4;
    uint64_t olo[8], ohi[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        olo[i] = target_off<3>(i, g);
        ohi[i] = ((i & 1) ? uint64_t(1) << g.t[3] : 0) | ((i & 2) ? uint64_t(1) << g.t[4] : 0) |
                 ((i & 4) ? uint64_t(1) << g.t[5] : 0);
    }
    for (uint64_t tile = (uint64_t)xcd_block() * 4 + (threadIdx.x >> 6); tile < ntiles; tile += stride) {
        const uint64_t base = deposit_cols<K>(tile * 32 + p, g);
        // the first cluster's index from the column's bits (its qubits among
        // the second's targets are rows: zero in base)
        int ic = 0;
#pragma unroll
        for (int m = 0; m < 7; ++m)
            if (m < f.k1) ic |= (int)((base >> f.t1[m]) & 1) << m;
        ColFactor<float> f1{0u, 0u, 1.0f, 0.0f}, f2{0u, 0u, 1.0f, 0.0f};
        if (epi1 != nullptr) f1 = col_factor<float>((c_epi*)epi1, base);
        if (epi2 != nullptr) f2 = col_factor<float>((c_epi*)epi2, base);
        const int pb = Wc[f1.w & 127u];
        float X[2 * HX];
#pragma unroll
        for (int j = 0; j < 2 * HX; ++j) X[j] = 0.0f;
#pragma unroll
        for (int sp = 0; sp < 4; ++sp) {
            if (sp < nsp) {
                const float2 wv = W[ic | iys[sp]];
                const vf4* row = reinterpret_cast<const vf4*>(Y + (pb + sp) * kFold7Row + h * HX);
#pragma unroll
                for (int q = 0; q < HX / 2; ++q) {
                    const vf4 v = row[q];
                    X[4 * q] = fmaf(wv.x, v.x, fmaf(-wv.y, v.y, X[4 * q]));
                    X[4 * q + 1] = fmaf(wv.x, v.y, fmaf(wv.y, v.x, X[4 * q + 1]));
                    X[4 * q + 2] = fmaf(wv.x, v.z, fmaf(-wv.y, v.w, X[4 * q + 2]));
                    X[4 * q + 3] = fmaf(wv.x, v.w, fmaf(wv.y, v.z, X[4 * q + 3]));
                }
            }
        }
        // the column factor of both epilogues (the first one's row signs are
        // in the table; the second one's sign mask over the lane's rows j and
        // its term on target 6, the lane's h)
        const uint32_t sgn = f1.sgn ^ f2.sgn ^ ((uint32_t)h & (f2.w >> (K - 1)));
        float ucr = f1.cr * f2.cr - f1.ci * f2.ci, uci = f1.cr * f2.ci + f1.ci * f2.cr;
        if (sgn & 1u) {
            ucr = -ucr;
            uci = -uci;
        }
        const uint32_t wl = f2.w & 63u;
        const uint64_t b0 = base | hoff;
#pragma unroll
        for (int j = 0; j < HX; j += 2) {
            float v[4];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const float xr = X[2 * (j + u)], xi = X[2 * (j + u) + 1];
                const float neg = (__popc((uint32_t)(j + u) & wl) & 1) ? -1.0f : 1.0f;
                v[2 * u] = neg * fmaf(xr, ucr, -(xi * uci));
                v[2 * u + 1] = neg * fmaf(xr, uci, xi * ucr);
            }
            float2* pa = psi + (b0 | ohi[j >> 3]);
            if (LOWT) {
                *reinterpret_cast<float4*>(pa + olo[j & 7]) = make_float4(v[0], v[1], v[2], v[3]);
            } else {
                pa[olo[j & 7]] = make_float2(v[0], v[1]);
                pa[olo[(j + 1) & 7]] = make_float2(v[2], v[3]);
            }
        }
    }
}

// ------------------------------------------------------------ batched persistent launch
// Many independent circuits in one launch. Work items (an op and a run of its
// tiles) are handed out by an atomic ticket in dependency order -
// the j-th op of every circuit before any (j+1)-th op - so an item only ever
// waits for items with smaller tickets, which running work-groups hold. Before
// starting, a work-group waits until all earlier items of its circuit are
// complete (per-circuit counter, release / acquire at device scope); the wait
// is bounded by the device's wall clock and sets an error flag instead of
// hanging. counters: [0] ticket, [1] error flag, [2 + c] completed items of
// circuit c.
//
// Loop shape: the loop body ends with a work-group barrier, and the single
// thread-0 block (publish the previous item, take a ticket) opens it, so the
// loop has one latch that every thread passes. A thread-0 block just before
// the back edge would give the header two back edges; the compiler may then
// split the loop into an inner loop that every other thread keeps running -
// through the barriers, re-reading a stale ticket - while thread 0 waits
// outside it. The ticket goes through readfirstlane so that the exit test is
// uniform, too.
__global__ __launch_bounds__(512, 1) void k_batch_f32(const BatchOp* __restrict__ ops,
                                                      const BatchItem* __restrict__ items, uint32_t n_items,
                                                      uint32_t* counters, uint32_t item_tiles, uint64_t wait_ticks) {
    constexpr int K = 5, C = 6, WAVES = 8;
    // One LDS buffer, two layouts. 5-qubit ops: the real-split matrix (16 KiB)
    // and a 16 KiB tile per wave; 6-qubit ops: the fp16 matrix halves (64 KiB)
    // and an 8 KiB half tile per wave. 144 KiB: one work-group per CU.
    __shared__ vf4 Lraw[1024 + WAVES * 1024];
    // the ticket is broadcast through the matrix region (read before the
    // barrier that precedes every matrix load)
    uint32_t* s_it = reinterpret_cast<uint32_t*>(Lraw);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    uint32_t* done = counters + 2;
    int prev = -1;  // circuit of the item just finished (uniform)
    for (;;) {
        if (threadIdx.x == 0) {
            // the previous item's stores are complete and released (fence + barrier below)
            if (prev >= 0) __hip_atomic_fetch_add(done + prev, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            *s_it = atomicAdd(counters, 1u);
        }
        __syncthreads();
        const uint32_t it = __builtin_amdgcn_readfirstlane(*s_it);
        if (it >= n_items) break;
        const BatchItem item = items[it];
        const BatchOp* op = ops + item.op;
        const uint32_t dep = op->dep;
        const int circ = op->circuit;
        if (threadIdx.x == 0 && dep > 0) {
            const uint64_t t0 = wall_clock64();
            while (__hip_atomic_load(done + circ, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < dep) {
                if (wall_clock64() - t0 > wait_ticks) {
                    atomicOr(counters + 1, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(4);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const uint64_t tiles = op->tiles;
        const uint64_t t_end = item.tile0 + item_tiles < tiles ? item.tile0 + item_tiles : tiles;
        g_float2* psi = (g_float2*)op->psi;
        if (op->kind == 0) {
            const g_vf4* A = (const g_vf4*)op->A;
            c_epi* epi = (c_epi*)op->epi;
            float* As = reinterpret_cast<float*>(Lraw);
            load_matrix<2 * 32 * 64, WAVES * 64>(As, A);
            __syncthreads();
            vf4* L4 = Lraw + 1024 + w * 1024;
            if (op->lowt)
                staged_f32_tiles<K, C, true>(psi, As, L4, epi, op->sg, item.tile0 + w, t_end, WAVES);
            else
                staged_f32_tiles<K, C, false>(psi, As, L4, epi, op->sg, item.tile0 + w, t_end, WAVES);
        } else if (op->kind == 3) {
            // a 6-qubit cluster: fp16 matrix halves, staged half tiles
            const g_vf4* A = (const g_vf4*)op->A;
            c_epi* epi = (c_epi*)op->epi;
            half8* Ah = reinterpret_cast<half8*>(Lraw);
            half8* Al = Ah + 2048;
            load_matrix<2048 * 8, WAVES * 64>(reinterpret_cast<_Float16*>(Ah), A);
            load_matrix<2048 * 8, WAVES * 64>(reinterpret_cast<_Float16*>(Al), A + 2048);
            __syncthreads();
            float2* L = reinterpret_cast<float2*>(Lraw + 4096 + w * 512);
            if (op->lowt)
                split6s_tiles<true>(psi, Ah, Al, L, epi, op->sg, item.tile0 + w, t_end, WAVES);
            else
                split6s_tiles<false>(psi, Ah, Al, L, epi, op->sg, item.tile0 + w, t_end, WAVES);
        } else if (op->kind == 4) {
            // the uniform start with the circuit's first cluster, written in one
            // pass: amplitude (column, target index y) = w[y] times the column's
            // epilogue factor, w = 2^(-n/2) times the row sums of the cluster
            // an opaque copy of the lane: what this branch derives from it is not
            // hoisted out of the item loop, where it would be live in every branch
            int ln = lane;
            asm volatile("" : "+v"(ln));
            const int k = (int)op->k, d = 1 << k, cb = 11 - k;
            const double2* M = reinterpret_cast<const double2*>(op->A);
            c_epi* epi = (c_epi*)op->epi;
            const bool has_ph = epi != nullptr && epi->n_ph > 0;
            float2* Wl = reinterpret_cast<float2*>(Lraw);  // 64 entries
            ColFactor<float>* Fl = reinterpret_cast<ColFactor<float>*>(Lraw + 32 + w * 64);  // per wave, 64
            row_sums(M, d, std::sqrt(__builtin_ldexp(1.0, -op->n)), Wl);
            __syncthreads();
            const StageGeom& sg = op->sg;
            // tile index tau -> (y over the targets, column index): linear over
            // OR, so the lane's, the chunk's and bit 0's parts are taken apart
            auto y_of = [&](int tau) {
                int y = 0;
                for (int m = 0; m < k; ++m) y |= ((tau >> sg.tpos[m]) & 1) << m;
                return y;
            };
            auto c_of = [&](int tau) {
                int c = 0;
                for (int b = 0; b < cb; ++b) c |= ((tau >> sg.cpos[b]) & 1) << b;
                return c;
            };
            const int yl = y_of(ln << 1), cl = c_of(ln << 1), y1 = y_of(1), c1 = c_of(1);
            // per chunk bit (tile bits 7..10): its row / column index bit and state offset
            int ych[4], cch[4];
            uint64_t och[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                ych[b] = y_of(128 << b);
                cch[b] = c_of(128 << b);
                och[b] = uint64_t(1) << sg.tb[7 + b];
            }
            uint64_t lane_off = 0;
#pragma unroll
            for (int b = 0; b < 6; ++b)
                if ((ln >> b) & 1) lane_off |= uint64_t(1) << sg.tb[b + 1];
            uint64_t cstate = 0;  // state bits of column `lane` (its factor is this lane's to compute)
            for (int b = 0; b < cb; ++b)
                if ((ln >> b) & 1) cstate |= uint64_t(1) << sg.tb[sg.cpos[b]];
            g_vf4* p4 = reinterpret_cast<g_vf4*>(psi);
            for (uint64_t t = item.tile0 + w; t < t_end; t += WAVES) {
                const uint64_t tb0 = tile_base<11>(t, sg);
                if (ln < (1 << cb)) {
                    ColFactor<float> f{0u, 0u, 1.0f, 0.0f};
                    if (epi != nullptr) f = col_factor<float>(epi, tb0 | cstate);
                    Fl[ln] = f;
                }
                wave_lds_fence();
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    int yi = 0, ci = 0;  // uniform
                    uint64_t o = tb0 | lane_off;
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        if ((i >> b) & 1) {
                            yi |= ych[b];
                            ci |= cch[b];
                            o |= och[b];
                        }
                    vf4 v;
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const int y = yl | yi | (b ? y1 : 0), c = cl | ci | (b ? c1 : 0);
                        const float2 a = Wl[y];
                        const ColFactor<float> f = Fl[c];
                        float re = a.x, im = a.y;
                        apply_factor(re, im, f, (uint32_t)y, has_ph);
                        v[2 * b] = re;
                        v[2 * b + 1] = im;
                    }
                    p4[o >> 1] = v;  // linear chunk i of the tile
                }
                wave_lds_fence();
            }
        } else {
            // initialisation: tile t is amplitudes [t 2^11, (t + 1) 2^11)
            // 2^(-n/2): a power of two, times 1/sqrt(2) for odd n (both exact scalings of a rounded constant)
            const float val = op->kind == 1 ? 0.0f
                                            : __builtin_ldexpf((op->n & 1) ? 0.70710678118654752440f : 1.0f,
                                                               -(op->n >> 1));
            g_vf4* p4 = reinterpret_cast<g_vf4*>(psi);
            for (uint64_t t = item.tile0 + w; t < t_end; t += WAVES) {
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const uint64_t q = (t << 10) + (uint64_t)(i * 64 + lane);  // index of an amplitude pair
                    vf4 v = {val, 0.0f, val, 0.0f};
                    if (op->kind == 1 && q == 0) v.x = 1.0f;
                    p4[q] = v;
                }
            }
        }
        // every wave waits until its stores are complete in L2; after the
        // barrier, thread 0's device-scope release (an L2 write-back, then the
        // counter) publishes them all. A release fence in every wave would
        // write the L2 back once per wave, which costs more than the tiles.
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        prev = circ;
    }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t n, uint32_t v) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------ cluster: vector ALU
// One column per thread; the matrix M[y][x] (complex) sits in LDS and is read
// as a broadcast. Used for small k and for states too small for a wave tile.
template <typename T, int K>
__global__ __launch_bounds__(256) void k_cluster_valu(typename Cplx<T>::type* __restrict__ psi,
                                                      const typename Cplx<T>::type* __restrict__ M,
                                                      const EpiDesc* __restrict__ epi, ClusterGeom g) {
    using V = typename Cplx<T>::type;
    constexpr int D = 1 << K;
    __shared__ V Ms[D * D];
    for (int i = threadIdx.x; i < D * D; i += 256) Ms[i] = M[i];
    __syncthreads();
    const bool has_epi = epi != nullptr;
    const bool has_ph = has_epi && epi->n_ph > 0;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t c = (uint64_t)blockIdx.x * 256 + threadIdx.x; c < g.ncols; c += stride) {
        const uint64_t base = deposit_cols<K>(c, g);
        V v[D];
#pragma unroll
        for (int x = 0; x < D; ++x) v[x] = psi[base | target_off<K>(x, g)];
        ColFactor<T> f{0u, 0u, T(1), T(0)};
        if (has_epi) f = col_factor<T>(epi, base);
#pragma unroll
        for (int y = 0; y < D; ++y) {
            T ar = 0, ai = 0;
#pragma unroll
            for (int x = 0; x < D; ++x) {
                const V m = Ms[y * D + x];
                ar += m.x * v[x].x - m.y * v[x].y;
                ai += m.x * v[x].y + m.y * v[x].x;
            }
            if (has_epi) apply_factor(ar, ai, f, (uint32_t)y, has_ph);
            V o;
            o.x = ar;
            o.y = ai;
            psi[base | target_off<K>(y, g)] = o;
        }
    }
}

// Two- and three-qubit clusters. With one column per thread, targets among
// the lowest state bits put lanes 2^k amplitudes apart, so each load
// instruction spreads over 2^k times the cache lines it uses, and a thread
// that holds its column and the matrix limits occupancy. Here a wave tile is
// 64 columns: the k targets and the 6 lowest non-target bits, whose lowest 6
// positions are always state bits 0..5. Chunk x of the tile (tau = 64 x +
// lane) is one contiguous run of 64 amplitudes; LDS hands each thread its
// column, then takes the results back for contiguous stores. STATS (float
// only): also sum p, p^2 and -p ln p of the stored amplitudes into part (per
// work-group), as the matrix-core kernels' STATS forms do.
template <typename T, int K, bool STATS = false>
__global__ __launch_bounds__(256) void k_cluster_valu_staged(typename Cplx<T>::type* __restrict__ psi,
                                                             const typename Cplx<T>::type* __restrict__ M,
                                                             const EpiDesc* __restrict__ epi, StageGeom sg,
                                                             uint64_t tiles, double* __restrict__ part) {
    static_assert(!STATS || std::is_same<T, float>::value, "sums of float states only");
    using V = typename Cplx<T>::type;
    constexpr int D = 1 << K, RS = D + 1;  // LDS row of a column, padded
    __shared__ V Ms[D * D];
    __shared__ V Ls[4][64 * RS];
    for (int i = threadIdx.x; i < D * D; i += 256) Ms[i] = M[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    V* L = Ls[threadIdx.x >> 6];
    // element tau = 64 x + lane: its column (bits cpos) and target index (bits tpos)
    int yl = 0, cl = 0, yx[D], cx[D];
#pragma unroll
    for (int m = 0; m < K; ++m)
        if (sg.tpos[m] < 6) yl |= ((lane >> sg.tpos[m]) & 1) << m;
#pragma unroll
    for (int b = 0; b < 6; ++b)
        if (sg.cpos[b] < 6) cl |= ((lane >> sg.cpos[b]) & 1) << b;
#pragma unroll
    for (int x = 0; x < D; ++x) {
        yx[x] = 0;
        cx[x] = 0;
#pragma unroll
        for (int m = 0; m < K; ++m)
            if (sg.tpos[m] >= 6) yx[x] |= ((x >> (sg.tpos[m] - 6)) & 1) << m;
#pragma unroll
        for (int b = 0; b < 6; ++b)
            if (sg.cpos[b] >= 6) cx[x] |= ((x >> (sg.cpos[b] - 6)) & 1) << b;
    }
    // state offset of this thread's column (lane = column inside the tile)
    uint64_t coff = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b)
        if ((lane >> b) & 1) coff |= uint64_t(1) << sg.tb[sg.cpos[b]];
    const bool has_epi = epi != nullptr;
    const bool has_ph = has_epi && epi->n_ph > 0;
    double sv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint64_t tile = (uint64_t)xcd_block() * 4 + (threadIdx.x >> 6); tile < tiles;
         tile += (uint64_t)gridDim.x * 4) {
        const uint64_t tb0 = tile_base<K + 6>(tile, sg);
        V v[D];
#pragma unroll
        for (int x = 0; x < D; ++x) v[x] = psi[tb0 | sg.ioff[x] | (uint64_t)lane];
#pragma unroll
        for (int x = 0; x < D; ++x) L[(cl | cx[x]) * RS + (yl | yx[x])] = v[x];
        wave_lds_fence();
#pragma unroll
        for (int x = 0; x < D; ++x) v[x] = L[lane * RS + x];
        ColFactor<T> f{0u, 0u, T(1), T(0)};
        if (has_epi) f = col_factor<T>(epi, tb0 | coff);
#pragma unroll
        for (int y = 0; y < D; ++y) {
            T ar = 0, ai = 0;
#pragma unroll
            for (int x = 0; x < D; ++x) {
                const V m = Ms[y * D + x];
                ar += m.x * v[x].x - m.y * v[x].y;
                ai += m.x * v[x].y + m.y * v[x].x;
            }
            if (has_epi) apply_factor(ar, ai, f, (uint32_t)y, has_ph);
            if constexpr (STATS) stats_acc_f(sv, ar, ai);
            V o;
            o.x = ar;
            o.y = ai;
            L[lane * RS + y] = o;  // a thread reads and writes only its own row here
        }
        wave_lds_fence();
#pragma unroll
        for (int x = 0; x < D; ++x) psi[tb0 | sg.ioff[x] | (uint64_t)lane] = L[(cl | cx[x]) * RS + (yl | yx[x])];
        wave_lds_fence();  // the next tile's writes come after these reads
    }
    if constexpr (STATS) block_reduce_store(sv, 3, 0u, part + blockIdx.x * 8);  // every thread gets here
}

// ------------------------------------------------------------ diagonal pass
// Every amplitude times the diagonal factor of its index (Sec. 3.5: diagonal
// gates need no gather). A wave covers windows of 128 consecutive amplitudes
// (2 per lane, 16-byte accesses), U neighbouring windows per step, all loaded
// before any factor is applied. The index splits into lo (bits 0..6, fixed per
// lane) and hi (the window, uniform per wave): terms of lo bits only are
// per-lane constants; CZ pairs with one bit in each half give a sign mask over
// lo. The hi part (sign, mask and phase) costs a loop over every gate of the
// pass, too much per window, so a wave takes runs of 64 windows: each lane
// forms the hi part of one window of the run and the window reads it from that
// lane. The descriptor lists the pairs in `cc` and the phases in `ph`.
template <typename T>
__device__ __forceinline__ void load_pair(const typename Cplx<T>::type* p, typename Cplx<T>::type (&v)[2]) {
    v[0] = p[0];
    v[1] = p[1];
}
template <>
__device__ __forceinline__ void load_pair<float>(const float2* p, float2 (&v)[2]) {
    const float4 w = *reinterpret_cast<const float4*>(p);  // p is 16-byte aligned (even index)
    v[0] = make_float2(w.x, w.y);
    v[1] = make_float2(w.z, w.w);
}
template <typename T>
__device__ __forceinline__ void store_pair(typename Cplx<T>::type* p, const typename Cplx<T>::type (&v)[2]) {
    p[0] = v[0];
    p[1] = v[1];
}
template <>
__device__ __forceinline__ void store_pair<float>(float2* p, const float2 (&v)[2]) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
}

template <typename T, int U>
__global__ __launch_bounds__(256) void k_diag(typename Cplx<T>::type* __restrict__ psi, int n,
                                              const EpiDesc* __restrict__ e) {
    using V = typename Cplx<T>::type;
    constexpr int LO = 7;         // amplitude index bits inside a window
    constexpr int RB = 6;         // a wave takes runs of 2^RB windows, one per lane
    constexpr int R = 1 << RB;
    const int lane = threadIdx.x & 63;
    const int np = e->n_cc, nph = e->n_ph;
    // per-lane constants: the factor of the two lo indices of this lane
    uint32_t sgn_lo[2] = {0u, 0u};
    double plr[2] = {1.0, 1.0}, pli[2] = {0.0, 0.0};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t lo = 2 * lane + h;
        for (int i = 0; i < np; ++i) {
            const int a = e->cc[i][0], b = e->cc[i][1];
            if (a < LO && b < LO) sgn_lo[h] ^= (lo >> a) & (lo >> b) & 1u;
        }
        for (int i = 0; i < nph; ++i) {
            const int q = e->ph_q[i];
            if (q < LO && ((lo >> q) & 1u)) {
                const double c = e->ph[i][0], sn = e->ph[i][1];
                const double r = plr[h] * c - pli[h] * sn;
                pli[h] = plr[h] * sn + pli[h] * c;
                plr[h] = r;
            }
        }
    }
    const uint64_t N = uint64_t(1) << n;
    const uint64_t nwin = (n >= LO) ? (uint64_t(1) << (n - LO)) : 1;
    const uint64_t nrun = (nwin + R - 1) >> RB;
    const uint64_t rstride = (uint64_t)gridDim.x * 4;
    for (uint64_t run = (uint64_t)xcd_block() * 4 + (threadIdx.x >> 6); run < nrun; run += rstride) {
        // lane j forms the hi part of the factor of window j of the run: the
        // sign of CZ pairs on hi bits, the sign mask over lo of pairs with
        // one bit in each half, and the phases of hi bits
        const uint64_t hi = ((run << RB) | (uint64_t)lane) << LO;
        uint32_t sgn_hi = 0u, wmask = 0u;
        double phr = 1.0, phi = 0.0;
        for (int i = 0; i < np; ++i) {
            const int a = e->cc[i][0], b = e->cc[i][1];
            if (a >= LO && b >= LO) sgn_hi ^= (uint32_t)((hi >> a) & (hi >> b) & 1);
            else if (a < LO && b >= LO) wmask ^= (uint32_t)((hi >> b) & 1) << a;
            else if (b < LO && a >= LO) wmask ^= (uint32_t)((hi >> a) & 1) << b;
        }
        for (int i = 0; i < nph; ++i) {
            const int q = e->ph_q[i];
            if (q >= LO && ((hi >> q) & 1)) {
                const double c = e->ph[i][0], sn = e->ph[i][1];
                const double r = phr * c - phi * sn;
                phi = phr * sn + phi * c;
                phr = r;
            }
        }
        const int sw = (int)(wmask | (sgn_hi << LO));  // wmask has bits 0..6 only
        const uint64_t left = nwin - (run << RB);
        const int wend = left < (uint64_t)R ? (int)left : R;  // uniform
        for (int w0 = 0; w0 < wend; w0 += U) {
            V v[U][2];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t i0 = (((run << RB) | (uint64_t)(w0 + u)) << LO) | (uint64_t)(2 * lane);
                // windows past the end, and lanes past the end of states of fewer than 7 qubits
                if (w0 + u < wend && i0 < N) load_pair<T>(psi + i0, v[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t i0 = (((run << RB) | (uint64_t)(w0 + u)) << LO) | (uint64_t)(2 * lane);
                if (w0 + u >= wend || i0 >= N) continue;
                const uint32_t swu = (uint32_t)__builtin_amdgcn_readlane(sw, w0 + u);
                const double hr = readlane_f64(phr, w0 + u), hq = readlane_f64(phi, w0 + u);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const uint32_t lo = 2 * lane + h;
                    const bool neg = ((sgn_lo[h] ^ (swu >> LO) ^ (uint32_t)__popc(lo & swu & 0x7fu)) & 1u) != 0;
                    const T fr = (T)(hr * plr[h] - hq * pli[h]);
                    const T fi = (T)(hr * pli[h] + hq * plr[h]);
                    const T re = v[u][h].x * fr - v[u][h].y * fi;
                    const T im = v[u][h].x * fi + v[u][h].y * fr;
                    v[u][h].x = neg ? -re : re;
                    v[u][h].y = neg ? -im : im;
                }
                store_pair<T>(psi + i0, v[u]);
            }
        }
    }
}

// ------------------------------------------------------------ per-gate kernels
// A single-qubit gate on the pairs (i, i + 2^q) with bit q of i clear (Sec. 2).
template <typename T>
__global__ __launch_bounds__(256) void k_gate1q(typename Cplx<T>::type* __restrict__ psi, int q, T m0r,
                                                T m0i, T m1r, T m1i, T m2r, T m2i, T m3r, T m3i,
                                                uint64_t npairs) {
    using V = typename Cplx<T>::type;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    const uint64_t bit = uint64_t(1) << q;
    for (uint64_t p = (uint64_t)xcd_block() * 256 + threadIdx.x; p < npairs; p += stride) {
        const uint64_t i = insert_zero(p, q);
        const V a = psi[i], b = psi[i | bit];
        V o0, o1;
        o0.x = (m0r * a.x - m0i * a.y) + (m1r * b.x - m1i * b.y);
        o0.y = (m0r * a.y + m0i * a.x) + (m1r * b.y + m1i * b.x);
        o1.x = (m2r * a.x - m2i * a.y) + (m3r * b.x - m3i * b.y);
        o1.y = (m2r * a.y + m2i * a.x) + (m3r * b.y + m3i * b.x);
        psi[i] = o0;
        psi[i | bit] = o1;
    }
}

// A diagonal single-qubit gate diag(1, e^{i phi}): only amplitudes with bit q set change.
template <typename T>
__global__ __launch_bounds__(256) void k_phase1q(typename Cplx<T>::type* __restrict__ psi, int q, T cr,
                                                 T ci, uint64_t nhalf) {
    using V = typename Cplx<T>::type;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    const uint64_t bit = uint64_t(1) << q;
    for (uint64_t p = (uint64_t)xcd_block() * 256 + threadIdx.x; p < nhalf; p += stride) {
        const uint64_t i = insert_zero(p, q) | bit;
        const V a = psi[i];
        V o;
        o.x = a.x * cr - a.y * ci;
        o.y = a.x * ci + a.y * cr;
        psi[i] = o;
    }
}

// CZ(a, b), a < b: negate the amplitudes with both bits set.
template <typename T>
__global__ __launch_bounds__(256) void k_cz(typename Cplx<T>::type* __restrict__ psi, int a, int b,
                                            uint64_t nquarter) {
    using V = typename Cplx<T>::type;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    const uint64_t m = (uint64_t(1) << a) | (uint64_t(1) << b);
    for (uint64_t p = (uint64_t)xcd_block() * 256 + threadIdx.x; p < nquarter; p += stride) {
        const uint64_t i = insert_zero(insert_zero(p, a), b) | m;
        V v = psi[i];
        v.x = -v.x;
        v.y = -v.y;
        psi[i] = v;
    }
}

// ------------------------------------------------------------ initialisation
template <typename T>
__global__ __launch_bounds__(256) void k_init(typename Cplx<T>::type* __restrict__ psi, uint64_t count,
                                              int mode, T val) {
    using V = typename Cplx<T>::type;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += stride) {
        V v;
        v.x = (mode == 0) ? (i == 0 ? T(1) : T(0)) : val;
        v.y = T(0);
        psi[i] = v;
    }
}

// ------------------------------------------------------------ initialisation folded into the first cluster
// The uniform state (the skipped leading H layer, Sec. 3.6) is a product state,
// and so is the first cluster's result on it: amplitude i is
// w[y(i)] = 2^(-n/2) sum_x M[y(i)][x], y(i) the target bits of i, times the
// cluster's diagonal epilogue factor. One write-only pass replaces the
// initialisation and the first cluster's read-and-write pass. M is the plain
// complex128 matrix; w is summed in float64 and rounded once.
template <typename T, int K>
__global__ __launch_bounds__(256) void k_init_cluster(typename Cplx<T>::type* __restrict__ psi, ClusterGeom g,
                                                      const double2* __restrict__ M,
                                                      const EpiDesc* __restrict__ epi, double amp) {
    using V = typename Cplx<T>::type;
    constexpr int D = 1 << K;
    __shared__ double2 w[D];
    __shared__ uint64_t toff[D];
    row_sums(M, D, amp, w);
    if ((int)threadIdx.x < D) {
        uint64_t o = 0;
        for (int m = 0; m < K; ++m)
            if ((threadIdx.x >> m) & 1) o |= uint64_t(1) << g.t[m];
        toff[threadIdx.x] = o;
    }
    __syncthreads();
    const bool has_epi = epi != nullptr;
    const bool has_ph = has_epi && epi->n_ph > 0;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    if constexpr (sizeof(T) == 4) {
        // float: 16-byte stores. With qubit 0 a target, amplitudes y, y + 1 of a
        // column are neighbours; otherwise columns 2c, 2c + 1 differ in bit 0 only
        // and a thread writes both, side by side.
        if (g.t[0] == 0) {
            for (uint64_t c = (uint64_t)xcd_block() * 256 + threadIdx.x; c < g.ncols; c += stride) {
                const uint64_t base = deposit_cols<K>(c, g);
                ColFactor<T> f{0u, 0u, T(1), T(0)};
                if (has_epi) f = col_factor<T>(epi, base);
#pragma unroll 8
                for (int y = 0; y < D; y += 2) {
                    const double2 v0 = w[y], v1 = w[y + 1];
                    T r0 = (T)v0.x, i0 = (T)v0.y, r1 = (T)v1.x, i1 = (T)v1.y;
                    if (has_epi) {
                        apply_factor(r0, i0, f, (uint32_t)y, has_ph);
                        apply_factor(r1, i1, f, (uint32_t)(y + 1), has_ph);
                    }
                    *reinterpret_cast<vf4*>(psi + (base | toff[y])) = vf4{r0, i0, r1, i1};
                }
            }
            return;
        }
        if (g.ncols >= 2) {
            for (uint64_t c = (uint64_t)xcd_block() * 256 + threadIdx.x; c < g.ncols / 2; c += stride) {
                const uint64_t base = deposit_cols<K>(2 * c, g);  // bit 0 clear; column 2c + 1 is base | 1
                ColFactor<T> f0{0u, 0u, T(1), T(0)}, f1 = f0;
                if (has_epi) {
                    f0 = col_factor<T>(epi, base);
                    f1 = col_factor<T>(epi, base | 1);
                }
#pragma unroll 8
                for (int y = 0; y < D; ++y) {
                    const double2 v = w[y];
                    T r0 = (T)v.x, i0 = (T)v.y, r1 = r0, i1 = i0;
                    if (has_epi) {
                        apply_factor(r0, i0, f0, (uint32_t)y, has_ph);
                        apply_factor(r1, i1, f1, (uint32_t)y, has_ph);
                    }
                    *reinterpret_cast<vf4*>(psi + (base | toff[y])) = vf4{r0, i0, r1, i1};
                }
            }
            return;
        }
    }
    // one thread per column (assignment of the non-target bits): its diagonal
    // factor once, then the column's 2^k amplitudes
    for (uint64_t c = (uint64_t)xcd_block() * 256 + threadIdx.x; c < g.ncols; c += stride) {
        const uint64_t base = deposit_cols<K>(c, g);
        ColFactor<T> f{0u, 0u, T(1), T(0)};
        if (has_epi) f = col_factor<T>(epi, base);
#pragma unroll
        for (int y = 0; y < D; ++y) {
            const double2 v = w[y];
            T re = (T)v.x, im = (T)v.y;
            if (has_epi) apply_factor(re, im, f, (uint32_t)y, has_ph);
            V o;
            o.x = re;
            o.y = im;
            psi[base | toff[y]] = o;
        }
    }
}

// ------------------------------------------------------------ cluster-matrix builder
// One work-group (64 threads) per cluster; a 7-qubit cluster takes
// kBuildParts7 of them, each with 32 of its columns. Thread x owns column x of
// the cluster matrix: it starts from the basis vector e_x of the 2^k space
// and applies the cluster's gates in order, in float64 (the matrix is reused
// for all 2^(n-k) columns of the state, Sec. 3.2, so building it is cheap).
// The result is then written in the layout of the kernel that will apply it.
// The columns are interleaved in LDS (real / imaginary part c of entry i of
// local column x at (2 i + c) * cs + x, cs = the work-group's column count):
// the threads touch consecutive words at every step (a column per contiguous
// block put them a multiple of 256 words apart, all in one bank).
// 4 waves per matrix (a quarter of a 7-qubit matrix): each column is worked
// on by kBuildThreads / (columns held) threads, every gate split over them
constexpr int kBuildThreads = 256;
constexpr int kBuildCols = 64;  // columns held for k <= 6 (32 for k = 7)
// entry i of a column: its doubles lie cs apart (the columns side by side)
__device__ __forceinline__ double& BV(double* v, int i, int cs) { return v[i * cs]; }

__global__ __launch_bounds__(kBuildThreads) void k_build(const BuildOp* __restrict__ ops,
                                                         const BuildGate* __restrict__ gates,
                                                         const double* __restrict__ dense, char* __restrict__ mat_base) {
    // 2 doubles per entry, 2^k entries per column, cs columns: 8192 doubles for k <= 6 and for k = 7
    __shared__ double Vs[64 * 2 * kBuildCols];
    __shared__ double Ws[64 * 2 * kBuildCols];
    const BuildOp op = ops[blockIdx.x];
    const int k = op.k, D = 1 << k, t = threadIdx.x;
    const int cs = k == 7 ? 32 : kBuildCols;   // columns held by this work-group
    const int x0 = k == 7 ? 32 * op.part : 0;  // its first column
    // thread t: column c, share sub of T
    const int T = kBuildThreads / cs, c = t % cs, sub = t / cs;
    const bool act = c < D;
    double* v = Vs + c;
    double* w = Ws + c;
    if (act)
        for (int i = sub; i < 2 * D; i += T) BV(v, i, cs) = i == 2 * (x0 + c) ? 1.0 : 0.0;
    __syncthreads();
    for (int gi = 0; gi < op.n_gates; ++gi) {
        const BuildGate bg = gates[op.gate0 + gi];
        if (bg.kind == G_CZ) {
            const int m = (1 << bg.pos[0]) | (1 << bg.pos[1]);
            if (act)
                for (int i = sub; i < D; i += T)
                    if ((i & m) == m) {
                        BV(v, 2 * i, cs) = -BV(v, 2 * i, cs);
                        BV(v, 2 * i + 1, cs) = -BV(v, 2 * i + 1, cs);
                    }
        } else if (bg.kind == G_DENSE) {
            // for each assignment `rest` of the entry bits outside the gate,
            // the dd entries rest | dep(xl) are multiplied by the gate's
            // matrix; 16 outputs at a time (one work item, dealt round-robin
            // to the column's threads) are summed in registers (dep puts bit j
            // of a gate index at the gate's position j)
            const int dq = bg.nq, dd = 1 << dq;
            const double* u = dense + bg.dense_off;
            int pm = 0;
            for (int j = 0; j < dq; ++j) pm |= 1 << bg.pos[j];
            auto dep = [&](int xl) {
                int o = 0;
                for (int j = 0; j < dq; ++j) o |= ((xl >> j) & 1) << bg.pos[j];
                return o;
            };
            if (act) {
                int item = 0;
                for (int rest = 0; rest < D; rest = ((rest | pm) + 1) & ~pm) {
                    for (int y0 = 0; y0 < dd; y0 += 16, ++item) {
                        if (item % T != sub) continue;
                        double sr[16], si[16];
#pragma unroll
                        for (int t2 = 0; t2 < 16; ++t2) sr[t2] = si[t2] = 0.0;
                        for (int xl = 0; xl < dd; ++xl) {
                            const int src = rest | dep(xl);
                            const double vr = BV(v, 2 * src, cs), vi = BV(v, 2 * src + 1, cs);
#pragma unroll
                            for (int t2 = 0; t2 < 16; ++t2) {
                                if (y0 + t2 >= dd) break;
                                const double mr = u[2 * ((y0 + t2) * dd + xl)], mi = u[2 * ((y0 + t2) * dd + xl) + 1];
                                sr[t2] += mr * vr - mi * vi;
                                si[t2] += mr * vi + mi * vr;
                            }
                        }
#pragma unroll
                        for (int t2 = 0; t2 < 16; ++t2) {
                            if (y0 + t2 >= dd) break;
                            const int dst = rest | dep(y0 + t2);
                            BV(w, 2 * dst, cs) = sr[t2];
                            BV(w, 2 * dst + 1, cs) = si[t2];
                        }
                    }
                }
            }
            __syncthreads();
            if (act)
                for (int i = sub; i < 2 * D; i += T) BV(v, i, cs) = BV(w, i, cs);
        } else {
            double m[8];
            gate2x2(bg.kind, bg.theta, m);
            const int a = bg.pos[0], lo = (1 << a) - 1;
            if (act)
                for (int pr = sub; pr < D / 2; pr += T) {
                    const int i = ((pr & ~lo) << 1) | (pr & lo), j = i | (1 << a);
                    const double ar = BV(v, 2 * i, cs), ai = BV(v, 2 * i + 1, cs), br = BV(v, 2 * j, cs),
                                 bi = BV(v, 2 * j + 1, cs);
                    BV(v, 2 * i, cs) = (m[0] * ar - m[1] * ai) + (m[2] * br - m[3] * bi);
                    BV(v, 2 * i + 1, cs) = (m[0] * ai + m[1] * ar) + (m[2] * bi + m[3] * br);
                    BV(v, 2 * j, cs) = (m[4] * ar - m[5] * ai) + (m[6] * br - m[7] * bi);
                    BV(v, 2 * j + 1, cs) = (m[4] * ai + m[5] * ar) + (m[6] * bi + m[7] * br);
                }
        }
        __syncthreads();
    }
    __syncthreads();
    // M[y][x] = entry y of column x (a column this work-group holds)
    auto Mre = [&](int y, int xx) { return Vs[(2 * y) * cs + (xx - x0)]; };
    auto Mim = [&](int y, int xx) { return Vs[(2 * y + 1) * cs + (xx - x0)]; };
    // k <= 6 layouts: lane l = t % 64 of the MFMA operand, the (row block,
    // step) pairs dealt to the 4 waves
    const int lane = t & 63, wv = t >> 6, NW = kBuildThreads / 64;
    // entry (R, Kc) of the real-split matrix [[Re, -Im], [Im, Re]]
    auto Ars = [&](int y, int a, int xx, int b) {
        const double re = Mre(y, xx), im = Mim(y, xx);
        return (a == b) ? re : (a == 0 ? -im : im);
    };
    char* out = mat_base + op.out_off;
    if (op.layout == LAYOUT_PLAIN) {
        const int nc = D < cs ? D : cs;  // columns held
        for (int e = t; e < D * nc; e += kBuildThreads) {
            const int y = e / nc, xc = x0 + e % nc;
            if (op.is_double) {
                reinterpret_cast<double2*>(out)[y * D + xc] = make_double2(Mre(y, xc), Mim(y, xc));
            } else {
                reinterpret_cast<float2*>(out)[y * D + xc] = make_float2((float)Mre(y, xc), (float)Mim(y, xc));
            }
        }
    } else if (op.layout == LAYOUT_SPLIT7) {
        // k = 7: fp16 halves of 16 Re M and 16 Im M for v_mfma_f32_32x32x16_f16
        // (k_cluster_f32_split7). Entry (rb, s, lane l, i) of each part:
        // physical row rho = l % 32 of row block rb is amplitude
        // (16 rb + 4 (rho / 8) + rho % 4) | ((rho / 4) % 2) << 6; inner element
        // i of the lanes with l / 32 = hin is amplitude (8 s + i) | hin << 6.
        // This work-group holds the columns whose bits 5, 6 equal op.part, i.e.
        // steps s with s / 4 = part % 2 and lanes with l / 32 = part / 2.
        constexpr int S7 = 8, NP7 = 4 * S7 * 64 * 8;  // halves per part
        _Float16* A = reinterpret_cast<_Float16*>(out);
        const int s_lo = 4 * (op.part & 1), hin = op.part >> 1;
        for (int e = t; e < 4 * 4 * 32 * 8; e += kBuildThreads) {
            const int i = e & 7, lr = (e >> 3) & 31, sl = (e >> 8) & 3, rb = e >> 10;
            const int s2 = s_lo + sl, l = lr | (hin << 5), rho = lr;
            const int y = (16 * rb + 4 * (rho >> 3) + (rho & 3)) | (((rho >> 2) & 1) << 6);
            const int xin = (8 * s2 + i) | (hin << 6);
            const float vr = (float)(16.0 * Mre(y, xin)), vi = (float)(16.0 * Mim(y, xin));
            const _Float16 hr = (_Float16)vr, hi = (_Float16)vi;
            const size_t at = ((size_t)(rb * S7 + s2) * 64 + l) * 8 + i;
            A[at] = hr;
            A[NP7 + at] = (_Float16)(vr - (float)hr);
            A[2 * NP7 + at] = hi;
            A[3 * NP7 + at] = (_Float16)(vi - (float)hi);
        }
    } else if (op.layout == LAYOUT_MFMA32F) {
        // entry (rb, s, lane l): row rho = l % 32 of row block rb, inner index 2 s + l / 32
        const int RB = 2 * D / 32, S = D, l = lane;
        const int rho = l & 31, hin = l >> 5;
        float* A = reinterpret_cast<float*>(out);
        for (int it = wv; it < RB * S; it += NW) {
            const int rb = it / S, s = it % S;
            const int jout = rb * 8 + 2 * (rho >> 3) + ((rho & 3) >> 1);
            const int hout = (rho >> 2) & 1;
            const int y = jout | (hout << (k - 1)), a = rho & 1;
            const int xin = (s >> 1) | (hin << (k - 1)), b = s & 1;
            A[(rb * S + s) * 64 + l] = (float)Ars(y, a, xin, b);
        }
    } else if (op.layout == LAYOUT_GAUSS32F) {
        // k = 6: three 64 x 64 real matrices P = 0: Re M, 1: Im M, 2: Re M + Im M,
        // for v_mfma_f32_16x16x4_f32. Entry (P, rb, s, lane l): physical row
        // i = l % 16 of row block rb, inner index s | (l / 16) << 4. The result
        // of physical row i lands in register i % 4 of the lanes with l / 16 =
        // i / 4, which own amplitude (4 rb + i % 4) | (i / 4) << 4.
        const int l = lane, i = l & 15, qin = l >> 4;
        float* A = reinterpret_cast<float*>(out);
        for (int it = wv; it < 4 * 16; it += NW) {
            const int rb = it / 16, s2 = it % 16;
            const int y = (4 * rb + (i & 3)) | ((i >> 2) << 4);
            const int xin = s2 | (qin << 4);
            const double re = Mre(y, xin), im = Mim(y, xin);
            A[((0 * 4 + rb) * 16 + s2) * 64 + l] = (float)re;
            A[((1 * 4 + rb) * 16 + s2) * 64 + l] = (float)im;
            A[((2 * 4 + rb) * 16 + s2) * 64 + l] = (float)(re + im);
        }
    } else if (op.layout == LAYOUT_SPLIT16F) {
        // k = 5 or 6, fp16 halves of 16 x the real-split matrix for
        // v_mfma_f32_32x32x16_f16: RB = 2^(k-4) row blocks, S = 2^(k-3) steps
        // of 16 inner indices. Entry (rb, s, lane l, i): physical row rho =
        // l % 32 of row block rb (result rows as in LAYOUT_MFMA32F), inner index
        // float 8 s + i of the lanes with l / 32 = hin, i.e. component i % 2 of
        // amplitude (4 s + i / 2) | hin << (k - 1). hi block, then lo block.
        const int l = lane, rho = l & 31, hin = l >> 5;
        const int RB = 1 << (k - 4), S = 1 << (k - 3);
        _Float16* Ahi = reinterpret_cast<_Float16*>(out);
        _Float16* Alo = Ahi + (size_t)RB * S * 64 * 8;
        for (int it = wv; it < RB * S; it += NW) {
            const int rb = it / S, s2 = it % S;
            const int jout = rb * 8 + 2 * (rho >> 3) + ((rho & 3) >> 1);
            const int hout = (rho >> 2) & 1;
            const int y = jout | (hout << (k - 1)), a = rho & 1;
            for (int i = 0; i < 8; ++i) {
                const int xin = (4 * s2 + (i >> 1)) | (hin << (k - 1)), b = i & 1;
                const float v = (float)(16.0 * Ars(y, a, xin, b));
                const _Float16 hi = (_Float16)v;
                const size_t at = ((size_t)(rb * S + s2) * 64 + l) * 8 + i;
                Ahi[at] = hi;
                Alo[at] = (_Float16)(v - (float)hi);
            }
        }
    } else {  // LAYOUT_MFMA16D
        // entry (rb, s, lane l): row rho = l % 16 of row block rb, inner index 4 s + l / 16.
        // The result row rho lands in register rho / 4 of the lanes with l / 16 = rho % 4.
        const int RB = 2 * D / 16, S = 2 * D / 4, l = lane;
        const int rho = l & 15, qin = l >> 4;
        double* A = reinterpret_cast<double*>(out);
        for (int it = wv; it < RB * S; it += NW) {
            const int rb = it / S, s = it % S;
            const int qout = rho & 3, ir = rho >> 2;
            const int y = (rb * 2 + (ir >> 1)) | (qout << (k - 2)), a = ir & 1;
            const int xin = (s >> 1) | (qin << (k - 2)), b = s & 1;
            A[(rb * S + s) * 64 + l] = Ars(y, a, xin, b);
        }
    }
}

// ------------------------------------------------------------ float64 reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Block reduction of up to 8 values; slot i is summed unless bit i of maxmask is set.
__device__ void block_reduce_store(double (&vals)[8], int nv, unsigned maxmask, double* out) {
    __shared__ double sh[4][8];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = 0; i < nv; ++i) vals[i] = ((maxmask >> i) & 1) ? wave_max(vals[i]) : wave_sum(vals[i]);
    if (lane == 0)
        for (int i = 0; i < nv; ++i) sh[w][i] = vals[i];
    __syncthreads();
    if (threadIdx.x < nv) {
        const int i = threadIdx.x;
        double r = sh[0][i];
        for (int ww = 1; ww < 4; ++ww) r = ((maxmask >> i) & 1) ? fmax(r, sh[ww][i]) : r + sh[ww][i];
        out[i] = r;
    }
}

// The grid-stride loops below are unrolled by kRedU with all loads of a
// round issued before any arithmetic: with one load in flight per lane the
// reductions were bound by memory latency, not bandwidth. Every load
// instruction stays coalesced (lane l reads element i + l, round after round).
constexpr int kRedU = 8;

template <typename T, typename P>
__global__ __launch_bounds__(256) void k_stats(const typename Cplx<T>::type* __restrict__ psi, uint64_t count,
                                               P* __restrict__ probs, double* __restrict__ part) {
    using V = typename Cplx<T>::type;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    auto acc = [&](const V& a, uint64_t i) {
        const double pr = (double)a.x * (double)a.x + (double)a.y * (double)a.y;
        if constexpr (sizeof(T) == 4) {
            stats_acc_f(v, a.x, a.y);
        } else {
            v[0] += pr;
            v[1] += pr * pr;
            if (pr > 0.0) v[2] -= pr * log(pr);
        }
        if (probs) probs[i] = (P)pr;
    };
    uint64_t i = (uint64_t)xcd_block() * 256 + threadIdx.x;  // any bijection: partials stay per work-group
    for (; i + (kRedU - 1) * stride < count; i += kRedU * stride) {
        V a[kRedU];
#pragma unroll
        for (int u = 0; u < kRedU; ++u) a[u] = psi[i + u * stride];
#pragma unroll
        for (int u = 0; u < kRedU; ++u) acc(a[u], i + u * stride);
    }
    for (; i < count; i += stride) acc(psi[i], i);
    block_reduce_store(v, 3, 0u, part + blockIdx.x * 8);
}

template <typename T, typename R>
__global__ __launch_bounds__(256) void k_compare(const typename Cplx<T>::type* __restrict__ psi,
                                                 const typename Cplx<R>::type* __restrict__ ref, uint64_t count,
                                                 double* __restrict__ part) {
    using V = typename Cplx<T>::type;
    using W = typename Cplx<R>::type;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    auto acc = [&](const V& a, const W& r) {
        const double ar = a.x, ai = a.y, rr = r.x, ri = r.y;
        v[0] += rr * ar + ri * ai;  // Re <ref|psi>
        v[1] += rr * ai - ri * ar;  // Im <ref|psi>
        v[2] += rr * rr + ri * ri;
        v[3] += ar * ar + ai * ai;
        const double dr = ar - rr, di = ai - ri;
        v[4] = fmax(v[4], sqrt(dr * dr + di * di));
    };
    uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    constexpr int U = kRedU / 2;
    for (; i + (U - 1) * stride < count; i += U * stride) {
        V a[U];
        W r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a[u] = psi[i + u * stride];
            r[u] = ref[i + u * stride];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc(a[u], r[u]);
    }
    for (; i < count; i += stride) acc(psi[i], ref[i]);
    block_reduce_store(v, 5, 1u << 4, part + blockIdx.x * 8);
}

// Sum (or max) the per-block partials in a fixed order: deterministic.
__global__ __launch_bounds__(256) void k_reduce_final(const double* __restrict__ part, int nblocks, int nv,
                                                      unsigned maxmask, double* __restrict__ res) {
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += 256)
        for (int i = 0; i < nv; ++i) {
            const double x = part[b * 8 + i];
            v[i] = ((maxmask >> i) & 1) ? fmax(v[i], x) : v[i] + x;
        }
    block_reduce_store(v, nv, maxmask, res);
}

// ------------------------------------------------------------ launchers
namespace {
inline unsigned grid_for(uint64_t work, unsigned per_block, unsigned cap) {
    const uint64_t b = (work + per_block - 1) / per_block;
    return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}
constexpr unsigned kStreamGrid = 8192;  // blocks of 256 threads for grid-stride streaming kernels
constexpr unsigned kPersistGrid = 2048; // work-groups of the persistent cluster kernels
constexpr unsigned kPairGrid = 256;     // one 12-wave work-group per compute unit (LDS-limited)
constexpr unsigned kStagedGrid = 256;   // one 8-wave work-group per compute unit (LDS-limited)
constexpr unsigned kSplit7Grid = 256;   // one 4-wave work-group per compute unit (LDS-limited)
}  // namespace

hipError_t launch_init(void* psi, int n, bool dbl, int mode, hipStream_t st) {
    const uint64_t cnt = uint64_t(1) << n;
    const unsigned grid = grid_for(cnt, 256, kStreamGrid);
    const double val = std::ldexp(1.0, -n) > 0 ? std::sqrt(std::ldexp(1.0, -n)) : 0.0;
    if (dbl)
        hipLaunchKernelGGL(k_init<double>, dim3(grid), dim3(256), 0, st, (double2*)psi, cnt, mode, val);
    else
        hipLaunchKernelGGL(k_init<float>, dim3(grid), dim3(256), 0, st, (float2*)psi, cnt, mode, (float)val);
    return hipGetLastError();
}

// Tile of 11 bits holding the targets of every cluster (their union plus the
// lowest other bits); sg[j] gets the tile bits and cluster j's positions.
constexpr bool kMultiSwz = true;

static void make_multi_geom(int n, int m, const int32_t (*t)[5], StageGeom* sg, int nt_want = 11) {
    uint64_t tile = 0;
    for (int j = 0; j < m; ++j)
        for (int q = 0; q < 5; ++q) tile |= uint64_t(1) << t[j][q];
    for (int b = 0; b < n && __builtin_popcountll(tile) < nt_want; ++b) tile |= uint64_t(1) << b;
    int tb[16], nt = 0;
    for (int b = 0; b < n; ++b)
        if (tile >> b & 1) tb[nt++] = b;
    for (int j = 0; j < m; ++j) {
        StageGeom& g = sg[j];
        std::memset(&g, 0, sizeof(g));
        g.nt = nt;
        for (int r = 0; r < nt; ++r) g.tb[r] = tb[r];
        int nc = 0;
        for (int r = 0; r < nt; ++r) {
            bool is_t = false;
            for (int q = 0; q < 5; ++q)
                if (tb[r] == t[j][q]) {
                    g.tpos[q] = r;
                    is_t = true;
                }
            if (!is_t) g.cpos[nc++] = r;
        }
        for (int i = 0; i < 16; ++i) {
            const uint64_t tau = uint64_t(i) << 7;
            uint64_t off = 0;
            for (int r = 0; r < nt; ++r)
                if (tau >> r & 1) off |= uint64_t(1) << tb[r];
            g.ioff[i] = off;
        }
    }
}

hipError_t launch_multi(void* psi, int n, int m, const int32_t (*targets)[5], const void* const* mats,
                        const EpiDesc* const* epis, hipStream_t st) {
    if (m < 1 || m > 2 || n < 11) return hipErrorInvalidValue;
    MultiArgs a;
    std::memset(&a, 0, sizeof(a));
    make_multi_geom(n, m, targets, a.sg);
    if (a.sg[0].nt != 11) return hipErrorInvalidValue;
    for (int j = 0; j < m; ++j) {
        a.A[j] = reinterpret_cast<const half8*>(mats[j]);
        a.epi[j] = epis[j];
        a.lowt[j] = a.sg[j].tpos[0] == 0;
    }
    const uint64_t ntiles = uint64_t(1) << (n - 11);
    MultiArgs a10 = a;
    if (m == 2 && g_pair_tile == 10) make_multi_geom(n, m, targets, a10.sg, 10);
    // the 10-bit tile needs state bit 0 (16-byte accesses of amplitude pairs)
    if (m == 2 && g_pair_tile == 10 && a10.sg[0].nt == 10 && a10.sg[0].tb[0] == 0) {
        const uint64_t nt10 = uint64_t(1) << (n - 10);
        const unsigned grid = grid_for(nt10, 12, kPairGrid);
        hipLaunchKernelGGL((k_cluster_f32_pair10<12>), dim3(grid), dim3(768), 0, st, (float2*)psi, a10, nt10);
    } else if (m == 2) {
        const unsigned grid = grid_for(ntiles, 8, kPersistGrid / 2);
        hipLaunchKernelGGL((k_cluster_f32_multi<2, 8, kMultiSwz>), dim3(grid), dim3(512), 0, st, (float2*)psi, a,
                           ntiles);
    } else {
        const unsigned grid = grid_for(ntiles, 4, kPersistGrid);
        hipLaunchKernelGGL((k_cluster_f32_multi<1, 4, kMultiSwz>), dim3(grid), dim3(256), 0, st, (float2*)psi, a,
                           ntiles);
    }
    return hipGetLastError();
}

hipError_t launch_fold2(void* psi, const ClusterGeom& g2, const void* mat2, const EpiDesc* epi2, const EpiDesc* epi1,
                        const ClusterGeom& g1, const void* mat1, int omask, int rmask, void* table,
                        hipStream_t st) {
    if (g2.k < 6 || g2.k > 7 || g2.n < 12 - (7 - g2.k) || g1.k < 1 || g1.k > g2.k) return hipErrorInvalidValue;
    if (g2.k == 7 && omask < 0) return hipErrorInvalidValue;  // a 7-qubit second cluster: the table form only
    Fold2Args f;
    std::memset(&f, 0, sizeof(f));
    f.M1 = reinterpret_cast<const double2*>(mat1);
    f.amp = std::sqrt(std::ldexp(1.0, -g2.n));
    f.k1 = g1.k;
    for (int m = 0; m < g1.k; ++m) f.t1[m] = g1.t[m];
    const StageGeom sg = make_stage_geom(g2, 5, 7);
    const uint64_t tiles = g2.ncols >> 5;
    const unsigned grid = grid_for(tiles, 8, kStagedGrid);
    if (omask >= 0) {
        const int no = __builtin_popcount((unsigned)omask), nr = __builtin_popcount((unsigned)rmask);
        const int rmax = g2.k == 7 ? kFoldTab7Rows : kFoldTabRows, mmax = (1 << g2.k) - 1;
        if (table == nullptr || omask > mmax || rmask < 0 || rmask > mmax || no > 2 || (1 << (no + nr)) > rmax)
            return hipErrorInvalidValue;
        FoldTabArgs a;
        a.M2 = reinterpret_cast<const double2*>(mat2);
        a.omask = omask;
        a.rmask = rmask;
        if (g2.k == 7) {
            hipLaunchKernelGGL(k_fold2_table<7>, dim3(1u << (no + nr)), dim3(128), 0, st, (float2*)table, a);
            const unsigned grid7 = grid_for(g2.ncols / 32, 4, 2 * kSplit7Grid);
            if (g2.t[0] == 0)
                hipLaunchKernelGGL(k_fold2t7_f32<true>, dim3(grid7), dim3(256), 0, st, (float2*)psi,
                                   (const float2*)table, epi2, epi1, g2, f, a);
            else
                hipLaunchKernelGGL(k_fold2t7_f32<false>, dim3(grid7), dim3(256), 0, st, (float2*)psi,
                                   (const float2*)table, epi2, epi1, g2, f, a);
            return hipGetLastError();
        }
        hipLaunchKernelGGL(k_fold2_table<6>, dim3(1u << (no + nr)), dim3(64), 0, st, (float2*)table, a);
        if (g2.t[0] == 0)
            hipLaunchKernelGGL(k_fold2t_f32<true>, dim3(grid), dim3(512), 0, st, (float2*)psi, (const float2*)table,
                               epi2, epi1, sg, f, a, tiles);
        else
            hipLaunchKernelGGL(k_fold2t_f32<false>, dim3(grid), dim3(512), 0, st, (float2*)psi,
                               (const float2*)table, epi2, epi1, sg, f, a, tiles);
        return hipGetLastError();
    }
    if (g2.t[0] == 0)
        hipLaunchKernelGGL(k_fold2_f32<true>, dim3(grid), dim3(512), 0, st, (float2*)psi, (const half8*)mat2, epi2,
                           epi1, sg, f, tiles);
    else
        hipLaunchKernelGGL(k_fold2_f32<false>, dim3(grid), dim3(512), 0, st, (float2*)psi, (const half8*)mat2, epi2,
                           epi1, sg, f, tiles);
    return hipGetLastError();
}

hipError_t launch_init_cluster(void* psi, bool dbl, const ClusterGeom& g, const void* mat, const EpiDesc* epi,
                               hipStream_t st) {
    const unsigned grid = grid_for(g.ncols, 256, kStreamGrid);
    const double amp = std::sqrt(std::ldexp(1.0, -g.n));
    auto go = [&](auto kc) {
        constexpr int K = decltype(kc)::value;
        if (dbl)
            hipLaunchKernelGGL((k_init_cluster<double, K>), dim3(grid), dim3(256), 0, st, (double2*)psi, g,
                               (const double2*)mat, epi, amp);
        else
            hipLaunchKernelGGL((k_init_cluster<float, K>), dim3(grid), dim3(256), 0, st, (float2*)psi, g,
                               (const double2*)mat, epi, amp);
    };
    switch (g.k) {
        case 1: go(std::integral_constant<int, 1>()); break;
        case 2: go(std::integral_constant<int, 2>()); break;
        case 3: go(std::integral_constant<int, 3>()); break;
        case 4: go(std::integral_constant<int, 4>()); break;
        case 5: go(std::integral_constant<int, 5>()); break;
        case 6: go(std::integral_constant<int, 6>()); break;
        case 7: go(std::integral_constant<int, 7>()); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_build(const BuildOp* ops, int n_ops, const BuildGate* gates, const double* dense,
                        char* mat_base, hipStream_t st) {
    if (n_ops <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_build, dim3(n_ops), dim3(kBuildThreads), 0, st, ops, gates, dense, mat_base);
    return hipGetLastError();
}

// Tile geometry of the staged kernels: the C lowest non-target bits are the
// columns; chunk i of the linear order starts at tau = i << unit.
StageGeom make_stage_geom(const ClusterGeom& g, int C, int unit) {
    StageGeom sg;
    std::memset(&sg, 0, sizeof(sg));
    uint64_t tmask = 0;
    for (int m = 0; m < g.k; ++m) tmask |= uint64_t(1) << g.t[m];
    int cols[8], nc = 0;
    for (int b = 0; b < g.n && nc < C; ++b)
        if (!(tmask >> b & 1)) cols[nc++] = b;
    uint64_t tilemask = tmask;
    for (int b = 0; b < nc; ++b) tilemask |= uint64_t(1) << cols[b];
    sg.nt = 0;
    for (int b = 0; b < g.n; ++b)
        if (tilemask >> b & 1) sg.tb[sg.nt++] = b;
    for (int r = 0; r < sg.nt; ++r) {
        for (int m = 0; m < g.k; ++m) if (sg.tb[r] == g.t[m]) sg.tpos[m] = r;
        for (int c = 0; c < nc; ++c) if (sg.tb[r] == cols[c]) sg.cpos[c] = r;
    }
    // LDS slots of the 6-qubit staged loop (11-bit tiles, half a tile per
    // wave): each column bit above tau bit 4 folds, by XOR, into a slot bit
    // among 1..4 that no lower column bit holds, so the 32 columns of an
    // 8-byte read have distinct slot bits 0..4 (no bank conflicts counted)
    // whatever bits the targets take; with target 0 on tau bit 0 (16-byte
    // reads) it is faster than a fixed fold as well, although conflicts are
    // still counted there. Bit 0 is never folded: it pairs amplitudes for
    // 16-byte accesses. The map is a bijection and linear over XOR.
    if (g.k == 6 && C == 5) {
        const bool lowt = g.t[0] == 0;
        int used = 1;
        for (int c = 0; c < nc; ++c)
            if (sg.cpos[c] < 5) used |= 1 << sg.cpos[c];
        for (int c = 0; c < (lowt ? 4 : 5) && c < nc; ++c) {
            if (sg.cpos[c] < 5) continue;
            int t = 1;
            while (t < 5 && ((used >> t) & 1)) ++t;
            if (t == 5) break;
            sg.swz[sg.cpos[c] - 5] = 1 << t;
            used |= 1 << t;
        }
    }
    const int chunks = 1 << (sg.nt - unit);
    for (int i = 0; i < chunks && i < 32; ++i) {
        const uint64_t tau = uint64_t(i) << unit;
        uint64_t off = 0;
        for (int r = 0; r < sg.nt; ++r)
            if (tau >> r & 1) off |= uint64_t(1) << sg.tb[r];
        sg.ioff[i] = off;
    }
    return sg;
}

int cluster_layout(bool dbl, int k, int n) {
    if (k == 7) return (!dbl && k <= max_cluster_k(dbl, n)) ? LAYOUT_SPLIT7 : -1;  // no other 7-qubit kernel
    if (!dbl) {
        if (k == 6) {
            if (n - k < 5) return LAYOUT_PLAIN;
            return g_k6_kernel == 2 ? LAYOUT_SPLIT16F : (g_k6_kernel == 1 ? LAYOUT_GAUSS32F : LAYOUT_MFMA32F);
        }
        return (k >= 4 && n - k >= 6) ? LAYOUT_MFMA32F : LAYOUT_PLAIN;
    }
    const int nb = (k == 6) ? 1 : 2;
    return (k >= 3 && n - k >= 4 + (nb == 2)) ? LAYOUT_MFMA16D : LAYOUT_PLAIN;
}

namespace {
template <int K>
hipError_t launch_valu_k(void* psi, bool dbl, const ClusterGeom& g, const void* mat, const EpiDesc* epi,
                         hipStream_t st, double* stats_part = nullptr, unsigned* stats_blocks = nullptr) {
    if (K >= 2 && K <= 3 && g.n - K >= 6) {
        constexpr int KS = K >= 2 && K <= 3 ? K : 2;
        const StageGeom sg = make_stage_geom(g, 6, 6);  // tile: the targets and 6 column bits
        for (int i = 0; i < 6; ++i)
            if (sg.tb[i] != i) return hipErrorInvalidValue;  // cannot happen: bits 0..5 are tile bits
        const uint64_t tiles = g.ncols >> 6;
        if (stats_part) {  // float (checked by the caller); the partials area holds kReduceBlocks work-groups
            if (dbl) return hipErrorInvalidValue;
            const unsigned grid = grid_for(tiles, 4, kReduceBlocks);
            *stats_blocks = grid;
            hipLaunchKernelGGL((k_cluster_valu_staged<float, KS, true>), dim3(grid), dim3(256), 0, st,
                               (float2*)psi, (const float2*)mat, epi, sg, tiles, stats_part);
            return hipGetLastError();
        }
        const unsigned grid = grid_for(tiles, 4, kStreamGrid);
        if (dbl)
            hipLaunchKernelGGL((k_cluster_valu_staged<double, KS>), dim3(grid), dim3(256), 0, st, (double2*)psi,
                               (const double2*)mat, epi, sg, tiles, nullptr);
        else
            hipLaunchKernelGGL((k_cluster_valu_staged<float, KS>), dim3(grid), dim3(256), 0, st, (float2*)psi,
                               (const float2*)mat, epi, sg, tiles, nullptr);
        return hipGetLastError();
    }
    if (stats_part) return hipErrorInvalidValue;  // no sums in the plain form
    const unsigned grid = grid_for(g.ncols, 256, kStreamGrid);
    if (dbl)
        hipLaunchKernelGGL((k_cluster_valu<double, K>), dim3(grid), dim3(256), 0, st, (double2*)psi,
                           (const double2*)mat, epi, g);
    else
        hipLaunchKernelGGL((k_cluster_valu<float, K>), dim3(grid), dim3(256), 0, st, (float2*)psi,
                           (const float2*)mat, epi, g);
    return hipGetLastError();
}

template <int K>
hipError_t launch_mfma32_k(void* psi, const ClusterGeom& g, const void* mat, const EpiDesc* epi, int variant,
                           hipStream_t st, double* stats_part, unsigned* stats_blocks) {
    if (stats_part && variant == 1) return hipErrorInvalidValue;  // sums come from the direct kernel only
    if (K <= 5 && variant == 1) {
        constexpr int KS = K <= 5 ? K : 5;
        const StageGeom sg = make_stage_geom(g, 6, 7);
        const uint64_t tiles = g.ncols >> 6;
        const unsigned grid = grid_for(tiles, 4, kPersistGrid);
        if (g.t[0] == 0)
            hipLaunchKernelGGL((k_cluster_f32_stage<KS, 6, true>), dim3(grid), dim3(256), 0, st, (float2*)psi,
                               (const float*)mat, epi, g, sg);
        else
            hipLaunchKernelGGL((k_cluster_f32_stage<KS, 6, false>), dim3(grid), dim3(256), 0, st, (float2*)psi,
                               (const float*)mat, epi, g, sg);
        return hipGetLastError();
    }
    constexpr int NB = (K == 6) ? 1 : 2;
    const uint64_t tiles = g.ncols / (32 * NB);
    const unsigned grid = grid_for(tiles, 4, kPersistGrid);
    if (stats_part) {
        *stats_blocks = grid;
        if (g.t[0] == 0)
            hipLaunchKernelGGL((k_cluster_f32_mfma<K, NB, true, true>), dim3(grid), dim3(256), 0, st, (float2*)psi,
                               (const float*)mat, epi, g, stats_part);
        else
            hipLaunchKernelGGL((k_cluster_f32_mfma<K, NB, false, true>), dim3(grid), dim3(256), 0, st,
                               (float2*)psi, (const float*)mat, epi, g, stats_part);
        return hipGetLastError();
    }
    if (g.t[0] == 0)
        hipLaunchKernelGGL((k_cluster_f32_mfma<K, NB, true>), dim3(grid), dim3(256), 0, st, (float2*)psi,
                           (const float*)mat, epi, g, nullptr);
    else
        hipLaunchKernelGGL((k_cluster_f32_mfma<K, NB, false>), dim3(grid), dim3(256), 0, st, (float2*)psi,
                           (const float*)mat, epi, g, nullptr);
    return hipGetLastError();
}

template <int K>
hipError_t launch_mfma64_k(void* psi, const ClusterGeom& g, const void* mat, const EpiDesc* epi, int variant,
                           hipStream_t st) {
    if (K <= 5 && variant == 1) {
        constexpr int KS = K <= 5 ? K : 5;
        constexpr int TH = KS == 5 ? 512 : 256;
        const StageGeom sg = make_stage_geom(g, 5, 6);
        const uint64_t tiles = g.ncols >> 5;
        const unsigned grid = grid_for(tiles, TH / 64, kPersistGrid);
        hipLaunchKernelGGL((k_cluster_f64_stage<KS, 5, TH>), dim3(grid), dim3(TH), 0, st, (vd2*)psi,
                           (const double*)mat, epi, g, sg);
        return hipGetLastError();
    }
    constexpr int NB = (K == 6) ? 1 : 2;
    constexpr int TH = (K == 6) ? 512 : 256;
    const uint64_t tiles = g.ncols / (16 * NB);
    const unsigned grid = grid_for(tiles, TH / 64, kPersistGrid);
    hipLaunchKernelGGL((k_cluster_f64_mfma<K, NB, TH>), dim3(grid), dim3(TH), 0, st, (double2*)psi,
                       (const double*)mat, epi, g);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_cluster(void* psi, bool dbl, const ClusterGeom& g, const void* mat, int layout,
                          const EpiDesc* epi, int variant, hipStream_t st, double* stats_part,
                          unsigned* stats_blocks) {
    // the sums of the stored amplitudes come from the direct float matrix-core kernels only
    if (stats_part && (!cluster_stats_supported(dbl, g.n, g.k, layout, variant) || !stats_blocks))
        return hipErrorInvalidValue;
    if (layout == LAYOUT_PLAIN) {
        switch (g.k) {
            case 1: return launch_valu_k<1>(psi, dbl, g, mat, epi, st);
            case 2: return launch_valu_k<2>(psi, dbl, g, mat, epi, st, stats_part, stats_blocks);
            case 3: return launch_valu_k<3>(psi, dbl, g, mat, epi, st, stats_part, stats_blocks);
            case 4: return launch_valu_k<4>(psi, dbl, g, mat, epi, st);
            case 5: return launch_valu_k<5>(psi, dbl, g, mat, epi, st);
            case 6: return launch_valu_k<6>(psi, dbl, g, mat, epi, st);
            default: return hipErrorInvalidValue;
        }
    }
    if (layout == LAYOUT_SPLIT7 && !dbl && g.k == 7 && g.n >= 12) {
        const uint64_t tiles = g.ncols / 32;
        const unsigned grid = grid_for(tiles, 4, kSplit7Grid);
        if (stats_part) {
            *stats_blocks = grid;
            if (g.t[0] == 0)
                hipLaunchKernelGGL((k_cluster_f32_split7<true, true>), dim3(grid), dim3(256), 0, st, (float2*)psi,
                                   (const half8*)mat, epi, g, stats_part);
            else
                hipLaunchKernelGGL((k_cluster_f32_split7<false, true>), dim3(grid), dim3(256), 0, st,
                                   (float2*)psi, (const half8*)mat, epi, g, stats_part);
            return hipGetLastError();
        }
        if (g.t[0] == 0)
            hipLaunchKernelGGL(k_cluster_f32_split7<true>, dim3(grid), dim3(256), 0, st, (float2*)psi,
                               (const half8*)mat, epi, g, nullptr);
        else
            hipLaunchKernelGGL(k_cluster_f32_split7<false>, dim3(grid), dim3(256), 0, st, (float2*)psi,
                               (const half8*)mat, epi, g, nullptr);
        return hipGetLastError();
    }
    if (layout == LAYOUT_SPLIT16F && !dbl && g.k == 6 && variant == 1) {
        const StageGeom sg = make_stage_geom(g, 5, 7);  // 11 tile bits; chunks of 2^7 amplitudes
        const uint64_t tiles = g.ncols >> 5;
        const unsigned grid = grid_for(tiles, 8, kStagedGrid);
        if (g.t[0] == 0)
            hipLaunchKernelGGL(k_cluster_f32_split6s<true>, dim3(grid), dim3(512), 0, st, (float2*)psi,
                               (const half8*)mat, epi, sg, tiles);
        else
            hipLaunchKernelGGL(k_cluster_f32_split6s<false>, dim3(grid), dim3(512), 0, st, (float2*)psi,
                               (const half8*)mat, epi, sg, tiles);
        return hipGetLastError();
    }
    if (layout == LAYOUT_SPLIT16F && !dbl && g.k == 6) {
        const uint64_t tiles = g.ncols / 32;
        const unsigned grid = grid_for(tiles, 4, kPersistGrid);
        if (stats_part) {
            *stats_blocks = grid;
            if (g.t[0] == 0)
                hipLaunchKernelGGL((k_cluster_f32_split6<true, true>), dim3(grid), dim3(256), 0, st, (float2*)psi,
                                   (const half8*)mat, epi, g, stats_part);
            else
                hipLaunchKernelGGL((k_cluster_f32_split6<false, true>), dim3(grid), dim3(256), 0, st,
                                   (float2*)psi, (const half8*)mat, epi, g, stats_part);
            return hipGetLastError();
        }
        if (g.t[0] == 0)
            hipLaunchKernelGGL(k_cluster_f32_split6<true>, dim3(grid), dim3(256), 0, st, (float2*)psi,
                               (const half8*)mat, epi, g, nullptr);
        else
            hipLaunchKernelGGL(k_cluster_f32_split6<false>, dim3(grid), dim3(256), 0, st, (float2*)psi,
                               (const half8*)mat, epi, g, nullptr);
        return hipGetLastError();
    }
    if (layout == LAYOUT_GAUSS32F && !dbl && g.k == 6) {
        const uint64_t tiles = g.ncols / 16;
        const unsigned grid = grid_for(tiles, 4, kPersistGrid);
        if (g.t[0] == 0)
            hipLaunchKernelGGL(k_cluster_f32_gauss6<true>, dim3(grid), dim3(256), 0, st, (float2*)psi,
                               (const float*)mat, epi, g);
        else
            hipLaunchKernelGGL(k_cluster_f32_gauss6<false>, dim3(grid), dim3(256), 0, st, (float2*)psi,
                               (const float*)mat, epi, g);
        return hipGetLastError();
    }
    if (layout == LAYOUT_MFMA32F && !dbl) {
        switch (g.k) {
            case 4: return launch_mfma32_k<4>(psi, g, mat, epi, variant, st, stats_part, stats_blocks);
            case 5: return launch_mfma32_k<5>(psi, g, mat, epi, variant, st, stats_part, stats_blocks);
            case 6: return launch_mfma32_k<6>(psi, g, mat, epi, variant, st, stats_part, stats_blocks);
            default: return hipErrorInvalidValue;
        }
    }
    if (layout == LAYOUT_MFMA16D && dbl) {
        switch (g.k) {
            case 3: return launch_mfma64_k<3>(psi, g, mat, epi, variant, st);
            case 4: return launch_mfma64_k<4>(psi, g, mat, epi, variant, st);
            case 5: return launch_mfma64_k<5>(psi, g, mat, epi, variant, st);
            case 6: return launch_mfma64_k<6>(psi, g, mat, epi, variant, st);
            default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_diag(void* psi, bool dbl, int n, const EpiDesc* epi, hipStream_t st) {
    // windows per wave step: 4 KiB of loads in flight per wave for either dtype
    constexpr int UF = 4, UD = 2;
    const uint64_t nwin = n >= 7 ? (uint64_t(1) << (n - 7)) : 1;
    const uint64_t nrun = (nwin + 63) >> 6;  // runs of 64 windows, one per wave at a time
    const unsigned grid = grid_for(nrun, 4, kStreamGrid);
    if (dbl)
        hipLaunchKernelGGL((k_diag<double, UD>), dim3(grid), dim3(256), 0, st, (double2*)psi, n, epi);
    else
        hipLaunchKernelGGL((k_diag<float, UF>), dim3(grid), dim3(256), 0, st, (float2*)psi, n, epi);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchOp* ops, const BatchItem* items, uint32_t n_items, uint32_t* counters,
                        uint32_t n_circuits, uint32_t item_tiles, uint64_t wait_ticks, unsigned grid,
                        hipStream_t st) {
    const uint32_t nc = n_circuits + 2;
    hipLaunchKernelGGL(k_fill_u32, dim3((nc + 255) / 256), dim3(256), 0, st, counters, nc, 0u);
    hipLaunchKernelGGL(k_batch_f32, dim3(grid), dim3(512), 0, st, ops, items, n_items, counters, item_tiles,
                       wait_ticks);
    return hipGetLastError();
}

hipError_t launch_gate1q(void* psi, bool dbl, int n, int q, const double m[8], hipStream_t st) {
    const uint64_t np = uint64_t(1) << (n - 1);
    const unsigned grid = grid_for(np, 256, kStreamGrid);
    if (dbl)
        hipLaunchKernelGGL(k_gate1q<double>, dim3(grid), dim3(256), 0, st, (double2*)psi, q, m[0], m[1], m[2],
                           m[3], m[4], m[5], m[6], m[7], np);
    else
        hipLaunchKernelGGL(k_gate1q<float>, dim3(grid), dim3(256), 0, st, (float2*)psi, q, (float)m[0],
                           (float)m[1], (float)m[2], (float)m[3], (float)m[4], (float)m[5], (float)m[6],
                           (float)m[7], np);
    return hipGetLastError();
}

hipError_t launch_phase1q(void* psi, bool dbl, int n, int q, double cs, double sn, hipStream_t st) {
    const uint64_t nh = uint64_t(1) << (n - 1);
    const unsigned grid = grid_for(nh, 256, kStreamGrid);
    if (dbl)
        hipLaunchKernelGGL(k_phase1q<double>, dim3(grid), dim3(256), 0, st, (double2*)psi, q, cs, sn, nh);
    else
        hipLaunchKernelGGL(k_phase1q<float>, dim3(grid), dim3(256), 0, st, (float2*)psi, q, (float)cs,
                           (float)sn, nh);
    return hipGetLastError();
}

hipError_t launch_cz(void* psi, bool dbl, int n, int a, int b, hipStream_t st) {
    if (a > b) { const int t = a; a = b; b = t; }
    const uint64_t nq = uint64_t(1) << (n - 2);
    const unsigned grid = grid_for(nq, 256, kStreamGrid);
    if (dbl)
        hipLaunchKernelGGL(k_cz<double>, dim3(grid), dim3(256), 0, st, (double2*)psi, a, b, nq);
    else
        hipLaunchKernelGGL(k_cz<float>, dim3(grid), dim3(256), 0, st, (float2*)psi, a, b, nq);
    return hipGetLastError();
}

hipError_t launch_stats(const void* psi, bool dbl, int n, void* probs, bool probs_dbl, double* part,
                        double* res, hipStream_t st) {
    const uint64_t cnt = uint64_t(1) << n;
    const unsigned grid = grid_for(cnt, 256, kReduceBlocks);
    if (dbl) {
        if (probs_dbl)
            hipLaunchKernelGGL((k_stats<double, double>), dim3(grid), dim3(256), 0, st, (const double2*)psi, cnt,
                               (double*)probs, part);
        else
            hipLaunchKernelGGL((k_stats<double, float>), dim3(grid), dim3(256), 0, st, (const double2*)psi, cnt,
                               (float*)probs, part);
    } else {
        if (probs_dbl)
            hipLaunchKernelGGL((k_stats<float, double>), dim3(grid), dim3(256), 0, st, (const float2*)psi, cnt,
                               (double*)probs, part);
        else
            hipLaunchKernelGGL((k_stats<float, float>), dim3(grid), dim3(256), 0, st, (const float2*)psi, cnt,
                               (float*)probs, part);
    }
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, st, part, (int)grid, 3, 0u, res);
    return hipGetLastError();
}

// ------------------------------------------------------------ bit permutation
// One work-group per tile (persistent grid): the whole tile is loaded into
// registers (every load in flight), written to LDS at its permuted index, and
// stored back in the original order of addresses, so loads and stores are
// both runs over the tile's lowest bits (the host puts the lowest non-moving
// state bits into the tile for that). In place: a tile is read completely
// before any of it is written, and tiles are disjoint.
template <typename V2, int NT>
__global__ __launch_bounds__(256) void k_permute(V2* __restrict__ psi, uint64_t ntiles, PermGeom pg) {
    constexpr int N = 1 << NT;
    constexpr int PER = (N + 255) / 256;
    __shared__ V2 buf[N];
    for (uint64_t tile = xcd_block(); tile < ntiles; tile += gridDim.x) {
        uint64_t base = tile;
#pragma unroll
        for (int i = 0; i < NT; ++i) base = insert_zero(base, pg.tb[i]);
        V2 v[PER];
        uint64_t addr[PER];
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int tau = r * 256 + (int)threadIdx.x;
            uint64_t off = 0;
#pragma unroll
            for (int j = 0; j < NT; ++j) off |= uint64_t((tau >> j) & 1) << pg.tb[j];
            addr[r] = base | off;
            if (tau < N) v[r] = psi[addr[r]];
        }
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int tau = r * 256 + (int)threadIdx.x;
            int dst = 0;
#pragma unroll
            for (int j = 0; j < NT; ++j) dst |= ((tau >> j) & 1) << pg.to[j];
            if (tau < N) buf[dst] = v[r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int tau = r * 256 + (int)threadIdx.x;
            if (tau < N) psi[addr[r]] = buf[tau];
        }
        __syncthreads();
    }
}

namespace {
template <int NT>
hipError_t launch_permute_nt(void* psi, bool dbl, int n, const PermGeom& pg, hipStream_t st) {
    const uint64_t tiles = uint64_t(1) << (n - NT);
    const unsigned grid = grid_for(tiles, 1, kPersistGrid);
    if (dbl)
        hipLaunchKernelGGL((k_permute<double2, NT>), dim3(grid), dim3(256), 0, st, (double2*)psi, tiles, pg);
    else
        hipLaunchKernelGGL((k_permute<float2, NT>), dim3(grid), dim3(256), 0, st, (float2*)psi, tiles, pg);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_permute(void* psi, bool dbl, int n, const PermGeom& pg, hipStream_t st) {
    if (pg.nt < 1 || pg.nt > kPermMaxBits || pg.nt > n) return hipErrorInvalidValue;
    switch (pg.nt) {
        case 1: return launch_permute_nt<1>(psi, dbl, n, pg, st);
        case 2: return launch_permute_nt<2>(psi, dbl, n, pg, st);
        case 3: return launch_permute_nt<3>(psi, dbl, n, pg, st);
        case 4: return launch_permute_nt<4>(psi, dbl, n, pg, st);
        case 5: return launch_permute_nt<5>(psi, dbl, n, pg, st);
        case 6: return launch_permute_nt<6>(psi, dbl, n, pg, st);
        case 7: return launch_permute_nt<7>(psi, dbl, n, pg, st);
        case 8: return launch_permute_nt<8>(psi, dbl, n, pg, st);
        case 9: return launch_permute_nt<9>(psi, dbl, n, pg, st);
        case 10: return launch_permute_nt<10>(psi, dbl, n, pg, st);
        case 11: return launch_permute_nt<11>(psi, dbl, n, pg, st);
        default: return launch_permute_nt<12>(psi, dbl, n, pg, st);
    }
}

hipError_t launch_reduce_stats(const double* part, unsigned nblocks, double* res, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, st, part, (int)nblocks, 3, 0u, res);
    return hipGetLastError();
}

hipError_t launch_compare(const void* psi, bool dbl, int n, const void* ref, bool ref_dbl, double* part,
                          double* res, hipStream_t st) {
    const uint64_t cnt = uint64_t(1) << n;
    const unsigned grid = grid_for(cnt, 256, kReduceBlocks);
    if (dbl) {
        if (ref_dbl)
            hipLaunchKernelGGL((k_compare<double, double>), dim3(grid), dim3(256), 0, st, (const double2*)psi,
                               (const double2*)ref, cnt, part);
        else
            hipLaunchKernelGGL((k_compare<double, float>), dim3(grid), dim3(256), 0, st, (const double2*)psi,
                               (const float2*)ref, cnt, part);
    } else {
        if (ref_dbl)
            hipLaunchKernelGGL((k_compare<float, double>), dim3(grid), dim3(256), 0, st, (const float2*)psi,
                               (const double2*)ref, cnt, part);
        else
            hipLaunchKernelGGL((k_compare<float, float>), dim3(grid), dim3(256), 0, st, (const float2*)psi,
                               (const float2*)ref, cnt, part);
    }
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, st, part, (int)grid, 5, 1u << 4, res);
    return hipGetLastError();
}

}  // namespace qsim
