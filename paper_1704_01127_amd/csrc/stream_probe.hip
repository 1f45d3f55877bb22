// Streaming-bandwidth probe for MI355X HBM: how fast plain read / write /
// in-place update passes over a buffer of the state's size can go, with
// normal and non-temporal accesses and different grid sizes. Its in-place
// pass is also the calibration kernel for the HBM traffic counters (a pass of
// known size: 2 x bytes).
//
//   stream_probe <log2 bytes> [reps]
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

typedef float f4 __attribute__((ext_vector_type(4)));

#define CHECK(x)                                                                  \
    do {                                                                          \
        hipError_t e = (x);                                                       \
        if (e != hipSuccess) {                                                    \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e));           \
            std::exit(1);                                                         \
        }                                                                         \
    } while (0)

template <int U, bool NT>
__global__ __launch_bounds__(256) void k_inplace(f4* __restrict__ p, size_t n4, float s) {
    const size_t stride = (size_t)gridDim.x * 256 * U;
    for (size_t i = (size_t)blockIdx.x * 256 * U + threadIdx.x; i < n4; i += stride) {
        f4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t j = i + (size_t)u * 256;
            if (j < n4) v[u] = NT ? __builtin_nontemporal_load(p + j) : p[j];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t j = i + (size_t)u * 256;
            if (j < n4) {
                f4 w = v[u] * s;
                if (NT) __builtin_nontemporal_store(w, p + j); else p[j] = w;
            }
        }
    }
}

template <int U>
__global__ __launch_bounds__(256) void k_copy(const f4* __restrict__ a, f4* __restrict__ b, size_t n4) {
    const size_t stride = (size_t)gridDim.x * 256 * U;
    for (size_t i = (size_t)blockIdx.x * 256 * U + threadIdx.x; i < n4; i += stride) {
        f4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t j = i + (size_t)u * 256;
            if (j < n4) v[u] = a[j];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const size_t j = i + (size_t)u * 256;
            if (j < n4) b[j] = v[u];
        }
    }
}

__global__ __launch_bounds__(256) void k_read(const f4* __restrict__ a, size_t n4, float* out) {
    float acc = 0.f;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (size_t)gridDim.x * 256) {
        const f4 v = a[i];
        acc += v.x + v.y + v.z + v.w;
    }
    if (acc == 12345.678f) out[0] = acc;  // keeps the loads alive
}

__global__ __launch_bounds__(256) void k_write(f4* __restrict__ a, size_t n4) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += (size_t)gridDim.x * 256)
        a[i] = f4{1.f, 2.f, 3.f, 4.f};
}

// The access pattern of the 6-qubit cluster kernel without its arithmetic:
// a wave owns 32 neighbouring columns x 64 rows (rows 2^tshift amplitudes
// apart, 8-byte amplitudes), lane (p, h) column p, rows j | h << 5, with the
// next tile's rows loaded into registers before the current tile is stored.
__global__ __launch_bounds__(256, 2) void k_rows(float* __restrict__ p, size_t ntiles, int tshift, float s) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    f2* q = reinterpret_cast<f2*>(p);
    const int lane = threadIdx.x & 63, col = lane & 31, h = lane >> 5;
    const size_t stride = (size_t)gridDim.x * 4;
    size_t tile = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= ntiles) return;
    const size_t last = ntiles - 1;
    auto addr = [&](size_t t, int j) { return t * 32 + col + ((size_t)(j | (h << 5)) << tshift); };
    f2 B[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) B[j] = q[addr(tile, j)];
    do {
        const size_t nxt = tile + stride < last ? tile + stride : last;
        f2 Bn[32];
#pragma unroll
        for (int j = 0; j < 32; ++j) Bn[j] = q[addr(nxt, j)];
#pragma unroll
        for (int j = 0; j < 32; ++j) q[addr(tile, j)] = B[j] * s;
#pragma unroll
        for (int j = 0; j < 32; ++j) B[j] = Bn[j];
        tile += stride;
    } while (tile < ntiles);
}

// Variants of the same pattern: MODE 1 gives each XCD (work-groups are
// dealt round-robin to 8 of them) a contiguous share of the tiles; MODE 2
// rotates each wave's row order by its tile number; WAVES 8 makes 2 KiB row
// runs per work-group.
template <int MODE, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_rows_v(float* __restrict__ p, size_t ntiles, int tshift, float s) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    f2* q = reinterpret_cast<f2*>(p);
    const int lane = threadIdx.x & 63, col = lane & 31, h = lane >> 5;
    const size_t waves = (size_t)gridDim.x * WAVES;
    size_t wid = (size_t)blockIdx.x * WAVES + (threadIdx.x >> 6);
    if (MODE == 1) {  // work-group b runs on XCD b % 8: renumber so that each XCD's waves are consecutive
        const size_t per = gridDim.x / 8;
        wid = ((blockIdx.x % 8) * per + blockIdx.x / 8) * WAVES + (threadIdx.x >> 6);
    }
    size_t tile = wid;
    if (tile >= ntiles) return;
    const size_t last = ntiles - 1;
    auto addr = [&](size_t t, int j) {
        const int r = MODE == 2 ? ((j + (int)(t & 31)) & 31) : j;
        return t * 32 + col + ((size_t)(r | (h << 5)) << tshift);
    };
    f2 B[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) B[j] = q[addr(tile, j)];
    do {
        const size_t nxt = tile + waves < last ? tile + waves : last;
        f2 Bn[32];
#pragma unroll
        for (int j = 0; j < 32; ++j) Bn[j] = q[addr(nxt, j)];
#pragma unroll
        for (int j = 0; j < 32; ++j) q[addr(tile, j)] = B[j] * s;
#pragma unroll
        for (int j = 0; j < 32; ++j) B[j] = Bn[j];
        tile += waves;
    } while (tile < ntiles);
}

template <typename F>
static float time_ms(F f, int reps) {
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    f();
    CHECK(hipDeviceSynchronize());
    std::vector<float> t(reps);
    for (int r = 0; r < reps; ++r) {
        CHECK(hipEventRecord(e0));
        f();
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        CHECK(hipEventElapsedTime(&t[r], e0, e1));
    }
    float best = t[0];
    for (float x : t) best = x < best ? x : best;
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return best;
}

int main(int argc, char** argv) {
    const int lg = argc > 1 ? std::atoi(argv[1]) : 33;
    const int reps = argc > 2 ? std::atoi(argv[2]) : 5;
    const size_t bytes = size_t(1) << lg;
    const size_t n4 = bytes / 16;
    f4 *a, *b;
    float* o;
    CHECK(hipMalloc(&a, bytes));
    CHECK(hipMalloc(&b, bytes));
    CHECK(hipMalloc(&o, 16));
    CHECK(hipMemset(a, 0, bytes));
    CHECK(hipMemset(b, 0, bytes));
    const double gb = bytes / 1e9;
    std::printf("buffer %.2f GB\n", gb);
    // the cluster kernel's pattern: 2^(lg-3) amplitudes, rows on the top 6 bits
    {
        const int na = lg - 3;
        const size_t ntiles = (size_t(1) << (na - 6)) / 32;
        for (unsigned grid : {512u, 1024u, 2048u, 8192u}) {
            const float t = time_ms([&] { hipLaunchKernelGGL(k_rows, dim3(grid), dim3(256), 0, 0, (float*)a, ntiles,
                                                             na - 6, 1.0f); }, reps);
            std::printf("rows     k=6 top grid %6u  %7.3f ms  %7.0f GB/s\n", grid, t, 2 * gb / t * 1e3);
        }
        for (unsigned grid : {512u, 1024u, 2048u}) {
            float t = time_ms([&] { hipLaunchKernelGGL((k_rows_v<1, 4>), dim3(grid), dim3(256), 0, 0, (float*)a,
                                                       ntiles, na - 6, 1.0f); }, reps);
            std::printf("rows xcd k=6 top grid %6u  %7.3f ms  %7.0f GB/s\n", grid, t, 2 * gb / t * 1e3);
            t = time_ms([&] { hipLaunchKernelGGL((k_rows_v<2, 4>), dim3(grid), dim3(256), 0, 0, (float*)a, ntiles,
                                                 na - 6, 1.0f); }, reps);
            std::printf("rows rot k=6 top grid %6u  %7.3f ms  %7.0f GB/s\n", grid, t, 2 * gb / t * 1e3);
            t = time_ms([&] { hipLaunchKernelGGL((k_rows_v<0, 8>), dim3(grid / 2), dim3(512), 0, 0, (float*)a,
                                                 ntiles, na - 6, 1.0f); }, reps);
            std::printf("rows 8w  k=6 top grid %6u  %7.3f ms  %7.0f GB/s\n", grid / 2, t, 2 * gb / t * 1e3);
        }
    }
    for (unsigned grid : {8192u, 32768u, 65536u}) {
        const float t = time_ms([&] { hipLaunchKernelGGL((k_inplace<8, false>), dim3(grid), dim3(256), 0, 0, a, n4,
                                                         1.0f); }, reps);
        std::printf("inplace  U8      grid %6u  %7.3f ms  %7.0f GB/s\n", grid, t, 2 * gb / t * 1e3);
    }
    for (unsigned grid : {1024u, 2048u, 4096u, 8192u, 32768u}) {
        float t;
        t = time_ms([&] { hipLaunchKernelGGL((k_inplace<1, false>), dim3(grid), dim3(256), 0, 0, a, n4, 1.0f); }, reps);
        std::printf("inplace  U1      grid %6u  %7.3f ms  %7.0f GB/s\n", grid, t, 2 * gb / t * 1e3);
        t = time_ms([&] { hipLaunchKernelGGL((k_inplace<4, false>), dim3(grid), dim3(256), 0, 0, a, n4, 1.0f); }, reps);
        std::printf("inplace  U4      grid %6u  %7.3f ms  %7.0f GB/s\n", grid, t, 2 * gb / t * 1e3);
        t = time_ms([&] { hipLaunchKernelGGL((k_inplace<4, true>), dim3(grid), dim3(256), 0, 0, a, n4, 1.0f); }, reps);
        std::printf("inplace  U4 nt   grid %6u  %7.3f ms  %7.0f GB/s\n", grid, t, 2 * gb / t * 1e3);
        t = time_ms([&] { hipLaunchKernelGGL((k_copy<4>), dim3(grid), dim3(256), 0, 0, a, b, n4); }, reps);
        std::printf("copy     U4      grid %6u  %7.3f ms  %7.0f GB/s\n", grid, t, 2 * gb / t * 1e3);
        t = time_ms([&] { hipLaunchKernelGGL(k_read, dim3(grid), dim3(256), 0, 0, a, n4, o); }, reps);
        std::printf("read             grid %6u  %7.3f ms  %7.0f GB/s\n", grid, t, gb / t * 1e3);
        t = time_ms([&] { hipLaunchKernelGGL(k_write, dim3(grid), dim3(256), 0, 0, a, n4); }, reps);
        std::printf("write            grid %6u  %7.3f ms  %7.0f GB/s\n", grid, t, gb / t * 1e3);
    }
    CHECK(hipFree(a));
    CHECK(hipFree(b));
    CHECK(hipFree(o));
    return 0;
}
