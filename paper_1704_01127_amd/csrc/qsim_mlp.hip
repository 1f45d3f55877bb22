// GPU training kernels of the learned cost model: a multilayer perceptron
// in -> H -> H -> 1 with ReLU, float32, mean-squared-error loss, Adam.
//
// Parameter layout (one flat float array): W1 [H][in], b1 [H], W2 [H][H],
// b2 [H], W3 [H], b3 [1]. Samples are rows of x [batch][in].
#include <hip/hip_runtime.h>

#include <cmath>

#include "qsim.h"

namespace {

constexpr int kMaxIn = 32;
constexpr int kMaxH = 64;
constexpr int kSB = 64;  // samples per backward block

struct Net {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
    __device__ __host__ Net(const float* p, int n_in, int h)
        : W1(p), b1(p + h * n_in), W2(p + h * n_in + h), b2(p + h * n_in + h + h * h),
          W3(p + h * n_in + 2 * h + h * h), b3(p + h * n_in + 3 * h + h * h) {}
};

__device__ __forceinline__ float relu(float s) { return s > 0.f ? s : 0.f; }

// Forward of one sample, dot products accumulated with fused multiply-adds
// in index order (the host evaluation uses the same order).
__device__ float forward_one(const Net& N, int n_in, int h, const float* x, float* a1, float* a2) {
    for (int i = 0; i < h; ++i) {
        float s = N.b1[i];
        for (int j = 0; j < n_in; ++j) s = __builtin_fmaf(N.W1[i * n_in + j], x[j], s);
        a1[i] = relu(s);
    }
    for (int i = 0; i < h; ++i) {
        float s = N.b2[i];
        for (int j = 0; j < h; ++j) s = __builtin_fmaf(N.W2[i * h + j], a1[j], s);
        a2[i] = relu(s);
    }
    float y = N.b3[0];
    for (int j = 0; j < h; ++j) y = __builtin_fmaf(N.W3[j], a2[j], y);
    return y;
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ p, int n_in, int h,
                                                     const float* __restrict__ x, int batch, float* __restrict__ y) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= batch) return;
    float a1[kMaxH], a2[kMaxH];
    const Net N(p, n_in, h);
    y[b] = forward_one(N, n_in, h, x + (size_t)b * n_in, a1, a2);
}

// Per block of kSB samples: forward, deltas, and the block's partial sums of
// every parameter gradient and of the squared error.
__global__ __launch_bounds__(256) void k_mlp_backward_partial(const float* __restrict__ p, int n_in, int h,
                                                              const float* __restrict__ x,
                                                              const float* __restrict__ t, int batch,
                                                              float* __restrict__ part) {
    __shared__ float sx[kSB][kMaxIn];
    __shared__ float sa1[kSB][kMaxH], sa2[kSB][kMaxH], sd1[kSB][kMaxH], sd2[kSB][kMaxH];
    __shared__ float sdy[kSB], se2[kSB];
    const Net N(p, n_in, h);
    const int P = h * n_in + h + h * h + h + h + 1;
    const int tid = threadIdx.x;
    if (tid < kSB) {
        const int b = blockIdx.x * kSB + tid;
        float a1[kMaxH], a2[kMaxH];
        if (b < batch) {
            for (int j = 0; j < n_in; ++j) sx[tid][j] = x[(size_t)b * n_in + j];
            const float yb = forward_one(N, n_in, h, &sx[tid][0], a1, a2);
            const float r = yb - t[b];
            const float dy = 2.0f * r / (float)batch;
            sdy[tid] = dy;
            se2[tid] = r * r;
            for (int i = 0; i < h; ++i) {
                sa1[tid][i] = a1[i];
                sa2[tid][i] = a2[i];
                sd2[tid][i] = a2[i] > 0.f ? dy * N.W3[i] : 0.f;
            }
            for (int j = 0; j < h; ++j) {
                float s = 0.f;
                for (int i = 0; i < h; ++i) s = __builtin_fmaf(N.W2[i * h + j], sd2[tid][i], s);
                sd1[tid][j] = a1[j] > 0.f ? s : 0.f;
            }
        } else {
            for (int j = 0; j < n_in; ++j) sx[tid][j] = 0.f;
            sdy[tid] = 0.f;
            se2[tid] = 0.f;
            for (int i = 0; i < h; ++i) sa1[tid][i] = sa2[tid][i] = sd1[tid][i] = sd2[tid][i] = 0.f;
        }
    }
    __syncthreads();
    float* out = part + (size_t)blockIdx.x * (P + 1);
    const int o1 = h * n_in, o2 = o1 + h, o3 = o2 + h * h, o4 = o3 + h, o5 = o4 + h;
    for (int w = tid; w < P; w += 256) {
        float s = 0.f;
        if (w < o1) {
            const int i = w / n_in, j = w % n_in;
            for (int b = 0; b < kSB; ++b) s = __builtin_fmaf(sd1[b][i], sx[b][j], s);
        } else if (w < o2) {
            const int i = w - o1;
            for (int b = 0; b < kSB; ++b) s += sd1[b][i];
        } else if (w < o3) {
            const int i = (w - o2) / h, j = (w - o2) % h;
            for (int b = 0; b < kSB; ++b) s = __builtin_fmaf(sd2[b][i], sa1[b][j], s);
        } else if (w < o4) {
            const int i = w - o3;
            for (int b = 0; b < kSB; ++b) s += sd2[b][i];
        } else if (w < o5) {
            const int j = w - o4;
            for (int b = 0; b < kSB; ++b) s = __builtin_fmaf(sdy[b], sa2[b][j], s);
        } else {
            for (int b = 0; b < kSB; ++b) s += sdy[b];
        }
        out[w] = s;
    }
    if (tid == 0) {
        float s = 0.f;
        for (int b = 0; b < kSB; ++b) s += se2[b];
        out[P] = s;
    }
}

// grad[w] = sum over blocks, in block order; loss = sum of squared errors / batch.
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ part, int nblocks, int P, int batch,
                                                    float* __restrict__ grad, float* __restrict__ loss) {
    const int w = blockIdx.x * 256 + threadIdx.x;
    if (w > P) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * (P + 1) + w];
    if (w < P) grad[w] = s;
    else if (loss) loss[0] = s / (float)batch;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int n, float lr,
                                              float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

bool dims_ok(int n_in, int h) { return n_in >= 1 && n_in <= kMaxIn && h >= 1 && h <= kMaxH; }
int param_count(int n_in, int h) { return h * n_in + h + h * h + h + h + 1; }

}  // namespace

extern "C" {

size_t qsim_mlp_param_count(int n_in, int n_hidden) { return (size_t)param_count(n_in, n_hidden); }

size_t qsim_mlp_scratch_floats(int n_in, int n_hidden, int batch) {
    const size_t nb = (size_t)(batch + kSB - 1) / kSB;
    return nb * (size_t)(param_count(n_in, n_hidden) + 1);
}

qsim_status qsim_mlp_forward(int n_in, int n_hidden, const float* dev_params, const float* dev_x, int batch,
                             float* dev_y, void* stream) {
    if (!dims_ok(n_in, n_hidden) || !dev_params || !dev_x || !dev_y || batch < 0) return QSIM_E_INVALID;
    if (batch == 0) return QSIM_OK;
    hipLaunchKernelGGL(k_mlp_forward, dim3((batch + 255) / 256), dim3(256), 0, (hipStream_t)stream, dev_params,
                       n_in, n_hidden, dev_x, batch, dev_y);
    return hipGetLastError() == hipSuccess ? QSIM_OK : QSIM_E_DEVICE;
}

qsim_status qsim_mlp_backward(int n_in, int n_hidden, const float* dev_params, const float* dev_x,
                              const float* dev_target, int batch, float* dev_grad, float* dev_loss,
                              float* dev_scratch, void* stream) {
    if (!dims_ok(n_in, n_hidden) || !dev_params || !dev_x || !dev_target || !dev_grad || !dev_scratch ||
        batch < 1)
        return QSIM_E_INVALID;
    const int nb = (batch + kSB - 1) / kSB;
    const int P = param_count(n_in, n_hidden);
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_backward_partial, dim3(nb), dim3(256), 0, st, dev_params, n_in, n_hidden, dev_x,
                       dev_target, batch, dev_scratch);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((P + 1 + 255) / 256), dim3(256), 0, st, dev_scratch, nb, P, batch,
                       dev_grad, dev_loss);
    return hipGetLastError() == hipSuccess ? QSIM_OK : QSIM_E_DEVICE;
}

qsim_status qsim_mlp_adam(int n_params, float* dev_params, const float* dev_grad, float* dev_m, float* dev_v,
                          int step, float lr, float beta1, float beta2, float eps, void* stream) {
    if (n_params < 1 || !dev_params || !dev_grad || !dev_m || !dev_v || step < 1) return QSIM_E_INVALID;
    const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((n_params + 255) / 256), dim3(256), 0, (hipStream_t)stream, dev_params,
                       dev_grad, dev_m, dev_v, n_params, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? QSIM_OK : QSIM_E_DEVICE;
}

}  // extern "C"
