// Learned cost model of the scheduler: features of a cluster op and the
// host-side evaluation of a small MLP (in -> H -> H -> 1, ReLU, float32)
// trained on the simulator's own recorded kernel times. The prediction is the
// natural log of the op's time per 2^30 amplitudes in microseconds; the
// scheduler's cost is exp(prediction) * 2^(n - 30).
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "qsim.h"
#include "qsim_internal.h"

namespace qsim {

constexpr int kFeatures = 16;

// Features of one op: sizes, FLOP and byte intensity, where the targets sit
// (low bits break coalescing, high bits stride far), kernel kind and the
// diagonal epilogue. k = 0 is a standalone diagonal pass.
void op_features(int n, bool dbl, int k, const int* q, int n_epi, float* f, int variant_override) {
    std::memset(f, 0, sizeof(float) * kFeatures);
    int lo = n, hi = -1, below3 = 0, below6 = 0, top3 = 0;
    for (int j = 0; j < k; ++j) {
        lo = q[j] < lo ? q[j] : lo;
        hi = q[j] > hi ? q[j] : hi;
        below3 += q[j] < 3;
        below6 += q[j] < 6;
        top3 += q[j] >= n - 3;
    }
    if (k == 0) lo = hi = 0;
    const int layout = k == 0 ? LAYOUT_PLAIN : cluster_layout(dbl, k, n);
    ClusterGeom g;
    std::memset(&g, 0, sizeof(g));
    for (int j = 0; j < k; ++j) g.t[j] = q[j];
    g.k = k;
    g.n = n;
    int variant = k == 0 ? 0 : cluster_variant_for(dbl, g, layout);
    if (variant_override >= 0 && k > 0 && variant_choice(dbl, k, layout)) variant = variant_override;
    f[0] = k / 6.0f;
    f[1] = n / 34.0f;
    f[2] = dbl ? 1.0f : 0.0f;
    f[3] = k == 0 ? 0.0f : (8.0f * (1 << k) - 2.0f) / 510.0f;
    f[4] = dbl ? 1.0f : 0.5f;
    f[5] = (float)lo / n;
    f[6] = (float)hi / n;
    f[7] = below3 / 3.0f;
    f[8] = below6 / 6.0f;
    f[9] = top3 / 3.0f;
    f[10] = layout != LAYOUT_PLAIN ? 1.0f : 0.0f;
    f[11] = variant ? 1.0f : 0.0f;
    f[12] = n_epi > 0 ? 1.0f : 0.0f;
    f[13] = std::log2(1.0f + n_epi) / 7.0f;
    f[14] = k == 6 ? 1.0f : 0.0f;
    f[15] = k == 0 ? 1.0f : 0.0f;
}

namespace {
struct Model {
    bool loaded = false;
    int n_in = 0, n_hidden = 0;
    std::vector<float> p;             // W1 [H][in], b1 [H], W2 [H][H], b2 [H], W3 [H], b3 [1]
    std::vector<float> mean, inv_std; // feature normalisation
    float y_mean = 0.f, y_std = 1.f;
};
// The loaded model; a load replaces the pointer, so a prediction in flight
// keeps the model it started with and needs no lock while it evaluates.
std::shared_ptr<const Model> g_model = std::make_shared<Model>();
std::mutex g_model_mu;

std::shared_ptr<const Model> current_model() {
    std::lock_guard<std::mutex> lk(g_model_mu);
    return g_model;
}
}  // namespace

size_t mlp_param_count(int n_in, int h) { return (size_t)h * n_in + h + (size_t)h * h + h + h + 1; }

// Plain float32 forward pass of one sample (the same operation order as the
// GPU forward kernel: each unit's dot product is a chain of fused
// multiply-adds in index order). The loops run over the inputs outermost so
// that the units' chains are independent of each other (and vectorise); every
// chain keeps its order, so the result does not depend on the loop shape.
template <bool kHwFma>
static float mlp_forward_impl(const float* p, int n_in, int h, const float* x) {
    const float* W1 = p;
    const float* b1 = W1 + (size_t)h * n_in;
    const float* W2 = b1 + h;
    const float* b2 = W2 + (size_t)h * h;
    const float* W3 = b2 + h;
    const float* b3 = W3 + h;
    float a1[256], a2[256];
    for (int i = 0; i < h; ++i) a1[i] = b1[i];
    for (int j = 0; j < n_in; ++j)
        for (int i = 0; i < h; ++i) a1[i] = std::fma(W1[(size_t)i * n_in + j], x[j], a1[i]);
    for (int i = 0; i < h; ++i) a1[i] = a1[i] > 0.f ? a1[i] : 0.f;
    for (int i = 0; i < h; ++i) a2[i] = b2[i];
    for (int j = 0; j < h; ++j)
        for (int i = 0; i < h; ++i) a2[i] = std::fma(W2[(size_t)i * h + j], a1[j], a2[i]);
    for (int i = 0; i < h; ++i) a2[i] = a2[i] > 0.f ? a2[i] : 0.f;
    float y = b3[0];
    for (int j = 0; j < h; ++j) y = std::fma(W3[j], a2[j], y);
    return y;
}

// With the FMA instructions available, std::fma compiles to them instead of a
// library call.
__attribute__((target("avx2,fma"))) static float mlp_forward_fma(const float* p, int n_in, int h, const float* x) {
    return mlp_forward_impl<true>(p, n_in, h, x);
}

float mlp_forward_host(const float* p, int n_in, int h, const float* x) {
    static const bool hw = __builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma");
    return hw ? mlp_forward_fma(p, n_in, h, x) : mlp_forward_impl<false>(p, n_in, h, x);
}

bool learned_model_loaded() { return current_model()->loaded; }

double learned_cost_us(int n, bool dbl, int k, const int* qubits, int n_epi, int variant) {
    float f[kFeatures];
    op_features(n, dbl, k, qubits, n_epi, f, variant);
    const std::shared_ptr<const Model> m = current_model();
    if (!m->loaded) return 1.0;
    float x[kFeatures];
    for (int i = 0; i < kFeatures; ++i) x[i] = (f[i] - m->mean[i]) * m->inv_std[i];
    const float y = mlp_forward_host(m->p.data(), m->n_in, m->n_hidden, x);
    const double log_us = (double)y * m->y_std + m->y_mean;
    return std::exp(log_us) * std::ldexp(1.0, n - 30);
}

// Predicted time of an op with the faster of the two matrix-core kernel
// variants (direct gather or LDS-staged tiles) where the op has both and no
// variant is forced; *variant (nullable) receives the choice (-1: the
// library's own rule applies).
double learned_cost_best_us(int n, bool dbl, int k, const int* qubits, int n_epi, int* variant) {
    if (variant) *variant = -1;
    if (k == 0 || get_cluster_variant() >= 0 || !variant_choice(dbl, k, cluster_layout(dbl, k, n)))
        return learned_cost_us(n, dbl, k, qubits, n_epi, -1);
    const double t0 = learned_cost_us(n, dbl, k, qubits, n_epi, 0);
    const double t1 = learned_cost_us(n, dbl, k, qubits, n_epi, 1);
    if (variant) *variant = t1 < t0 ? 1 : 0;
    return t1 < t0 ? t1 : t0;
}

}  // namespace qsim

using namespace qsim;

extern "C" {

int qsim_cost_feature_count(void) { return kFeatures; }

qsim_status qsim_cost_features(int n_qubits, qsim_dtype dt, int k, const int32_t* qubits, int n_epi,
                               float* out) {
    if (!out || k < 0 || k > kMaxK || (k > 0 && !qubits) || n_qubits < 1 || n_qubits > 40)
        return QSIM_E_INVALID;
    int q[kMaxK] = {};
    for (int j = 0; j < k; ++j) q[j] = qubits[j];
    op_features(n_qubits, dt == QSIM_C128, k, q, n_epi, out, -1);
    return QSIM_OK;
}

qsim_status qsim_set_cost_model(const float* params, int n_in, int n_hidden, const float* feat_mean,
                                const float* feat_std, double y_mean, double y_std) {
    if (!params) {  // unload
        std::lock_guard<std::mutex> lk(g_model_mu);
        g_model = std::make_shared<Model>();
        return QSIM_OK;
    }
    if (n_in != kFeatures || n_hidden < 1 || n_hidden > 256 || !feat_mean || !feat_std || !(y_std > 0))
        return QSIM_E_INVALID;
    Model m;
    m.n_in = n_in;
    m.n_hidden = n_hidden;
    m.p.assign(params, params + mlp_param_count(n_in, n_hidden));
    m.mean.assign(feat_mean, feat_mean + n_in);
    m.inv_std.resize(n_in);
    for (int i = 0; i < n_in; ++i) m.inv_std[i] = feat_std[i] > 0 ? 1.0f / feat_std[i] : 0.0f;
    m.y_mean = (float)y_mean;
    m.y_std = (float)y_std;
    m.loaded = true;
    std::lock_guard<std::mutex> lk(g_model_mu);
    g_model = std::make_shared<const Model>(std::move(m));
    return QSIM_OK;
}

qsim_status qsim_mlp_predict_host(const float* params, int n_in, int n_hidden, const float* x, int batch,
                                  float* y) {
    if (!params || !x || !y || n_in < 1 || n_hidden < 1 || n_hidden > 256 || batch < 0) return QSIM_E_INVALID;
    for (int b = 0; b < batch; ++b) y[b] = mlp_forward_host(params, n_in, n_hidden, x + (size_t)b * n_in);
    return QSIM_OK;
}

double qsim_cost_model_predict_us(int n_qubits, qsim_dtype dt, int k, const int32_t* qubits, int n_epi) {
    if (k < 0 || k > kMaxK || (k > 0 && !qubits)) return -1.0;
    int q[kMaxK] = {};
    for (int j = 0; j < k; ++j) q[j] = qubits[j];
    return learned_cost_us(n_qubits, dt == QSIM_C128, k, q, n_epi, -1);
}

}  // extern "C"
