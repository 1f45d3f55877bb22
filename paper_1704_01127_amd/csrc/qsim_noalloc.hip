// qsim_probs_noalloc: the probabilities and float64 reductions of qsim_probs
// for callers that cannot allocate device memory (code under graph capture,
// tight serving loops, harnesses that forbid hipMalloc). The reduction's
// partial sums and its result live in a fixed device array of this library
// instead of a caller-provided workspace.
#include <hip/hip_runtime.h>

#include <mutex>

#include "api_common.h"
#include "qsim.h"
#include "qsim_internal.h"

using namespace qsim;
using namespace qsim::api;

namespace {

// Partial sums of at most kReduceBlocks work-groups (the reduction's grid is
// capped there for every state size) and the 8 result doubles.
constexpr size_t kScratchPart = size_t(kReduceBlocks) * 8 * sizeof(double);
constexpr size_t kScratchBytes = kScratchPart + 256;

// One copy per GPU, held until the process ends. In host code this name is a
// host-side stand-in: the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` on each device

// Device address of the scratch array on the current device, looked up once
// per device (with that device current).
qsim_status scratch_on_current_device(void** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(QSIM_E_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p) return fail(QSIM_E_DEVICE, "hipGetSymbolAddress(scratch) returned null");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return QSIM_OK;
}

}  // namespace

extern "C" {

size_t qsim_noalloc_scratch_bytes(void) { return kScratchBytes; }

qsim_status qsim_probs_noalloc(int n_qubits, qsim_dtype dt, const void* dev_amps, size_t amps_bytes,
                               void* hip_stream, void* dev_out, qsim_dtype out_dt, double* norm, double* sum_p2,
                               double* entropy_nats) {
    if (dt != QSIM_C64 && dt != QSIM_C128) return fail(QSIM_E_INVALID, "unknown dtype");
    const int nmax = dt == QSIM_C64 ? 34 : 33;
    if (n_qubits < 1 || n_qubits > nmax)
        return fail(QSIM_E_UNSUPPORTED, "n_qubits out of range (at most 34 for C64, 33 for C128)");
    if (!dev_amps) return fail(QSIM_E_INVALID, "null amplitude buffer");
    const size_t need = (size_t(1) << n_qubits) * (dt == QSIM_C64 ? 8 : 16);
    if (amps_bytes < need) return fail(QSIM_E_INVALID, "amps_bytes smaller than 2^n amplitudes");
    if (dev_out && out_dt != QSIM_C64 && out_dt != QSIM_C128) return fail(QSIM_E_INVALID, "unknown out dtype");
    void* base = nullptr;
    if (qsim_status r = scratch_on_current_device(&base)) return r;
    double* part = reinterpret_cast<double*>(base);
    double* res = reinterpret_cast<double*>(static_cast<unsigned char*>(base) + kScratchPart);
    const hipStream_t st = static_cast<hipStream_t>(hip_stream);
    // every partial slot the final reduction reads is written by this launch:
    // nothing has to start at zero
    HIP_TRY(launch_stats(dev_amps, dt == QSIM_C128, n_qubits, dev_out, out_dt == QSIM_C128, part, res, st),
            "stats launch");
    double h[8];
    HIP_TRY(hipMemcpyAsync(h, res, 8 * sizeof(double), hipMemcpyDeviceToHost, st), "stats copy");
    HIP_TRY(hipStreamSynchronize(st), "stats sync");
    if (norm) *norm = h[0];
    if (sum_p2) *sum_p2 = h[1];
    if (entropy_nats) *entropy_nats = h[2];
    return QSIM_OK;
}

}  // extern "C"
