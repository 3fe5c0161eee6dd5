// Fused log-likelihood (+ gradient) for callers that cannot allocate device memory: the
// workspace of pd_loglike_and_grad lives in a fixed file-scope device array instead of a
// caller-owned buffer.
//
// The array is device memory of the module: each GPU the library runs on holds its own copy,
// at its own address, until the process ends.  Host code never uses the array's name as a
// device address (in host code it is only a stand-in symbol); the address is looked up once per
// device with hipGetSymbolAddress and cached, and that pointer is what the launches receive.
// Calls on one GPU share the array, so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/phenomd.h"
#include "pd_launch.h"

namespace {

constexpr size_t kScratchBytes = PD_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

int fail(int code, const std::string& msg) {
    pd::set_last_error(msg.c_str());
    return code;
}

// Device address of this GPU's copy of `scratch`, looked up once per device (with that device
// current) and kept for the life of the process.
std::mutex g_mu;
std::vector<void*> g_ptr;   // indexed by device id; nullptr = not looked up yet

int scratch_ptr(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(PD_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_mu);
    if (dev >= static_cast<int>(g_ptr.size())) g_ptr.resize(static_cast<size_t>(dev) + 1, nullptr);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PD_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return PD_OK;
}

}  // namespace

extern "C" {

int pd_loglike_and_grad_noalloc(const double* theta, int64_t n, int param, const pd_grid* grid,
                                const double* lambda, const double* data, const double* inv_psd, int precision,
                                double* lnl, double* grad, int32_t* status, void* stream) {
    if (!grid) return fail(PD_EINVAL, "grid is NULL");
    if (n <= 0 || grid->n_bins <= 0) return fail(PD_EINVAL, "n and grid n_bins must be > 0");
    if (n > (int64_t(1) << 31) / 64 || grid->n_bins > (int64_t(1) << 28))
        return fail(PD_EINVAL, "n or grid n_bins too large");
    const size_t need = pd::op_workspace_bytes(grad ? PD_OP_LOGLIKE_GRAD : PD_OP_LOGLIKE, n, grid->n_bins);
    if (need == 0 || need > kScratchBytes)
        return fail(PD_EUNSUPPORTED, "batch too large for the fixed scratch array: needs " + std::to_string(need) +
                                         " bytes, the array holds " + std::to_string(kScratchBytes) +
                                         " (PD_NOALLOC_SCRATCH_BYTES)");
    void* ws = nullptr;
    int rc = scratch_ptr(&ws);
    if (rc != PD_OK) return rc;
    // everything on the caller's stream: no side streams or events are created
    return pd::loglike_and_grad(theta, n, param, grid, lambda, data, inv_psd, precision, lnl, grad, status, ws,
                                kScratchBytes, static_cast<hipStream_t>(stream), false, false);
}

}  // extern "C"
