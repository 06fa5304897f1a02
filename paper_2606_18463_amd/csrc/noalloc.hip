// casgd_fit_noalloc: the dense fit with its workspace in a file-scope device
// array instead of a caller-provided buffer, for callers that cannot
// allocate device memory. Same kernels and launch plan as casgd_fit.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>

#include "internal.hpp"

namespace casgd {

// Upper bound of the workspace this entry point can hold (64 MiB; the dense
// 2^20 x 2048 FP32 fit at b = 64, s = 16 needs about 36 MiB). Every device
// the library runs on holds its own copy until the process ends.
constexpr size_t kScratchBytes = size_t(64) << 20;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// The device address of `scratch` on each device, looked up once per device
// with that device current (the host-side symbol is not a device address).
// Atomic slots (no lock, nothing to destroy at exit): concurrent first calls
// on one device look the address up twice and store the same value.
static std::atomic<void*> g_scratch_ptr[64];

static casgd_status scratch_ptr(void** out) {
    int dev = 0;
    CASGD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) {
        set_error("device index %d out of range", dev);
        return CASGD_EUNSUPPORTED;
    }
    void* p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (!p) {
        CASGD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("hipGetSymbolAddress returned a null address for the scratch array");
            return CASGD_EDEVICE;
        }
        g_scratch_ptr[dev].store(p, std::memory_order_release);
    }
    *out = p;
    return CASGD_OK;
}

// status_out[0] = CASGD_OK / CASGD_ETIMEOUT / CASGD_ENONFINITE from the
// workspace flags (the same precedence as casgd_check).
__global__ void k_flags_to_status(const unsigned* flags, int32_t* status_out) {
    if (threadIdx.x == 0) {
        int32_t st = CASGD_OK;
        if (flags[FLAG_NONFINITE]) st = CASGD_ENONFINITE;
        if (flags[FLAG_TIMEOUT]) st = CASGD_ETIMEOUT;
        status_out[0] = st;
    }
}

}  // namespace casgd

using namespace casgd;

extern "C" casgd_status casgd_fit_noalloc(const casgd_matrix* X, const float* y, float* x,
                                          double eta, double lambda, int32_t b, int32_t s,
                                          uint64_t seed, uint64_t outer_begin, int64_t n_outer,
                                          const casgd_opts* opts, int32_t* status_out,
                                          void* stream) {
    if (X && X->layout == CASGD_CSR) {
        set_error("casgd_fit_noalloc takes a dense X only");
        return CASGD_EUNSUPPORTED;
    }
    size_t need = 0;
    casgd_status rc = casgd_workspace_size(X, b, s, &need);
    if (rc != CASGD_OK) return rc;
    if (need > kScratchBytes) {
        set_error("casgd_fit_noalloc: this problem needs a %zu-byte workspace, more than the "
                  "%zu bytes of the static scratch array (use casgd_fit with a workspace)",
                  need, kScratchBytes);
        return CASGD_EUNSUPPORTED;
    }
    void* ws = nullptr;
    if ((rc = scratch_ptr(&ws)) != CASGD_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    // The array keeps the previous call's contents: clear every flag word
    // (the fit itself clears its barrier, split-K and exchange words).
    if ((rc = run_zero(static_cast<unsigned*>(ws), FLAG_WORDS, st)) != CASGD_OK) return rc;
    rc = casgd_fit(X, y, x, eta, lambda, b, s, seed, outer_begin, n_outer, opts, ws,
                   kScratchBytes, stream);
    if (rc != CASGD_OK) return rc;
    if (status_out) {
        hipLaunchKernelGGL(k_flags_to_status, dim3(1), dim3(64), 0, st,
                           static_cast<const unsigned*>(ws), status_out);
        CASGD_HIP(hipGetLastError());
    }
    return CASGD_OK;
}
