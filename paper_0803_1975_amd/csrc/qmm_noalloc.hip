// qmm_gemm_mod_p without a caller workspace and without any device allocation:
// the packed operands go to `scratch`, a file-scope device array that every GPU
// the library runs on holds until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory, so its
// device address is looked up once per device (with that device current) and
// only that address is handed to the kernels.  No kernel of qmm_gemm_mod_p needs
// its workspace to start at zero (each conversion writes every byte the product
// reads, padding included), so nothing is cleared between calls.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "qmm_internal.h"

namespace {

static __device__ __align__(256) uint8_t scratch[QMM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each device, once looked up

// The device address of the current device's copy of `scratch`.
qmm_status scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return qmm::fail(QMM_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return qmm::fail(QMM_EUNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return qmm::fail(QMM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        if ((uintptr_t)p % 256 != 0) return qmm::fail(QMM_EDEVICE, "scratch is not 256-byte aligned");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return QMM_OK;
}

}  // namespace

extern "C" qmm_status qmm_gemm_mod_p_noalloc(const qmm_plan *plan, int64_t m, int64_t n, int64_t k, uint32_t p,
                                             const uint8_t *A, int64_t lda, const uint8_t *B, int64_t ldb,
                                             uint8_t *C, int64_t ldc, void *stream) {
    if (p < 2 || p > 256) return qmm::fail(QMM_EINVAL, "byte residues need 2 <= p <= 256");
    if (m < 0 || n < 0 || k < 0) return qmm::fail(QMM_EINVAL, "negative size");
    qmm_plan pl;
    qmm_status st;
    if (plan) {
        pl = *plan;
    } else if ((st = qmm_choose_Qd(p, m, n, k, 0, QMM_PATH_AUTO, 0, &pl)) != QMM_OK) {
        return st;
    }
    size_t need = 0;
    if ((st = qmm_gemm_workspace_size(&pl, m, n, k, &need)) != QMM_OK) return st;
    if (need > (size_t)QMM_NOALLOC_SCRATCH_BYTES)
        return qmm::fail(QMM_ENOSPACE, "qmm_gemm_mod_p_noalloc: this product needs " + std::to_string(need) +
                                           " bytes of workspace, above the " +
                                           std::to_string((size_t)QMM_NOALLOC_SCRATCH_BYTES) +
                                           "-byte scratch (use qmm_gemm_mod_p with a caller workspace)");
    void *ws = nullptr;
    if (need > 0 && (st = scratch_address(&ws)) != QMM_OK) return st;
    // the caller's plan (or NULL) as given, so the product is the one qmm_gemm_mod_p runs
    return qmm_gemm_mod_p(plan, m, n, k, p, A, lda, B, ldb, C, ldc, ws, need > 0 ? (size_t)QMM_NOALLOC_SCRATCH_BYTES : 0,
                          stream);
}
