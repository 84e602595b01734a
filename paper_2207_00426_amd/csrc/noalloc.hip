// pss_ipls_iterate_noalloc: the iterated smoother with its workspace in a
// file-scope device array instead of caller memory, for callers that cannot
// allocate device memory.
#include <mutex>
#include <string>

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace pss {

// Largest workspace the array holds; problems needing more are refused.
constexpr size_t kScratchBytes = size_t(64) << 20;

// One copy per GPU, held for the life of the process.  In host code this
// name is only a stand-in for the symbol: device code is handed the address
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// address of the current device's copy of `scratch`, looked up once per
// device with that device current
int scratch_ptr(void **out)
{
    int dev = -1;
    int rc = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (rc)
        return rc;
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("noalloc: device index out of range");
        return PSS_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                       "hipGetSymbolAddress(scratch)");
        if (rc)
            return rc;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PSS_OK;
}
} // namespace

} // namespace pss

using namespace pss;

extern "C" {

size_t pss_noalloc_max_bytes(void) { return kScratchBytes; }

int pss_ipls_iterate_noalloc(const pss_problem *p, const pss_gamma *g, const void *y,
                             int32_t n_iter, void *m_nom, void *N_nom, void *m_f, void *N_f,
                             hipStream_t stream)
{
    try {
        int rc = pss_validate(p);
        if (rc)
            return rc;
        const size_t need = pss_workspace_size(p, PSS_OP_IPLS);
        if (need > kScratchBytes) {
            set_error("ipls_iterate_noalloc: the problem needs " + std::to_string(need) +
                      " bytes of workspace, more than the " + std::to_string(kScratchBytes) +
                      " bytes of the library's static scratch array; use pss_ipls_iterate with "
                      "a caller workspace");
            return PSS_EWORKSPACE;
        }
        void *ws = nullptr;
        rc = scratch_ptr(&ws);
        if (rc)
            return rc;
        // the IPLS passes read nothing from the workspace that they have not
        // written earlier in the same call, so no clearing is needed
        return pss_ipls_iterate(p, g, y, n_iter, m_nom, N_nom, m_f, N_f, ws, kScratchBytes,
                                stream);
    } catch (...) {
        set_error("exception in pss_ipls_iterate_noalloc");
        return PSS_EINVAL;
    }
}

} // extern "C"
