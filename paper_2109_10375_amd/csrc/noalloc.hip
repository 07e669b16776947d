// amber_zre for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid allocation): the
// same ranking and matching launches as amber_zre, with their scratch in a
// library-owned static device array instead of a caller workspace.
//
// The array is part of the library's code object, so every device the
// library runs on holds one copy of it until the process ends.  Its device
// address is looked up once per device at plan creation (with that device
// current) and kept in the plan; host code never passes the array's own name
// to a kernel, whose host-side value is not a device address.  Calls on one
// device share its copy, so calls that overlap in time on one device race:
// the caller orders them (one stream, or events between streams).  Every
// region a call relies on starting at zero is cleared by that call's own
// kernels, exactly as in a fresh workspace.
#include <mutex>

#include "internal.h"

namespace {

constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[AMBER_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

int noalloc_scratch_address(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return AMBER_E_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return AMBER_E_HIP;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return AMBER_OK;
}

extern "C" int amber_zre_noalloc(amber_plan plan, const float* d_J, const float* d_w, const amber_weibull* hist,
                                 int n_hist, float* const* d_zre, void* stream) {
    if (!plan) return AMBER_E_ARG;
    if (plan->n > AMBER_NOALLOC_MAX_N) return AMBER_E_SIZE;
    if (!plan->d_scratch) return AMBER_E_HIP;  // the address lookup failed at plan creation
    const WsLayout L = ws_layout(plan->n, 1);
    if (L.total > (size_t)AMBER_NOALLOC_SCRATCH_BYTES) return AMBER_E_SIZE;
    return amber_zre(plan, d_J, d_w, hist, n_hist, d_zre, plan->d_scratch, L.total, stream);
}
