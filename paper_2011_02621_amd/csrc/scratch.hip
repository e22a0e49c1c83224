// Static device workspace of tns_amplitudes_noalloc.
//
// Callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc) get a workspace that
// exists from module load to process end: one file-scope device array per
// GPU.  In host code the array's name is only a host-side stand-in; the
// array's device address is looked up once per device with
// hipGetSymbolAddress (with that device current, from tns_init) and only that
// address is ever handed to kernels or copies.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"

namespace tns {

static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

void scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) fail(TNS_E_UNSUPPORTED, "device index beyond the static workspace table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        fail(TNS_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[device] = ptr;
}

void *scratch_device_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace tns
