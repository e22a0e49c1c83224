// Sampling from correlated batches: the frugal acceptance decision, taken on
// the device amplitudes of one tns_sample_frugal call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "internal.h"

namespace tns {
namespace {

// Frugal rejection sampling (published method of the cited sampling
// literature, applied to the amplitudes of a correlated batch): a candidate
// bitstring with probability p = |amp|^2 is accepted when p * 2^N / M > u for
// its uniform number u (scale = 2^N / M), i.e. with probability
// min(1, 2^N p / M).  One thread per amplitude, FP64.
__global__ void k_frugal_accept(const double *__restrict__ amps, const double *__restrict__ u,
                                double scale, uint8_t *__restrict__ flags, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double re = amps[2 * i], im = amps[2 * i + 1];
        flags[i] = (re * re + im * im) * scale > u[i] ? 1 : 0;
    }
}

}  // namespace

namespace launch {

static void check_launch(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(TNS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void frugal_accept(const double *amps, const double *uniforms, double scale, uint8_t *flags,
                   int64_t n, void *stream) {
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536));
    hipLaunchKernelGGL(k_frugal_accept, dim3(blocks), dim3(256), 0, (hipStream_t)stream, amps, uniforms,
                       scale, flags, n);
    check_launch("frugal_accept");
}

}  // namespace launch
}  // namespace tns
