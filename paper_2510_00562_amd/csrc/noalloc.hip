// geo_project_l1_noalloc: the l1-ball projection of geo_project_l1 with its
// scratch (the threshold search state and one radix level's histogram) in a
// fixed device array of this library instead of a caller workspace, and the
// threshold written to device memory: the call allocates nothing, copies
// nothing to the host and does not synchronise, so it can be captured into
// a HIP graph or issued from loops that may not allocate.
#include <math.h>

#include <mutex>

#include "solver.hpp"

namespace geo {
namespace {

// Bytes of the fixed scratch: the search state (one 256-byte-aligned slot)
// and the histogram of one field at the widest radix level.
constexpr size_t kL1StateBytes = 256;
constexpr size_t kL1ScratchBytes = 32768;
static_assert(sizeof(SelState) <= kL1StateBytes, "search state slot");
static_assert(kL1StateBytes + sizeof(Hist) <= kL1ScratchBytes, "scratch holds state and histogram");

// One copy per device, held until the process ends. Host code reaches it
// only through the address hipGetSymbolAddress gives on each device.
static __device__ __align__(256) unsigned char scratch[kL1ScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch` on each device (null: not yet)

// The scratch's address on the current device, looked up on the first call
// on that device (with it current). Returns null and sets *err on failure.
void *device_scratch(hipError_t *err)
{
    int dev = 0;
    *err = hipGetDevice(&dev);
    if (*err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) return nullptr;
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

__global__ void k_tau_out(const SelState *sel, double *tau)
{
    if (threadIdx.x == 0) *tau = sel->tau;
}

}  // namespace
}  // namespace geo

using namespace geo;

extern "C" int geo_project_l1_noalloc(const float *x, int64_t n, double radius, float *out,
                                      double *tau_dev, void *stream)
{
    if (n < 0 || n > (int64_t)0x7fffffff || !isfinite(radius) || radius < 0.0 || (n > 0 && (!x || !out)))
        return GEO_EINVAL;
    hipError_t e = hipSuccess;
    char *ws = (char *)device_scratch(&e);
    if (!ws) return geo_hip_status(e);
    const hipStream_t st = (hipStream_t)stream;
    // the search state and the histogram are reset by the first launch
    SelState *sel = (SelState *)ws;
    Hist *hist = (Hist *)(ws + kL1StateBytes);
    e = launch_l1_threshold(x, n, radius, sel, hist, st);
    if (e == hipSuccess && n > 0) e = launch_soft(x, n, sel, out, st);
    if (e == hipSuccess && tau_dev) {
        hipLaunchKernelGGL(k_tau_out, dim3(1), dim3(64), 0, st, (const SelState *)sel, tau_dev);
        e = hipGetLastError();
    }
    return geo_hip_status(e);
}
