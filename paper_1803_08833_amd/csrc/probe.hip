// probe.hip -- device capability probe used by the benchmark (not part of the
// method): the rate of scattered device-scope int32 atomic adds, the unit of
// direct delivery, against which the delivery kernels' atomic throughput is
// read.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "snn.h"

namespace {

// Add number i goes to a hashed word of the buffer (a 64-bit mix of i), so
// consecutive lanes hit unrelated cache lines, as a spike's targets do.
__global__ __launch_bounds__(256) void k_probe_atomics(int32_t* buf, uint64_t n_targets, uint64_t n_adds)
{
    const uint64_t stride = (uint64_t)gridDim.x * 256u;
    for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < n_adds; i += stride) {
        uint64_t h = i * 0x9E3779B97F4A7C15ull;
        h ^= h >> 29;
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 32;
        __hip_atomic_fetch_add(buf + (h % n_targets), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace

extern "C" snn_status snn_probe_atomics(uint64_t n_targets, uint64_t n_adds, void* hip_stream, double* adds_per_s)
{
    if (n_targets == 0 || n_adds == 0 || !adds_per_s) return SNN_E_INVAL;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int32_t* buf = nullptr;
    if (hipMalloc(&buf, n_targets * 4) != hipSuccess) return SNN_E_NOMEM;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipMemsetAsync(buf, 0, n_targets * 4, s);
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    const uint32_t grid = 256u * 64u;
    if (e == hipSuccess) {   // one launch untimed (warm caches and clocks), one timed
        hipLaunchKernelGGL(k_probe_atomics, dim3(grid), dim3(256), 0, s, buf, n_targets, n_adds);
        e = hipEventRecord(a, s);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_probe_atomics, dim3(grid), dim3(256), 0, s, buf, n_targets, n_adds);
        e = hipEventRecord(b, s);
    }
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipFree(buf);
    if (e != hipSuccess || ms <= 0.0f) return SNN_E_HIP;
    *adds_per_s = (double)n_adds / (ms * 1e-3);
    return SNN_OK;
}
