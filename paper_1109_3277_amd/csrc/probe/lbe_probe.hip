// liblbe_probe: calibration copy for hardware traffic counters, kept out of
// the method's library. A profiler's fetch / write byte counters read for this
// plain streaming copy of a known size give the factor that turns the same
// counters of a kernel into bytes.
//
//   extern "C" int lbe_probe_copy(void* dev_dst, const void* dev_src,
//                                 size_t bytes, void* hip_stream);
//
// Copies `bytes` (a multiple of 16) from dev_src to dev_dst (device memory,
// not overlapping) on hip_stream (hipStream_t as void*, NULL = default stream)
// and returns 0, or -1 for a bad argument and -3 for a launch error.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

__global__ void k_probe_copy16(const uint4* __restrict__ a, uint4* __restrict__ b, size_t n) {
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        b[k] = a[k];
}

extern "C" int lbe_probe_copy(void* dev_dst, const void* dev_src, size_t bytes, void* hip_stream) {
    if (!dev_dst || !dev_src || bytes % 16 != 0) return -1;
    const size_t n = bytes / 16;
    size_t g = (n + 255) / 256;
    if (g > (1u << 20)) g = 1u << 20;
    if (g == 0) g = 1;
    hipLaunchKernelGGL(k_probe_copy16, dim3((unsigned)g), dim3(256), 0, (hipStream_t)hip_stream,
                       (const uint4*)dev_src, (uint4*)dev_dst, n);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
