// Streaming-read probe: the practical HBM read bandwidth of a kernel that,
// like the step, reads far more than it writes (16-byte non-temporal loads,
// one float written per thread).  Measurement helper, not part of the method.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mlbm.h"
#include "mlbm_internal.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

template <int U>
__global__ void __launch_bounds__(256) k_read_probe(const f4 *__restrict__ in, float *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    float s = 0.f;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const f4 v = __builtin_nontemporal_load(in + t + u * stride);
        s += v.x + v.y + v.z + v.w;
    }
    out[t] = s;
}

}  // namespace

extern "C" int mlbm_read_probe(const void *buf, int64_t bytes, int32_t per_thread, float *out, void *stream) {
    using mlbm::fail;
    mlbm::clear_error();
    if (!buf || !out) return fail(MLBM_ERR_ARG, "null buffer");
    if (((uintptr_t)buf & 15u) != 0) return fail(MLBM_ERR_ARG, "buffer not 16-byte aligned");
    if (per_thread != 2 && per_thread != 4 && per_thread != 8) return fail(MLBM_ERR_ARG, "per_thread must be 2, 4 or 8");
    const int64_t quantum = 16LL * 256 * per_thread;
    if (bytes <= 0 || bytes % quantum != 0) return fail(MLBM_ERR_ARG, "bytes must be a positive multiple of %lld", (long long)quantum);
    const int64_t grid = bytes / quantum;
    if (grid > INT32_MAX) return fail(MLBM_ERR_ARG, "buffer too large");
    hipStream_t s = (hipStream_t)stream;
    const f4 *in = (const f4 *)buf;
    if (per_thread == 2) hipLaunchKernelGGL(k_read_probe<2>, dim3((unsigned)grid), dim3(256), 0, s, in, out);
    else if (per_thread == 4) hipLaunchKernelGGL(k_read_probe<4>, dim3((unsigned)grid), dim3(256), 0, s, in, out);
    else hipLaunchKernelGGL(k_read_probe<8>, dim3((unsigned)grid), dim3(256), 0, s, in, out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MLBM_ERR_HIP, "mlbm_read_probe launch: %s", hipGetErrorString(e));
    return MLBM_OK;
}
