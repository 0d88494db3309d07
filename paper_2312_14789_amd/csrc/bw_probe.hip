// Streaming-read probe (libmlbm_probe.so, include/mlbm_probe.h): the practical
// HBM read bandwidth of a kernel that, like the step, reads far more than it
// writes (16-byte non-temporal loads, one float written per thread).  A
// measurement helper kept out of the method's library.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "mlbm_probe.h"

namespace {

thread_local std::string g_probe_error;

int probe_fail(int code, const char *msg, const char *detail = "") {
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s%s", msg, detail);
    g_probe_error = buf;
    return code;
}

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
    g_probe_error.clear();
    if (!buf || !out) return probe_fail(MLBM_PROBE_ERR_ARG, "null buffer");
    if (((uintptr_t)buf & 15u) || ((uintptr_t)out & 3u)) return probe_fail(MLBM_PROBE_ERR_ARG, "misaligned buffer");
    if (per_thread != 2 && per_thread != 4 && per_thread != 8) return probe_fail(MLBM_PROBE_ERR_ARG, "per_thread must be 2, 4 or 8");
    const int64_t unit = 16 * 256 * (int64_t)per_thread;
    if (bytes < unit || bytes % unit) return probe_fail(MLBM_PROBE_ERR_ARG, "bytes must be a positive multiple of 4096 * per_thread");
    const int64_t grid = bytes / unit;
    if (grid > (int64_t)INT32_MAX) return probe_fail(MLBM_PROBE_ERR_ARG, "buffer too large");
    hipStream_t s = (hipStream_t)stream;
    const f4 *in = (const f4 *)buf;
    if (per_thread == 2) hipLaunchKernelGGL(k_read_probe<2>, dim3((unsigned)grid), dim3(256), 0, s, in, out);
    else if (per_thread == 4) hipLaunchKernelGGL(k_read_probe<4>, dim3((unsigned)grid), dim3(256), 0, s, in, out);
    else hipLaunchKernelGGL(k_read_probe<8>, dim3((unsigned)grid), dim3(256), 0, s, in, out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return probe_fail(MLBM_PROBE_ERR_HIP, "mlbm_read_probe launch: ", hipGetErrorString(e));
    return MLBM_PROBE_OK;
}

extern "C" const char *mlbm_probe_last_error(void) { return g_probe_error.c_str(); }
