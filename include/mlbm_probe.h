/*
 * mlbm_probe.h - C ABI of libmlbm_probe.so, a bandwidth measurement helper
 * that sits beside the meshless LBM library and is not part of the method.
 *
 * The step kernels of libmlbm.so mostly read (weights, indices, gathered
 * state) and write one state per node.  Timing a plain streaming read on the
 * same device gives the practical read bandwidth against which their
 * measured traffic can be set, next to the published HBM peak.
 */
#ifndef MLBM_PROBE_H
#define MLBM_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLBM_PROBE_OK       0
#define MLBM_PROBE_ERR_ARG -1  /* null or misaligned buffer, bad sizes        */
#define MLBM_PROBE_ERR_HIP -4  /* the launch failed                           */

/*
 * One kernel that reads the device buffer buf (bytes, 16-byte aligned, a
 * positive multiple of 4096 * per_thread) once with 16-byte non-temporal
 * loads, per_thread (2, 4 or 8) loads per thread, and writes one float per
 * thread (the sum of what it read) to the device array out (bytes /
 * (16 * per_thread) floats, 4-byte aligned).  Both buffers are owned by the
 * caller; the launch is asynchronous on hip_stream (NULL = default stream).
 * Errors: MLBM_PROBE_ERR_ARG, MLBM_PROBE_ERR_HIP; the message of the last
 * failure on the calling thread is returned by mlbm_probe_last_error().
 */
int mlbm_read_probe(const void *buf, int64_t bytes, int32_t per_thread, float *out, void *hip_stream);

const char *mlbm_probe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MLBM_PROBE_H */
