/*
 * npm_probe.h -- achievable rates of the device, measured by libnpm itself.
 *
 * The fractions of peak that the benchmark reports for the hot-path kernels
 * are taken against the published MI355X peaks (8 TB/s HBM3E, 157.3 TFLOP/s
 * FP32 and 2.5 PFLOP/s BF16 dense matrix throughput).  This call measures
 * what the same device reaches with plain kernels that do nothing else, so
 * that each kernel can also be put against an achievable ceiling.  It is not
 * part of the method of the paper; it exists for that measurement only.
 */
#ifndef NPM_PROBE_H
#define NPM_PROBE_H

#include "npm.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * out[0]  FP32 matrix rate, TFLOP/s: v_mfma_f32_32x32x2_f32 in four
 *         independent accumulator chains per wave, four waves per SIMD;
 * out[1]  BF16 matrix rate, TFLOP/s: v_mfma_f32_32x32x16_bf16, the same way;
 * out[2]  HBM read rate, GB/s (1e9 bytes/s): one pass of 16-byte loads over a
 *         2 GiB buffer (eight times the 256 MB Infinity Cache);
 * out[3]  HBM copy rate, GB/s of bytes read plus bytes written: 1 GiB copied
 *         into another 1 GiB with 16-byte loads and stores.
 * Each figure is the best of `reps` timed launches (HIP events) after one
 * untimed launch.  The call allocates 3 GiB of device memory on the current
 * device for its duration, frees it, and synchronises the device.
 * Errors: NPM_ERR_INVALID_ARG for a null `out` or reps < 1 (checked first,
 * without touching a device); NPM_ERR_NO_DEVICE without a gfx950 device;
 * NPM_ERR_OOM if the buffers cannot be allocated; NPM_ERR_HIP for a failed
 * launch or event.  `out` is written only on success.
 */
npm_status npm_measure_peaks(double out[4], int32_t reps);

#ifdef __cplusplus
}
#endif

#endif /* NPM_PROBE_H */
