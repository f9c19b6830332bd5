/*
 * fwi_calib.h -- measurement aid of the library (not part of the paper's
 * computation): a STREAM-style device copy of known size, used to measure
 * the HBM rate a plain streaming kernel attains on the device and to scale
 * hardware traffic counters (FETCH_SIZE, WRITE_SIZE) to bytes.
 */
#ifndef FWI_MI355X_CALIB_H
#define FWI_MI355X_CALIB_H

#include <stddef.h>

#include "fwi.h"

#ifdef __cplusplus
extern "C" {
#endif

/* dst[0..bytes) = src[0..bytes) on the device (DEVICE pointers, 16-byte
 * aligned, bytes a multiple of 16, no overlap), enqueued on `stream`
 * (hipStream_t, NULL = default).  `variant` selects the launch form:
 *   bit 0      non-temporal loads and stores (bypass the caches' retention);
 *   bit 1      four 16-byte elements per thread per pass instead of one;
 *   bits 2..3  grid: 0 one pass over the array, 1 2048 workgroups, 2 8192
 *              workgroups (grid-stride loops).
 * FWI_EINVAL for bad sizes, alignment or variant; FWI_EHIP if the launch
 * fails.  Reads `bytes` and writes `bytes`. */
int fwi_calib_copy(void *dst, const void *src, size_t bytes, int variant, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FWI_MI355X_CALIB_H */
