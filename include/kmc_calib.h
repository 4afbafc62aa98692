/*
 * kmc_calib.h — measurement helper exported by the rail-KMC library.
 *
 * kmc_calib_copy copies `bytes` bytes from src to dst (both device memory on
 * the current device, non-overlapping, 16-byte aligned, bytes a multiple of
 * 16) with a plain streaming kernel enqueued on `stream` (a hipStream_t as
 * void*, NULL = null stream).  Profiling this kernel with hardware counters
 * (FETCH_SIZE / WRITE_SIZE) gives the factor between those counters and the
 * bytes actually moved, which converts the counters of the hop kernels into
 * HBM bytes.  Returns KMC_OK, KMC_EINVAL for bad arguments, KMC_EHIP on a
 * launch error.
 */
#ifndef KMC_CALIB_H
#define KMC_CALIB_H
#include <stddef.h>

#include "kmc.h"

#ifdef __cplusplus
extern "C" {
#endif

kmc_status kmc_calib_copy(const void *src, void *dst, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif
