/* amh_yardstick.h -- C ABI of the achievable-bandwidth yardsticks in libamh.so.
 *
 * These calls are not part of the sampler.  They measure what the memory system of
 * the GPU at hand delivers to the access patterns of the sweep kernel, so that its
 * measured rates can be stated as fractions of achievable, not only of published,
 * figures.  The pattern they stand for is the pair sum of the energy mapped onto the
 * GPU (Sec. 2.4: one pair per thread, then a reduction), which here gathers one
 * 16-byte spline stencil per near pair from the distogram table.
 *
 * Every call launches one kernel on `stream` (a hipStream_t, NULL = default) and
 * returns at once; time it with events on that stream.  All pointers are device
 * pointers owned by the caller.  Invalid arguments give AMH_E_INVAL with nothing
 * launched; a failed launch gives AMH_E_DEVICE.
 */
#ifndef AMH_YARDSTICK_H
#define AMH_YARDSTICK_H

#include <stdint.h>

#include "amh.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Streaming read: `blocks` workgroups of 256 threads read the n_float4 16-byte
 * elements of src_dev once (coalesced, grid-stride).  sink_dev: float[blocks * 256],
 * written (one value per thread).  Bytes moved: 16 n_float4. */
amh_status amh_yard_stream(const float* src_dev, int64_t n_float4, int32_t blocks, float* sink_dev,
                           void* stream);

/* Independent 16-byte gathers from a table of `rows` rows of `stride` floats (the
 * padded distogram layout): each of the blocks * 256 threads makes per_thread reads of
 * the 4 floats at row * stride + bin, row uniform on [0, rows), bin uniform on
 * [0, max_bin]; needs max_bin + 4 <= stride.  sink_dev: float[blocks * 256].
 * Useful bytes: 16 * blocks * 256 * per_thread. */
amh_status amh_yard_gather(const float* table_dev, int64_t rows, int32_t stride, int32_t max_bin,
                           int32_t per_thread, int32_t blocks, float* sink_dev, void* stream);

/* LDS reads: `blocks` workgroups of 512 threads each read per_thread float4 values
 * from a 64-KiB LDS block at strided addresses.  sink_dev: float[blocks * 512].
 * Bytes read from LDS: 16 * blocks * 512 * per_thread. */
amh_status amh_yard_lds(int32_t per_thread, int32_t blocks, float* sink_dev, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* AMH_YARDSTICK_H */
