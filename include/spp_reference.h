/*
 * spp_reference.h -- measurement reference shipped with the solver library:
 * a plain device-to-device copy at the streaming rate of the memory system.
 *
 * The memory-bound kernels of the solver (the FFTs along phi, the face
 * fluxes, the momentum source) read and write whole fields once.  Their
 * rates are reported beside the HBM peak and beside the rate this copy
 * reaches on the same device in the same process: one read stream and one
 * write stream of 16-byte accesses, several in flight per thread, over
 * enough workgroups to fill every compute unit.
 */
#ifndef SPP_REFERENCE_H
#define SPP_REFERENCE_H

#include <stddef.h>

#include "sphpoisson.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Copies `bytes` bytes from src_dev to dst_dev on `stream` (hipStream_t as
 * void*; NULL: the null stream).  Both are device pointers of the current
 * device, 16-byte aligned, and the ranges do not overlap; `bytes` is a
 * multiple of 16 (0 enqueues nothing).  Work is only enqueued; the library
 * allocates nothing.
 * Errors: SPP_EINVAL for a NULL pointer with bytes > 0, a misaligned pointer
 * or a size not a multiple of 16; SPP_EDEVICE when the launch fails. */
spp_status spp_stream_copy(const void* src_dev, void* dst_dev, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SPP_REFERENCE_H */
