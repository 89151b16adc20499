/*
 * mcs_noalloc.h -- an update entry point that allocates nothing, for callers
 * that cannot call hipMalloc: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  Needs mcs.h.
 */
#ifndef MCS_NOALLOC_H
#define MCS_NOALLOC_H

#include "mcs.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Size of the library's fixed scratch array: one copy per device the library
 * runs on, held from the library's load until the process ends. */
#define CS_NOALLOC_SCRATCH_BYTES (64u << 20)

/* cs_update with the same arguments, kernels and result, except that the
 * two-pass path (BINNED) keeps its records and group offsets in the scratch
 * array instead of the sketch's workspace: it runs in rounds of as many keys
 * as the array holds (about 64 MiB / (4.25 * rows) keys per round).  No call
 * allocates or frees device or host memory.  The other paths need no scratch.
 * Errors: CS_EINVAL for the arguments cs_update rejects, when the sketch does
 * not live on the current device, or when one round of a single tile would
 * not fit the array (it always fits for rows <= 64).  Every call on a device
 * shares that device's array and leaves its contents behind (each round
 * writes all it reads): calls that overlap in time on one device, on any
 * streams, race and give undefined counters; order them, for example on one
 * stream. */
cs_status cs_update_noalloc(cs_sketch* s, const void* keys, cs_dtype key_type, const void* weights,
                            cs_dtype weight_type, uint64_t n, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* MCS_NOALLOC_H */
