/*
 * mcs_ceilings.h -- probes that measure the ceilings the rooflines divide by,
 * on the GPU the library runs on: the issue rate of each VALU instruction the
 * Horner step of Algorithm 1 compiles to (the measured counterpart of the
 * arithmetic cost the paper times on its CPUs in Section 5), the HBM read
 * stream, and the LDS and global atomics the update kernels use.
 * Needs mcs.h.
 */
#ifndef MCS_CEILINGS_H
#define MCS_CEILINGS_H

#include "mcs.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CS_CEIL_VALU_ADD32 = 0,              /* v_add_u32: the full-rate reference */
  CS_CEIL_MAD_U64_U32 = 1,             /* v_mad_u64_u32 (32 x 32 + 64 -> 64) */
  CS_CEIL_LSHL_ADD_U64 = 2,            /* v_lshl_add_u64 */
  CS_CEIL_LSHRREV_B64 = 3,             /* v_lshrrev_b64 */
  CS_CEIL_HBM_READ = 4,                /* 16-byte coalesced loads over the buffer */
  CS_CEIL_LDS_ADD_U64 = 5,             /* ds_add_u64 at random addresses of a 64 KiB table */
  CS_CEIL_LDS_ADD_RTN_U32 = 6,         /* ds_add_rtn_u32 at random addresses of a 64 KiB table */
  CS_CEIL_GLOBAL_ATOMIC_RANDOM = 7,    /* device-scope int64 atomics at random counters */
  CS_CEIL_GLOBAL_ATOMIC_COALESCED = 8, /* the same, a wave's lanes on consecutive counters */
  CS_CEIL_MOV_B32 = 9,                 /* v_mov_b32 (register copy) */
  CS_CEIL_BFE_U32 = 10,                /* v_bfe_u32 (a three-operand 32-bit instruction) */
  CS_CEIL_AND_OR_B32 = 11,             /* v_and_or_b32 */
  CS_CEIL_XAD_U32 = 12,                /* v_xad_u32 */
  CS_CEIL_LSHLREV_B32 = 13,            /* v_lshlrev_b32 (a two-operand shift) */
  CS_CEIL_AND_B32 = 14,                /* v_and_b32 (two-operand) */
  CS_CEIL_ADD_CO_U32 = 15,             /* v_add_co_u32 and v_addc_co_u32 in turn (a 64-bit add in two) */
  CS_CEIL_ADD32_ONE_WAVE = 16,         /* v_add_u32 with one wave per SIMD (1 block per CU) */
  CS_CEIL_MIX_MAD_ADD = 17             /* v_mad_u64_u32 and v_add_u32 in turn */
} cs_ceiling;

/* Enqueues one launch of probe `probe` on `stream` and writes to *ops (host)
 * the number of operations it performs: lane-instructions for the issue
 * probes, bytes read for CS_CEIL_HBM_READ, atomics for the atomic probes.
 *   buffer, bytes  device memory: at least 8 bytes (a sink the probes write
 *                  only in an impossible case) for the issue and LDS probes;
 *                  the region read (at least 1 MiB) for CS_CEIL_HBM_READ; the
 *                  int64 counters for the global-atomic probes (zeroed by the
 *                  caller if their values matter)
 *   iters          loop trips per thread (issue, LDS and atomic probes)
 * The probes run 8 blocks of 256 threads per compute unit (8 waves per SIMD),
 * CS_CEIL_ADD32_ONE_WAVE one block per compute unit.  Returns CS_EINVAL
 * for an unknown probe or a buffer too small for it. */
cs_status cs_ceiling_run(int probe, void* buffer, uint64_t bytes, uint32_t iters, uint64_t* ops, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* MCS_CEILINGS_H */
