/*
 * mcs_batch.h -- batched Count Sketch update: many independent sketches
 * (same prime, mode and polynomial degree; each with its own coefficients,
 * table size and stream) updated by a few persistent launches instead of one
 * launch per sketch.  Each sketch's result is exactly what cs_update on that
 * sketch alone gives (Algorithm 2, Process, for every key of its stream).
 * Needs mcs.h.
 */
#ifndef MCS_BATCH_H
#define MCS_BATCH_H

#include "mcs.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One member of a batch: the sketch and its stream (device pointers, n keys
 * and n weights).  The pointers are kept by the batch: every cs_batch_update
 * reads the current contents of the same buffers. */
typedef struct {
  cs_sketch* sketch;
  const void* keys;
  const void* weights;
  uint64_t n;
} cs_batch_item;

/* Tuning knobs (0 = default).  A sketch is updated
 *   - with direct device-scope atomics when n < direct_fraction * buckets
 *     (default 1/8; negative: never), where fewer updates reach the table
 *     than clearing and flushing a per-block copy would touch,
 *   - in LDS with int64 counters when rows*buckets*8 <= lds_table_max
 *     (default 8, which puts no table there, or 65536 when row_resident is
 *     negative; at most 163840),
 *   - else row-resident when a row of 16-bit fields fits a block's LDS
 *     (buckets <= 2^16; the single-sketch row-resident update, one row group
 *     of one sketch per work item), unless row_resident is negative,
 *   - else with the two-pass update (buckets <= 2^18 and rows <= 16 here).
 * Row-resident and direct members share one persistent launch whose blocks
 * take (sketch, row group, key range) items from a queue, largest first.
 * keys_per_thread: keys per lane of a wave tile in that launch, 2, 4 or 8
 *   (default 8).
 * lds_chunk_keys: keys per LDS work item (default 65536).
 * combine: the two-pass update combines repeated keys inside tiles (default 1;
 *   set -1 to disable).
 * use_graph: capture the launches once into a HIP graph and replay it
 *   (default 1; set -1 to disable). */
typedef struct {
  uint32_t lds_table_max;
  uint32_t lds_chunk_keys;
  int combine;
  int use_graph;
  double direct_fraction;
  uint32_t keys_per_thread;
  int row_resident;
} cs_batch_options;

typedef struct cs_batch cs_batch;

/* Builds a batch over `count` items.  All sketches must live on the current
 * device and share prime, mode and k; key_type / weight_type apply to every
 * item.  opts may be NULL.  Allocates the batch's descriptors and workspace
 * (freed by cs_batch_destroy); the sketches stay owned by the caller and must
 * outlive the batch. */
cs_status cs_batch_create(const cs_batch_item* items, uint32_t count, cs_dtype key_type, cs_dtype weight_type,
                          const cs_batch_options* opts, cs_batch** out);
/* Enqueues one update of every member on `stream` (adds each stream into its
 * sketch, as cs_update would). */
cs_status cs_batch_update(cs_batch* b, hipStream_t stream);
/* Tunes the options on the real batch and writes the choice to *chosen (may
 * be NULL); use_graph is kept.  It first tries every combination of the class
 * limits (row-resident on or off; LDS table limit 8, 20480, 40960, 65536 or
 * 163840 bytes; direct fraction 1/128, 1/8 or 1), then, from the fastest,
 * keys per thread 2, 4 and 8, LDS chunk 2^15 and 2^17 keys and combining on and
 * off, one knob at a time.  Each candidate is timed as the median of three
 * updates after a warm-up.  The members' counters and flags are copied aside
 * first and put back at the end, so the sketches keep what they held (this
 * needs device memory for one copy of every member's table).  Synchronises
 * `stream`. */
cs_status cs_batch_autotune(cs_batch* b, hipStream_t stream, cs_batch_options* chosen);
cs_status cs_batch_get_options(const cs_batch* b, cs_batch_options* out);
/* Counts of members per update class: direct atomics, LDS (int64 counters),
 * row-resident, two-pass.  Any pointer may be NULL. */
cs_status cs_batch_classes(const cs_batch* b, uint32_t* n_global, uint32_t* n_lds, uint32_t* n_rows,
                           uint32_t* n_twopass);
/* Waits for the batch's work and frees it.  NULL is accepted. */
void cs_batch_destroy(cs_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* MCS_BATCH_H */
