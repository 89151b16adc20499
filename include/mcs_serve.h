/*
 * mcs_serve.h -- serving runtime for many tenants' Count Sketches on one
 * MI355X: tenants are admitted against a device-memory budget, update and
 * F2 requests are queued, and one worker thread runs them in continuous
 * batches (every step takes the queued updates of all tenants into one
 * batched update, then answers the F2 queries that were waiting on them).
 *
 * The arithmetic is exactly that of cs_update and cs_estimate_f2 (Algorithm 2
 * of Ahle, Knudsen and Thorup, arXiv 2008.08654, with the hashing of
 * Algorithm 1 and the sign/bucket split of Algorithm 3).  The counters are
 * integers and the sketch is linear (Section 1.3.1), so a tenant's counters
 * and answers do not depend on which other tenants' requests share its steps.
 *
 * Ordering: requests of one tenant take effect in submission order.  An F2
 * request sees exactly the updates of its tenant submitted before it.
 * Requests of different tenants are not ordered with respect to each other.
 *
 * Key and weight buffers of an update are caller-owned device memory and
 * must stay valid and unchanged until the update's ticket completes.  The
 * server reads them on a stream of its own, which is not ordered with the
 * caller's streams: their contents must be complete when the update is
 * submitted (a caller that fills them asynchronously synchronises that work,
 * for example its stream, before submitting).
 * All calls are thread-safe.
 */
#ifndef MCS_SERVE_H
#define MCS_SERVE_H

#include "mcs.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cs_server cs_server; /* opaque, library-owned */

typedef struct {
  /* Device bytes the server may hold: the sketches of admitted tenants plus
   * the server's own step buffers (two-pass workspace, work lists).
   * 0 selects 64 GiB. */
  uint64_t hbm_budget;
  /* Most update keys one step takes (0: 2^26).  A request with more keys
   * runs in a step of its own. */
  uint64_t step_keys;
  /* Two-pass workspace of a step in bytes (0: 2 GiB, enough for the records
   * of a full default step in one round); a step whose records exceed it
   * runs in several rounds over the same workspace. */
  uint64_t work_bytes;
  /* An update with n < direct_fraction * buckets keys goes to the table with
   * direct atomics instead of the two-pass update (as in cs_batch_options;
   * 0: 1/128, negative: never). */
  double direct_fraction;
} cs_server_options;

typedef enum { CS_REQ_UPDATE = 0, CS_REQ_F2 = 1 } cs_request_kind;

typedef struct {
  cs_status status;    /* CS_OK, or the F2 call's error (CS_EDOMAIN, CS_EOVERFLOW) */
  int64_t f2;          /* F2 requests: median of the row estimates; updates: 0 */
  uint64_t arrival_ns; /* submission (replay: scheduled arrival) time, steady clock */
  uint64_t done_ns;    /* time the worker saw the step complete, same clock */
  uint64_t step;       /* index of the step that ran the request */
} cs_server_result;

/* One request of a trace for cs_server_replay. */
typedef struct {
  uint32_t tenant;
  uint32_t kind;       /* cs_request_kind */
  const void* keys;    /* device, n values (updates only) */
  const void* weights; /* device, n values (updates only) */
  uint64_t n;
} cs_server_request;

typedef struct {
  uint64_t steps;          /* steps run */
  uint64_t requests;       /* requests completed */
  uint64_t keys;           /* update keys processed */
  uint64_t resident_bytes; /* device bytes held (tenants and step buffers) */
  uint64_t budget_bytes;
  uint32_t tenants;        /* admitted tenants */
} cs_server_stats;

/* Creates a server on the current HIP device for sketches over `prime`
 * (CS_P61 or CS_P89) in `mode` with k coefficients per polynomial, for keys
 * of key_type (CS_U32, CS_U64) and weights of weight_type (CS_I32, CS_I64).
 * opts may be NULL (all defaults).  CS_EBUSY if the step buffers alone
 * exceed the budget. */
cs_status cs_server_create(cs_prime prime, cs_mode mode, uint32_t k, cs_dtype key_type, cs_dtype weight_type,
                           const cs_server_options* opts, cs_server** out);

/* Admits a tenant with a sketch of `rows` rows and `buckets` = 2^l counters
 * per row, coefficients from `seed` (as cs_create_ex).  rows <= 16 and
 * buckets <= 2^18 (the shapes of the batched update).  CS_EBUSY, with
 * nothing allocated, if its sketch would take the server past its budget.
 * *tenant receives the tenant's id. */
cs_status cs_server_admit(cs_server* s, uint32_t rows, uint64_t buckets, uint64_t seed, uint32_t* tenant);
/* Waits until the tenant's submitted requests have completed, then frees its
 * sketch and returns its bytes to the budget.  Later requests for it fail
 * with CS_EINVAL. */
cs_status cs_server_evict(cs_server* s, uint32_t tenant);

/* Queue an update (n keys and weights, device) or an F2 request; *ticket
 * (may be NULL for updates) identifies it for cs_server_wait. */
cs_status cs_server_submit_update(cs_server* s, uint32_t tenant, const void* keys, const void* weights, uint64_t n,
                                  uint64_t* ticket);
cs_status cs_server_submit_f2(cs_server* s, uint32_t tenant, uint64_t* ticket);
/* Blocks until the ticket's request has completed and returns its result
 * (host).  A ticket can be waited for once. */
cs_status cs_server_wait(cs_server* s, uint64_t ticket, cs_server_result* out);
/* Blocks until every request submitted so far has completed. */
cs_status cs_server_drain(cs_server* s);
/* Copies a tenant's counters (rows * buckets int64, row-major) to host memory
 * once its submitted requests have completed. */
cs_status cs_server_read_counters(cs_server* s, uint32_t tenant, int64_t* host_dst);
cs_status cs_server_get_stats(cs_server* s, cs_server_stats* out);

/* Open-loop load generator: submits request i at arrival_s[i] seconds (host,
 * non-decreasing) after the call starts, each with that scheduled time as its
 * arrival, then waits for all of them and writes results[i] (host).  Latency
 * is results[i].done_ns - results[i].arrival_ns, so time a request spends
 * behind a late submission counts. */
cs_status cs_server_replay(cs_server* s, const cs_server_request* reqs, uint32_t count, const double* arrival_s,
                           cs_server_result* results);

/* Drains the queue, stops the worker and frees every tenant.  NULL is accepted. */
void cs_server_destroy(cs_server* s);

#ifdef __cplusplus
}
#endif
#endif /* MCS_SERVE_H */
