// serve_host.cpp -- host side of include/mcs_serve.h: tenant admission
// against a device-memory budget, a request queue, and one worker thread that
// runs continuous batches on its own stream.
//
// A step takes queued requests in arrival order: all updates (up to the step's
// key limit) become one batched update (the classes and kernels of the
// batched path, planned per step, launched without a graph since every step
// has another shape), and the step's F2 requests are estimated after it.  A
// tenant's update that arrives after one of its F2 requests in the step waits
// for a later step, and so does every later request of that tenant; other
// tenants' requests behind it still join the step.  So each tenant's requests
// in a step are a prefix of its queued requests with its updates before its
// F2 requests, and every answer sees exactly the updates submitted before it.  Two steps can
// be in flight: the next is planned and enqueued while the GPU runs the
// previous one; each has its own work-list buffers, and both share the
// two-pass workspace, which stream order makes safe.
#include <hip/hip_runtime.h>

#include <sys/prctl.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "mcs.h"
#include "mcs_batch.h"
#include "mcs_internal.hpp"
#include "mcs_serve.h"
#include "sketch_kernels.hpp"

using namespace mcs;

namespace {

constexpr uint64_t kDefaultBudget = 64ull << 30;
constexpr uint64_t kDefaultStepKeys = 1ull << 26;
constexpr uint64_t kDefaultWork = 2ull << 30;
constexpr size_t kListsInit = 4u << 20;
constexpr size_t kResultWords = 32768;  // pinned int64 F2 outputs per step
constexpr int kDepth = 2;               // steps in flight
constexpr size_t kScanMax = 16384;      // queued requests one step looks at
constexpr int kIdlePollUs = 100;        // an idle worker looks at the queue this often
// Served tables are mostly far larger than the last-level cache, where
// random 64-bit atomics cost much more than pass 2's coalesced flushes: only
// the shortest updates take them.
constexpr double kServerDirect = 1.0 / 128;

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  uint64_t ticket;
  uint32_t tenant, kind;
  const void* keys;
  const void* weights;
  uint64_t n;
  uint64_t arrival_ns;
  bool keep;  // someone will wait for the ticket
};

struct Tenant {
  cs_sketch* sk = nullptr;
  size_t bytes = 0;
  uint64_t pending = 0;  // submitted, not completed
  bool evicting = false;
};

struct Slot {  // buffers of one in-flight step
  char* d_lists = nullptr;
  char* h_lists = nullptr;  // pinned staging of the lists
  size_t lists_cap = 0;
  int64_t* d_results = nullptr;  // F2 outputs (median, rows, flags per queried tenant)
  int64_t* h_results = nullptr;  // pinned copy
  hipEvent_t done = nullptr;
};

struct Step {
  std::vector<Request> reqs;
  std::vector<size_t> res_off;  // per request: offset in h_results (F2) or SIZE_MAX
  std::vector<uint32_t> rows;   // per request: rows of the tenant (F2)
  std::vector<std::pair<uint32_t, size_t>> estimates;  // (tenant, offset): one per queried tenant
  size_t result_words = 0;
  int slot = 0;
  uint64_t index = 0;
  uint64_t keys = 0;
  cs_status status = CS_OK;  // a planning or launch error fails the whole step
};

struct DeviceGuard {  // makes `dev` current for the calling thread, restores on exit
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

struct cs_server {
  int device = 0;
  cs_prime cprime = CS_P61;
  cs_mode cmode = CS_TWO_FOR_ONE;
  uint32_t k = 4;
  int prime = kPrime61, mode = 0, kb = 8, wb = 4;
  uint64_t budget = 0, step_keys = 0;
  size_t work_bytes = 0;
  double direct_fraction = 0.0;
  hipStream_t stream = nullptr;
  void* d_work = nullptr;
  Slot slots[kDepth];

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request> queue;
  std::vector<std::unique_ptr<Tenant>> tenants;  // index = tenant id
  std::unordered_set<uint64_t> open;             // tickets that can be waited for
  std::unordered_map<uint64_t, cs_server_result> done;
  uint64_t next_ticket = 1;
  uint64_t submitted = 0, completed = 0;
  uint64_t queued_keys = 0;  // update keys waiting in the queue
  uint64_t resident = 0;
  uint64_t steps = 0, keys_done = 0;
  uint32_t live_tenants = 0;
  bool stop = false;
  std::thread worker;
};

namespace {

void free_slot(Slot& sl) {
  if (sl.d_lists) (void)hipFree(sl.d_lists);
  if (sl.h_lists) (void)hipHostFree(sl.h_lists);
  sl.d_lists = sl.h_lists = nullptr;
  sl.lists_cap = 0;
}

bool alloc_lists(Slot& sl, size_t bytes) {
  free_slot(sl);
  if (hipMalloc(&sl.d_lists, bytes) != hipSuccess) return false;
  if (hipHostMalloc(&sl.h_lists, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(sl.d_lists);
    sl.d_lists = nullptr;
    return false;
  }
  sl.lists_cap = bytes;
  return true;
}

// Takes the next step's requests from the queue (lock held).  A request that
// cannot join (its tenant's F2 is in the step, the key or result limit is
// reached, or an earlier request of its tenant was held back) is held back
// and stays queued, in order, ahead of the requests not looked at.
void form_step(cs_server* S, Step& st) {
  std::unordered_map<uint32_t, size_t> queried;  // tenant -> its estimate's offset
  std::unordered_set<uint32_t> held;             // tenants with a request held back
  std::vector<Request> back;
  size_t scanned = 0;
  while (!S->queue.empty() && scanned < kScanMax) {
    const Request r = S->queue.front();
    S->queue.pop_front();
    ++scanned;
    bool take = !held.count(r.tenant);
    if (take && r.kind == CS_REQ_UPDATE) {
      // this tenant's F2 must not see it; the step's keys are full
      take = !queried.count(r.tenant) && (st.reqs.empty() || st.keys + r.n <= S->step_keys);
      if (take) {
        st.keys += r.n;
        S->queued_keys -= r.n;
        st.res_off.push_back(SIZE_MAX);
        st.rows.push_back(0);
      }
    } else if (take) {
      const uint32_t rows = S->tenants[r.tenant]->sk->rows;
      auto it = queried.find(r.tenant);
      size_t off = 0;
      if (it != queried.end()) {
        off = it->second;  // same tenant, no update in between: same answer
      } else if (st.result_words + rows + 2 > kResultWords) {
        take = false;
      } else {
        off = st.result_words;
        st.result_words += rows + 2;
        queried.emplace(r.tenant, off);
        st.estimates.emplace_back(r.tenant, off);
      }
      if (take) {
        st.res_off.push_back(off);
        st.rows.push_back(rows);
      }
    }
    if (take) {
      st.reqs.push_back(r);
    } else {
      held.insert(r.tenant);
      back.push_back(r);
    }
    if (st.keys >= S->step_keys) break;  // no further update fits
  }
  S->queue.insert(S->queue.begin(), back.begin(), back.end());
}

// Plans and enqueues a step on the server's stream (lock not held): one
// batched update over the step's update requests, then one batched estimate
// over its queried tenants; the work lists of both go up in one copy.
void launch_step(cs_server* S, Step& st) {
  Slot& sl = S->slots[st.slot];
  std::vector<cs_batch_item> items;
  std::vector<cs_sketch*> sks(st.reqs.size()), est_sks(st.estimates.size());
  {
    std::lock_guard<std::mutex> lk(S->mu);
    for (size_t i = 0; i < st.reqs.size(); ++i) sks[i] = S->tenants[st.reqs[i].tenant]->sk;
    for (size_t i = 0; i < st.estimates.size(); ++i) est_sks[i] = S->tenants[st.estimates[i].first]->sk;
  }
  for (size_t i = 0; i < st.reqs.size(); ++i) {
    const Request& r = st.reqs[i];
    if (r.kind == CS_REQ_UPDATE && r.n) items.push_back(cs_batch_item{sks[i], r.keys, r.weights, r.n});
  }
  BatchPlan P;
  if (!items.empty()) {
    BatchPlanLimits lim;
    lim.work_cap = S->work_bytes;
    lim.cus = (uint32_t)device_info(S->device).cus;
    cs_batch_options opts{};
    opts.direct_fraction = S->direct_fraction;
    st.status = batch_plan(items.data(), items.size(), S->kb, S->wb, opts, lim, &P);
    if (st.status != CS_OK) return;
  }
  const size_t est_off = (P.lists_bytes + 255) & ~(size_t)255;
  const size_t need = est_off + st.estimates.size() * sizeof(BatchEstItem);
  if (need > sl.lists_cap) {
    // this slot's previous step has completed, so its buffers are free
    const size_t old_cap = sl.lists_cap;
    size_t cap = std::max<size_t>(old_cap, kListsInit);
    while (cap < need) cap *= 2;
    if (!alloc_lists(sl, cap)) {
      std::lock_guard<std::mutex> lk(S->mu);
      S->resident -= old_cap;
      st.status = fail(CS_ENOMEM, "step work lists of %zu bytes", cap);
      return;
    }
    std::lock_guard<std::mutex> lk(S->mu);
    S->resident += cap - old_cap;  // counted against the budget like the rest
  }
  const DeviceInfo& dev = device_info(S->device);
  BatchLaunch L{};
  std::vector<BatchRound> rounds;
  if (!items.empty())
    batch_emit(P, S->prime, S->mode, (int)S->k, S->kb, S->wb, dev, sl.d_lists, (char*)S->d_work, sl.h_lists, &L,
               &rounds);
  BatchEstItem* est = (BatchEstItem*)(sl.h_lists + est_off);
  uint32_t blocks = 0;
  for (size_t i = 0; i < st.estimates.size(); ++i) {
    cs_sketch* s = est_sks[i];
    est[i] = BatchEstItem{s->d_table, (EstPartial*)s->d_est_part, s->d_flags, s->rows, s->log2m, s->est_slices,
                          blocks, st.estimates[i].second};
    blocks += s->rows * s->est_slices;
  }
  hipError_t e = hipSuccess;
  if (need) e = hipMemcpyAsync(sl.d_lists, sl.h_lists, need, hipMemcpyHostToDevice, S->stream);
  if (e == hipSuccess && !items.empty()) e = launch_batch(L, S->stream);
  if (e == hipSuccess && !st.estimates.empty()) {
    e = launch_batch_estimate((const BatchEstItem*)(sl.d_lists + est_off), (uint32_t)st.estimates.size(), blocks,
                              sl.d_results, (uint32_t)dev.cus, S->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(sl.h_results, sl.d_results, st.result_words * sizeof(int64_t), hipMemcpyDeviceToHost,
                         S->stream);
  }
  if (e != hipSuccess) st.status = hip_fail(e, "step launch");
}

// Waits for a launched step and publishes its results.
void complete_step(cs_server* S, Step& st, bool launched) {
  cs_status dev_status = CS_OK;
  if (launched && hipEventSynchronize(S->slots[st.slot].done) != hipSuccess)
    dev_status = fail(CS_EDEVICE, "step did not complete");
  const uint64_t t = now_ns();
  const int64_t* res = S->slots[st.slot].h_results;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    for (size_t i = 0; i < st.reqs.size(); ++i) {
      const Request& r = st.reqs[i];
      cs_server_result out{};
      out.status = st.status != CS_OK ? st.status : dev_status;
      out.arrival_ns = r.arrival_ns;
      out.done_ns = t;
      out.step = st.index;
      if (r.kind == CS_REQ_F2 && out.status == CS_OK) {
        out.f2 = res[st.res_off[i]];
        out.status = flags_status((uint32_t)res[st.res_off[i] + 1 + st.rows[i]]);
      }
      Tenant* tn = S->tenants[r.tenant].get();
      --tn->pending;
      if (r.keep) S->done[r.ticket] = out;
      ++S->completed;
    }
    ++S->steps;
    S->keys_done += st.keys;
  }
  S->cv_done.notify_all();
}

void worker_main(cs_server* S) {
  (void)hipSetDevice(S->device);
  std::deque<Step> inflight;  // launched, in order
  uint64_t index = 0;
  for (;;) {
    // retire finished steps without blocking
    while (!inflight.empty() && hipEventQuery(S->slots[inflight.front().slot].done) != hipErrorNotReady) {
      complete_step(S, inflight.front(), true);
      inflight.pop_front();
    }
    Step st;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->queue.empty()) {
        if (inflight.empty()) {
          if (S->stop) break;
          // A timed wait: waking a thread blocked without a timeout took
          // 2-4 ms here, which the first requests after an idle spell paid
          // in full (and the queue they built up made the next steps large).
          S->cv_work.wait_for(lk, std::chrono::microseconds(kIdlePollUs),
                              [&] { return S->stop || !S->queue.empty(); });
        } else {
          // a step is running: wake for a new arrival or to poll its event
          S->cv_work.wait_for(lk, std::chrono::microseconds(20), [&] { return !S->queue.empty(); });
        }
        continue;
      }
      if ((int)inflight.size() == kDepth) {
        lk.unlock();
        complete_step(S, inflight.front(), true);
        inflight.pop_front();
        continue;
      }
      // While the GPU is busy, let a second step grow to a worthwhile size; an
      // idle GPU takes whatever is queued at once.
      if (!inflight.empty() && !S->stop && S->queued_keys < S->step_keys / 4) {
        S->cv_work.wait_for(lk, std::chrono::microseconds(20),
                            [&] { return S->stop || S->queued_keys >= S->step_keys / 4; });
        continue;
      }
      form_step(S, st);
    }
    st.index = index++;
    st.slot = (int)(st.index % kDepth);
    launch_step(S, st);
    if (st.status != CS_OK) {
      // part of the step may be enqueued: let it finish before its slot is reused
      (void)hipStreamSynchronize(S->stream);
      complete_step(S, st, false);
      continue;
    }
    if (hipEventRecord(S->slots[st.slot].done, S->stream) != hipSuccess) {
      st.status = fail(CS_EDEVICE, "step event");
      (void)hipStreamSynchronize(S->stream);
      complete_step(S, st, false);
      continue;
    }
    inflight.push_back(std::move(st));
  }
}

// Queues one request (lock held).
cs_status submit_locked(cs_server* S, uint32_t tenant, uint32_t kind, const void* keys, const void* weights,
                        uint64_t n, uint64_t arrival_ns, bool keep, uint64_t* ticket) {
  if (kind == CS_REQ_UPDATE && n && (!keys || !weights)) return fail(CS_EINVAL, "keys or weights is NULL");
  if (S->stop) return fail(CS_EINVAL, "server is shutting down");
  if (tenant >= S->tenants.size() || !S->tenants[tenant] || S->tenants[tenant]->evicting)
    return fail(CS_EINVAL, "unknown tenant %u", tenant);
  const uint64_t t = S->next_ticket++;
  S->queue.push_back(Request{t, tenant, kind, keys, weights, n, arrival_ns, keep});
  if (kind == CS_REQ_UPDATE) S->queued_keys += n;
  ++S->tenants[tenant]->pending;
  ++S->submitted;
  if (keep) S->open.insert(t);
  if (ticket) *ticket = t;
  return CS_OK;
}

cs_status submit(cs_server* S, uint32_t tenant, uint32_t kind, const void* keys, const void* weights, uint64_t n,
                 uint64_t arrival_ns, bool keep, uint64_t* ticket) {
  cs_status st;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    st = submit_locked(S, tenant, kind, keys, weights, n, arrival_ns, keep, ticket);
  }
  if (st == CS_OK) S->cv_work.notify_one();
  return st;
}

}  // namespace

extern "C" cs_status cs_server_create(cs_prime prime, cs_mode mode, uint32_t k, cs_dtype key_type,
                                      cs_dtype weight_type, const cs_server_options* opts, cs_server** out) {
  if (!out) return fail(CS_EINVAL, "out is NULL");
  *out = nullptr;
  if (prime != CS_P61 && prime != CS_P89) return fail(CS_EINVAL, "sketches use CS_P61 or CS_P89");
  if (mode != CS_TWO_FOR_ONE && mode != CS_TWO_FOR_ONE_MSB && mode != CS_TWO_POLY && mode != CS_ARB_R)
    return fail(CS_EINVAL, "unknown mode %d", (int)mode);
  if (k != 2 && k != 4 && k != 8) return fail(CS_EINVAL, "k must be 2, 4 or 8");
  if (key_type != CS_U32 && key_type != CS_U64) return fail(CS_EINVAL, "key type must be CS_U32 or CS_U64");
  if (weight_type != CS_I32 && weight_type != CS_I64) return fail(CS_EINVAL, "weight type must be CS_I32 or CS_I64");
  auto S = std::make_unique<cs_server>();
  if (hipGetDevice(&S->device) != hipSuccess) return fail(CS_EDEVICE, "no current device");
  S->cprime = prime;
  S->cmode = mode;
  S->k = k;
  S->prime = prime == CS_P61 ? kPrime61 : kPrime89;
  S->mode = (int)mode;
  S->kb = key_type == CS_U32 ? 4 : 8;
  S->wb = weight_type == CS_I32 ? 4 : 8;
  S->budget = opts && opts->hbm_budget ? opts->hbm_budget : kDefaultBudget;
  S->step_keys = opts && opts->step_keys ? opts->step_keys : kDefaultStepKeys;
  S->work_bytes = opts && opts->work_bytes ? (size_t)opts->work_bytes : (size_t)kDefaultWork;
  S->direct_fraction = opts && opts->direct_fraction != 0.0 ? opts->direct_fraction : kServerDirect;
  if (S->work_bytes < (1u << 20)) return fail(CS_EINVAL, "work_bytes below 1 MiB");
  const uint64_t own = S->work_bytes + kDepth * (kListsInit + kResultWords * sizeof(int64_t));
  if (own > S->budget) return fail(CS_EBUSY, "step buffers (%llu bytes) exceed the budget", (unsigned long long)own);
  if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess)
    return fail(CS_EDEVICE, "stream creation");
  bool ok = hipMalloc(&S->d_work, S->work_bytes) == hipSuccess;
  for (Slot& sl : S->slots) {
    ok = ok && alloc_lists(sl, kListsInit);
    ok = ok && hipHostMalloc(&sl.h_results, kResultWords * sizeof(int64_t), hipHostMallocDefault) == hipSuccess;
    ok = ok && hipMalloc(&sl.d_results, kResultWords * sizeof(int64_t)) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
  }
  cs_server* raw = S.release();
  if (!ok) {
    cs_server_destroy(raw);
    return fail(CS_ENOMEM, "server buffers");
  }
  raw->resident = own;
  BatchLaunch prep{};
  prep.prime = raw->prime;
  prep.mode = raw->mode;
  prep.k = (int)k;
  prep.key_bytes = raw->kb;
  prep.weight_bytes = raw->wb;
  prep.prepare_only = true;
  hipError_t e = launch_batch(prep, 0);
  if (e != hipSuccess) {
    cs_server_destroy(raw);
    return hip_fail(e, "batch kernel attributes");
  }
  raw->worker = std::thread(worker_main, raw);
  *out = raw;
  return CS_OK;
}

extern "C" cs_status cs_server_admit(cs_server* S, uint32_t rows, uint64_t buckets, uint64_t seed, uint32_t* tenant) {
  if (!S || !tenant) return fail(CS_EINVAL, "server or tenant is NULL");
  if (rows < 1 || rows > 16) return fail(CS_EINVAL, "served sketches have 1..16 rows, got %u", rows);
  if (buckets < 2 || buckets > (1u << 18) || (S->cmode != CS_ARB_R && (buckets & (buckets - 1))))
    return fail(CS_EINVAL, "served sketches have up to 2^18 buckets, a power of two except in CS_ARB_R");
  uint32_t l = 0;
  while ((1ull << l) < buckets) ++l;
  const size_t bytes = sketch_device_bytes(rows, l, S->cmode, S->k);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->resident + bytes > S->budget)
      return fail(CS_EBUSY, "admitting %zu bytes would exceed the budget (%llu of %llu bytes held)", bytes,
                  (unsigned long long)S->resident, (unsigned long long)S->budget);
    S->resident += bytes;  // reserved while the sketch is created
  }
  cs_sketch* sk = nullptr;
  cs_status st;
  {
    DeviceGuard g(S->device);
    st = create_unreserved(rows, buckets, S->cprime, seed, S->cmode, S->k, &sk);
  }
  std::lock_guard<std::mutex> lk(S->mu);
  if (st != CS_OK) {
    S->resident -= bytes;
    return st;
  }
  auto t = std::make_unique<Tenant>();
  t->sk = sk;
  t->bytes = bytes;
  *tenant = (uint32_t)S->tenants.size();
  S->tenants.push_back(std::move(t));
  ++S->live_tenants;
  return CS_OK;
}

extern "C" cs_status cs_server_evict(cs_server* S, uint32_t tenant) {
  if (!S) return fail(CS_EINVAL, "server is NULL");
  cs_sketch* sk;
  size_t bytes;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    if (tenant >= S->tenants.size() || !S->tenants[tenant] || S->tenants[tenant]->evicting)
      return fail(CS_EINVAL, "unknown tenant %u", tenant);
    Tenant* t = S->tenants[tenant].get();
    t->evicting = true;
    S->cv_done.wait(lk, [&] { return t->pending == 0; });
    sk = t->sk;
    bytes = t->bytes;
  }
  {
    DeviceGuard g(S->device);
    cs_destroy(sk);
  }
  std::lock_guard<std::mutex> lk(S->mu);
  S->tenants[tenant].reset();
  S->resident -= bytes;
  --S->live_tenants;
  return CS_OK;
}

extern "C" cs_status cs_server_submit_update(cs_server* S, uint32_t tenant, const void* keys, const void* weights,
                                             uint64_t n, uint64_t* ticket) {
  if (!S) return fail(CS_EINVAL, "server is NULL");
  return submit(S, tenant, CS_REQ_UPDATE, keys, weights, n, now_ns(), ticket != nullptr, ticket);
}

extern "C" cs_status cs_server_submit_f2(cs_server* S, uint32_t tenant, uint64_t* ticket) {
  if (!S || !ticket) return fail(CS_EINVAL, "server or ticket is NULL");
  return submit(S, tenant, CS_REQ_F2, nullptr, nullptr, 0, now_ns(), true, ticket);
}

extern "C" cs_status cs_server_wait(cs_server* S, uint64_t ticket, cs_server_result* out) {
  if (!S || !out) return fail(CS_EINVAL, "server or out is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  if (!S->open.count(ticket)) return fail(CS_EINVAL, "ticket %llu is not waitable", (unsigned long long)ticket);
  S->cv_done.wait(lk, [&] { return S->done.count(ticket) != 0; });
  *out = S->done[ticket];
  S->done.erase(ticket);
  S->open.erase(ticket);
  return CS_OK;
}

extern "C" cs_status cs_server_drain(cs_server* S) {
  if (!S) return fail(CS_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  const uint64_t target = S->submitted;
  S->cv_done.wait(lk, [&] { return S->completed >= target; });
  return CS_OK;
}

extern "C" cs_status cs_server_read_counters(cs_server* S, uint32_t tenant, int64_t* host_dst) {
  if (!S || !host_dst) return fail(CS_EINVAL, "server or host_dst is NULL");
  cs_sketch* sk;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    if (tenant >= S->tenants.size() || !S->tenants[tenant] || S->tenants[tenant]->evicting)
      return fail(CS_EINVAL, "unknown tenant %u", tenant);
    Tenant* t = S->tenants[tenant].get();
    S->cv_done.wait(lk, [&] { return t->pending == 0; });
    sk = t->sk;
  }
  DeviceGuard g(S->device);
  return cs_read_counters(sk, host_dst, nullptr);
}

extern "C" cs_status cs_server_get_stats(cs_server* S, cs_server_stats* out) {
  if (!S || !out) return fail(CS_EINVAL, "server or out is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  out->steps = S->steps;
  out->requests = S->completed;
  out->keys = S->keys_done;
  out->resident_bytes = S->resident;
  out->budget_bytes = S->budget;
  out->tenants = S->live_tenants;
  return CS_OK;
}

extern "C" cs_status cs_server_replay(cs_server* S, const cs_server_request* reqs, uint32_t count,
                                      const double* arrival_s, cs_server_result* results) {
  if (!S || (count && (!reqs || !arrival_s || !results))) return fail(CS_EINVAL, "NULL argument");
  for (uint32_t i = 0; i < count; ++i) {
    if (reqs[i].kind != CS_REQ_UPDATE && reqs[i].kind != CS_REQ_F2)
      return fail(CS_EINVAL, "request %u has unknown kind %u", i, reqs[i].kind);
    if (!(arrival_s[i] >= 0.0) || (i && arrival_s[i] < arrival_s[i - 1]))
      return fail(CS_EINVAL, "arrival times must be non-negative and non-decreasing (request %u)", i);
  }
  std::vector<uint64_t> tickets(count, 0);
  std::vector<cs_status> sub(count, CS_OK);
  const int slack = prctl(PR_GET_TIMERSLACK, 0, 0, 0, 0);
  (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0, 0, 0);  // this thread's sleeps end within ~1 us
  // every request that is due goes into the queue under one lock acquisition
  const uint64_t t0 = now_ns();
  for (uint32_t i = 0; i < count;) {
    const uint64_t target = t0 + (uint64_t)(arrival_s[i] * 1e9);
    // Sleep until the arrival rather than spin: a thread that spins with yields
    // kept the CPU the worker woke on for milliseconds.  The timer slack is
    // cut to 1 us for the replay (see below), so a wake-up is a few us late.
    for (uint64_t t = now_ns(); t < target; t = now_ns())
      std::this_thread::sleep_for(std::chrono::nanoseconds(target - t));
    const uint64_t now = now_ns();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (; i < count; ++i) {
        const uint64_t due = t0 + (uint64_t)(arrival_s[i] * 1e9);
        if (due > now) break;
        const cs_server_request& r = reqs[i];
        sub[i] = submit_locked(S, r.tenant, r.kind, r.keys, r.weights, r.n, due, true, &tickets[i]);
      }
    }
    S->cv_work.notify_one();
  }
  if (slack > 0) (void)prctl(PR_SET_TIMERSLACK, (unsigned long)slack, 0, 0, 0);
  cs_status first = CS_OK;
  for (uint32_t i = 0; i < count; ++i) {
    if (sub[i] != CS_OK) {
      results[i] = cs_server_result{sub[i], 0, 0, 0, 0};
      if (first == CS_OK) first = sub[i];
      continue;
    }
    cs_status st = cs_server_wait(S, tickets[i], &results[i]);
    if (st != CS_OK && first == CS_OK) first = st;
  }
  return first;
}

extern "C" void cs_server_destroy(cs_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  DeviceGuard g(S->device);
  for (auto& t : S->tenants)
    if (t) cs_destroy(t->sk);
  if (S->stream) (void)hipStreamSynchronize(S->stream);
  for (Slot& sl : S->slots) {
    free_slot(sl);
    if (sl.h_results) (void)hipHostFree(sl.h_results);
    if (sl.d_results) (void)hipFree(sl.d_results);
    if (sl.done) (void)hipEventDestroy(sl.done);
  }
  if (S->d_work) (void)hipFree(S->d_work);
  if (S->stream) (void)hipStreamDestroy(S->stream);
  delete S;
}
