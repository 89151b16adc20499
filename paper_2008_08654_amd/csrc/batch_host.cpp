// batch_host.cpp -- host side of include/mcs_batch.h: classifies each member
// sketch (direct atomics / LDS / two-pass), builds the device work lists and
// the two-pass workspace, captures the launches in a HIP graph, and tunes the
// thresholds on the real batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "mcs.h"
#include "mcs_batch.h"
#include "mcs_internal.hpp"
#include "sketch_kernels.hpp"

using namespace mcs;

struct cs_batch {
  std::vector<cs_batch_item> items;
  int kb = 8, wb = 8;
  int prime = kPrime61, mode = 0, k = 4;
  int device = 0;
  cs_batch_options opts{};
  // plan
  void* d_lists = nullptr;
  size_t lists_bytes = 0;
  void* d_work = nullptr;
  size_t work_bytes = 0;
  std::vector<BatchRound> rounds;
  BatchLaunch launch{};
  uint32_t n_global = 0, n_lds = 0, n_rows = 0, n_twopass = 0;
  bool planned = false;
  // graph
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// ---------------------------------------------------------------------------
// planning (shared with the serving runtime)
// ---------------------------------------------------------------------------
namespace {
constexpr uint32_t kDefaultLdsMax = 65536;
constexpr uint32_t kMaxLdsTable = 160 * 1024;
constexpr uint32_t kDefaultChunk = 1u << 16;
constexpr uint32_t kGlobalChunk = kBlock * kKeysPerThread;  // one pass of a block: spreads short streams over CUs
constexpr double kDefaultDirect = 0.125;
constexpr uint32_t kBatchRangeLog2 = 13;
size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
}  // namespace

// Range width of the two-pass update in a batch: 2^13 counters (a 64 KiB
// pass-2 table, two 16-wave blocks per CU; 2^14 halves that occupancy and
// measured 11% slower on the 4096-sketch batch), wider only where a row would
// otherwise need more than the 16 ranges wave tiles take.
bool mcs::batch_twopass_shape(uint32_t rows, uint32_t log2m, uint32_t* log2g, uint32_t* log2r) {
  if (log2m > 18 || rows > 16) return false;
  const uint32_t lr = std::min(log2m, std::max(kBatchRangeLog2, log2m > 4 ? log2m - 4 : 0u));
  *log2r = lr;
  *log2g = log2m - lr;
  return (1u << *log2g) <= 16;
}

cs_status mcs::batch_plan(const cs_batch_item* items, size_t count, int kb, int wb, const cs_batch_options& opts,
                          const BatchPlanLimits& lim, BatchPlan* out) {
  BatchPlan& P = *out;
  P = BatchPlan{};
  const bool rows_on = opts.row_resident >= 0;
  // with the row-resident class on, no table goes to the LDS class unless asked
  const uint32_t lds_max = opts.lds_table_max ? std::min(opts.lds_table_max, kMaxLdsTable)
                           : rows_on          ? 8u
                                              : kDefaultLdsMax;
  const uint64_t chunk = opts.lds_chunk_keys ? opts.lds_chunk_keys : kDefaultChunk;
  P.combine = opts.combine >= 0;
  const double direct = opts.direct_fraction == 0.0 ? kDefaultDirect : opts.direct_fraction;
  if (opts.keys_per_thread != 0 && opts.keys_per_thread != 2 && opts.keys_per_thread != 4 &&
      opts.keys_per_thread != 8)
    return fail(CS_EINVAL, "keys_per_thread must be 0, 2, 4 or 8");
  P.row_kpt = opts.keys_per_thread ? (int)opts.keys_per_thread : 8;
  struct RowMember {
    uint32_t id, rpg, rows, log2m;
    uint64_t n;
  };
  std::vector<RowMember> row_members;
  std::vector<uint64_t> round_keys(1, 0);
  std::vector<size_t> round_bytes(1, 0);
  P.round_tiles.assign(1, 0);

  for (size_t idx = 0; idx < count; ++idx) {
    const cs_batch_item& it = items[idx];
    if (it.n == 0) continue;
    cs_sketch* s = it.sketch;
    const uint64_t m = 1ull << s->log2m;
    const uint64_t cells = (uint64_t)s->rows << s->log2m;
    BatchSketch bs{it.keys, it.weights, it.n, (const uint4*)s->d_coeffs, (unsigned long long*)s->d_table,
                   s->d_flags, s->rows, s->log2m};
    const uint32_t rpg = rows_on ? rows_per_group(s->rows, s->log2m) : 0;
    if (direct > 0.0 && (double)it.n < direct * (double)m) {  // fewer updates than a flush would touch
      const uint32_t id = (uint32_t)P.sks.size();
      P.sks.push_back(bs);
      if (rows_on) {
        row_members.push_back(RowMember{id, 0, s->rows, s->log2m, it.n});
      } else {
        for (uint64_t o = 0; o < it.n; o += kGlobalChunk)
          P.glb_items.push_back(BatchLdsItem{id, 0, o, std::min(it.n, o + kGlobalChunk)});
      }
      ++P.n_global;
    } else if (cells * 8 <= lds_max) {
      const uint32_t id = (uint32_t)P.sks.size();
      P.sks.push_back(bs);
      const uint64_t c = std::max<uint64_t>(chunk, 4 * cells);
      for (uint64_t o = 0; o < it.n; o += c) P.lds_items.push_back(BatchLdsItem{id, 0, o, std::min(it.n, o + c)});
      P.max_table = std::max<uint32_t>(P.max_table, (uint32_t)(cells * 8));
      ++P.n_lds;
    } else if (rpg) {
      const uint32_t id = (uint32_t)P.sks.size();
      P.sks.push_back(bs);
      row_members.push_back(RowMember{id, rpg, s->rows, s->log2m, it.n});
      ++P.n_rows;
    } else {
      uint32_t log2g, log2r;
      if (!batch_twopass_shape(s->rows, s->log2m, &log2g, &log2r))
        return fail(CS_EINVAL, "a member's table (rows %u, buckets 2^%u) is too large for the batched update",
                    s->rows, s->log2m);
      const uint32_t G = 1u << log2g;
      P.max_span = std::max<uint32_t>(P.max_span, 1u << log2r);
      P.max_wave_lds = std::max<uint32_t>(P.max_wave_lds, P.combine ? binw_lds_per_wave<true>(s->rows, G)
                                                                    : binw_lds_per_wave<false>(s->rows, G));
      // records and descriptors of one tile (plus up to 512 bytes of alignment per segment)
      const size_t tile_bytes = (size_t)s->rows * kWaveTile * 4 + (size_t)s->rows * (G + 1) * 4;
      if (lim.work_cap < tile_bytes + 512)
        return fail(CS_EINVAL, "workspace of %zu bytes holds no tile of a member with %u rows", lim.work_cap, s->rows);
      uint64_t off = 0;
      while (off < it.n) {
        uint32_t r = (uint32_t)round_keys.size() - 1;
        uint64_t fit_tiles = round_bytes[r] + tile_bytes + 512 <= lim.work_cap
                                 ? (lim.work_cap - round_bytes[r] - 512) / tile_bytes
                                 : 0;
        if (round_keys[r] >= lim.round_keys || fit_tiles == 0) {
          round_keys.push_back(0);
          round_bytes.push_back(0);
          P.round_tiles.push_back(0);
          ++r;
          fit_tiles = (lim.work_cap - 512) / tile_bytes;
        }
        const uint64_t len = std::min({it.n - off, lim.round_keys - round_keys[r], fit_tiles * kWaveTile});
        const uint32_t tiles = (uint32_t)((len + kWaveTile - 1) / kWaveTile);
        BatchPlan::Seg sg{};
        sg.s = BatchSegment{(const char*)it.keys + off * kb, (const char*)it.weights + off * wb, len,
                            (const uint4*)s->d_coeffs, (unsigned long long*)s->d_table, s->d_flags, nullptr, nullptr,
                            s->rows, s->log2m, log2g, log2r, P.round_tiles[r], tiles};
        sg.round = r;
        sg.rec_off = round_bytes[r];
        round_bytes[r] = align256(round_bytes[r] + (size_t)tiles * s->rows * kWaveTile * 4);
        sg.desc_off = round_bytes[r];
        round_bytes[r] = align256(round_bytes[r] + (size_t)tiles * s->rows * (G + 1) * 4);
        round_keys[r] += len;
        P.round_tiles[r] += tiles;
        P.segs.push_back(sg);
        off += len;
      }
      ++P.n_twopass;
    }
  }
  // Row items: each row group (or, for a direct member, the whole sketch) over
  // ranges of wave tiles, cut so that no item holds more than about 1/6 of a
  // CU's share of the batch's key-rows, then ordered largest first so that
  // the persistent blocks finish together.
  if (!row_members.empty()) {
    const uint64_t wt_keys = 64ull * (uint64_t)P.row_kpt;
    uint64_t total = 0;
    for (const RowMember& r : row_members) total += r.n * r.rows;
    const uint64_t target = std::max<uint64_t>(1ull << 18, total / ((uint64_t)lim.cus * 6));
    struct Costed {
      uint64_t cost;
      BatchRowItem item;
    };
    std::vector<Costed> all;
    for (const RowMember& r : row_members) {
      const uint64_t tiles = (r.n + wt_keys - 1) / wt_keys;
      const uint32_t per = r.rpg ? r.rpg : r.rows;     // rows an item adds a key to
      const uint64_t groups = r.rpg ? r.rows / r.rpg : 1;
      const uint64_t per_tile = wt_keys * per * (r.rpg ? 1 : 2);  // direct atomics cost about twice a field add
      // at most one piece per 16 wave tiles (a tile per wave) and, for a rows
      // item, per 2m keys (its flush then costs at most about half its adds)
      const uint64_t most = std::min<uint64_t>((tiles + 15) / 16, r.rpg ? r.n / (2ull << r.log2m) : ~0ull);
      const uint64_t pieces =
          std::max<uint64_t>(1, std::min<uint64_t>(most, (tiles * per_tile + target - 1) / target));
      const uint64_t fields = r.rpg ? ((uint64_t)r.rpg << r.log2m) / 4 : 0;  // clearing and flushing the fields
      for (uint64_t g = 0; g < groups; ++g)
        for (uint64_t pc = 0; pc < pieces; ++pc) {
          const uint64_t b = tiles * pc / pieces, e = tiles * (pc + 1) / pieces;
          const uint32_t spread = (uint32_t)(pc & 0xFFFF) | (uint32_t)std::min<uint64_t>(pieces, 0xFFFF) << 16;
          all.push_back(Costed{(e - b) * per_tile + fields,
                               BatchRowItem{r.id, (uint32_t)(g * r.rpg), r.rpg, spread, b, e}});
        }
    }
    std::stable_sort(all.begin(), all.end(), [](const Costed& a, const Costed& b) { return a.cost > b.cost; });
    P.row_items.reserve(all.size());
    for (const Costed& c : all) P.row_items.push_back(c.item);
  }
  for (size_t v : round_bytes) P.work_bytes = std::max(P.work_bytes, v);
  // segments are appended round by round, so each round's are contiguous
  const uint32_t nr = (uint32_t)round_keys.size();
  P.seg_first.assign(nr + 1, 0);
  P.acc_first.assign(nr + 1, 0);
  uint32_t si = 0;
  for (uint32_t r = 0; r < nr; ++r) {
    P.seg_first[r] = si;
    P.acc_first[r] = (uint32_t)P.acc_items.size();
    for (; si < P.segs.size() && P.segs[si].round == r; ++si) {
      const BatchSegment& x = P.segs[si].s;
      const uint64_t m = 1ull << x.log2m;
      const uint32_t parts = x.rows << x.log2g;
      const uint32_t slices = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(64, (uint64_t)x.tiles * 128 / m));
      const uint32_t local = si - P.seg_first[r];
      for (uint32_t pt = 0; pt < parts; ++pt)
        for (uint32_t sl = 0; sl < slices; ++sl) P.acc_items.push_back(BatchAccItem{local, pt, sl, slices});
    }
  }
  P.seg_first[nr] = si;
  P.acc_first[nr] = (uint32_t)P.acc_items.size();
  P.o_sk = 0;
  P.o_lds = align256(P.o_sk + P.sks.size() * sizeof(BatchSketch));
  P.o_glb = align256(P.o_lds + P.lds_items.size() * sizeof(BatchLdsItem));
  P.o_seg = align256(P.o_glb + P.glb_items.size() * sizeof(BatchLdsItem));
  P.o_acc = align256(P.o_seg + P.segs.size() * sizeof(BatchSegment));
  P.o_row = align256(P.o_acc + P.acc_items.size() * sizeof(BatchAccItem));
  P.o_queue = align256(P.o_row + P.row_items.size() * sizeof(BatchRowItem));
  P.lists_bytes = P.o_queue + 256;
  return CS_OK;
}

void mcs::batch_emit(BatchPlan& P, int prime, int mode, int k, int kb, int wb, const DeviceInfo& dev, char* d_lists,
                     char* d_work, char* host, BatchLaunch* launch, std::vector<BatchRound>* rounds) {
  memset(host, 0, P.lists_bytes);
  memcpy(host + P.o_sk, P.sks.data(), P.sks.size() * sizeof(BatchSketch));
  memcpy(host + P.o_lds, P.lds_items.data(), P.lds_items.size() * sizeof(BatchLdsItem));
  memcpy(host + P.o_glb, P.glb_items.data(), P.glb_items.size() * sizeof(BatchLdsItem));
  BatchSegment* segs = (BatchSegment*)(host + P.o_seg);
  for (size_t i = 0; i < P.segs.size(); ++i) {
    segs[i] = P.segs[i].s;
    segs[i].recs = (uint32_t*)(d_work + P.segs[i].rec_off);
    segs[i].desc = (uint32_t*)(d_work + P.segs[i].desc_off);
  }
  memcpy(host + P.o_acc, P.acc_items.data(), P.acc_items.size() * sizeof(BatchAccItem));
  memcpy(host + P.o_row, P.row_items.data(), P.row_items.size() * sizeof(BatchRowItem));
  rounds->clear();
  for (uint32_t r = 0; r + 1 < P.seg_first.size(); ++r) {
    if (P.seg_first[r + 1] == P.seg_first[r]) continue;
    BatchRound rd{};
    rd.segs = (const BatchSegment*)(d_lists + P.o_seg) + P.seg_first[r];
    rd.nsegs = P.seg_first[r + 1] - P.seg_first[r];
    rd.total_tiles = P.round_tiles[r];
    rd.acc_items = (const BatchAccItem*)(d_lists + P.o_acc) + P.acc_first[r];
    rd.nacc = P.acc_first[r + 1] - P.acc_first[r];
    rounds->push_back(rd);
  }
  const uint32_t acc_lds = std::max<uint32_t>(P.max_span, 1) * 8;
  const uint32_t acc_max = dev.cus * std::max<uint32_t>(1, std::min<uint32_t>(2, kMaxLdsTable / acc_lds));
  for (BatchRound& rd : *rounds) {
    rd.bin_blocks = std::max<uint32_t>(1, std::min<uint32_t>(dev.cus * 8, (rd.total_tiles + 3) / 4));
    rd.acc_blocks = std::max<uint32_t>(1, std::min<uint32_t>(acc_max, rd.nacc));
  }
  BatchLaunch& L = *launch;
  L = BatchLaunch{};
  L.prime = prime;
  L.mode = mode;
  L.k = k;
  L.key_bytes = kb;
  L.weight_bytes = wb;
  L.dedup = P.combine;
  L.sketches = (const BatchSketch*)(d_lists + P.o_sk);
  L.lds_item_list = (const BatchLdsItem*)(d_lists + P.o_lds);
  L.lds_items = (uint32_t)P.lds_items.size();
  L.lds_bytes = std::max<uint32_t>(P.max_table, 8);
  const uint32_t lds_per_cu = std::max<uint32_t>(1, std::min<uint32_t>(8, kMaxLdsTable / L.lds_bytes));
  L.lds_blocks = std::max<uint32_t>(1, std::min<uint32_t>(L.lds_items, dev.cus * lds_per_cu));
  L.glb_item_list = (const BatchLdsItem*)(d_lists + P.o_glb);
  L.glb_items = (uint32_t)P.glb_items.size();
  L.glb_blocks = std::max<uint32_t>(1, std::min<uint32_t>(L.glb_items, dev.cus * 8));
  L.round_list = rounds->data();
  L.rounds = (uint32_t)rounds->size();
  L.bin_lds_per_wave = std::max<uint32_t>(P.max_wave_lds, 16);
  L.bin_lds_bytes = (kBlock / 64) * L.bin_lds_per_wave;
  L.bin_blocks = dev.cus * 8;
  L.acc_lds_bytes = acc_lds;
  L.acc_blocks = acc_max;
  L.row_item_list = (const BatchRowItem*)(d_lists + P.o_row);
  L.row_items = (uint32_t)P.row_items.size();
  L.row_blocks = std::max<uint32_t>(1, std::min<uint32_t>(L.row_items, dev.cus));
  L.row_queue = (uint32_t*)(d_lists + P.o_queue);
  L.row_kpt = P.row_kpt;
}

namespace {

void drop_graph(cs_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

void drop_plan(cs_batch* b) {
  drop_graph(b);
  if (b->d_lists) (void)hipFree(b->d_lists);
  b->d_lists = nullptr;
  b->lists_bytes = 0;
  b->rounds.clear();
  b->planned = false;
}

cs_status build_plan(cs_batch* b) {
  drop_plan(b);
  const DeviceInfo& dev = device_info(b->device);
  BatchPlan P;
  BatchPlanLimits lim;
  lim.cus = (uint32_t)dev.cus;
  cs_status st = batch_plan(b->items.data(), b->items.size(), b->kb, b->wb, b->opts, lim, &P);
  if (st != CS_OK) return st;
  b->n_global = P.n_global;
  b->n_lds = P.n_lds;
  b->n_rows = P.n_rows;
  b->n_twopass = P.n_twopass;
  if (P.work_bytes > b->work_bytes) {
    if (b->d_work) (void)hipFree(b->d_work);
    b->d_work = nullptr;
    b->work_bytes = 0;
    if (hipMalloc(&b->d_work, P.work_bytes) != hipSuccess)
      return fail(CS_ENOMEM, "batch workspace of %zu bytes", P.work_bytes);
    b->work_bytes = P.work_bytes;
  }
  if (hipMalloc(&b->d_lists, P.lists_bytes) != hipSuccess) return fail(CS_ENOMEM, "batch lists");
  b->lists_bytes = P.lists_bytes;
  std::vector<char> host(P.lists_bytes, 0);
  batch_emit(P, b->prime, b->mode, b->k, b->kb, b->wb, dev, (char*)b->d_lists, (char*)b->d_work, host.data(),
             &b->launch, &b->rounds);
  hipError_t e = hipMemcpy(b->d_lists, host.data(), P.lists_bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "batch lists upload");
  BatchLaunch prep = b->launch;
  prep.prepare_only = true;
  e = launch_batch(prep, 0);
  if (e != hipSuccess) return hip_fail(e, "batch kernel attributes");
  b->planned = true;
  return CS_OK;
}

cs_status run_plan(cs_batch* b, hipStream_t stream, bool graph) {
  if (!graph) {
    hipError_t e = launch_batch(b->launch, stream);
    return e == hipSuccess ? CS_OK : hip_fail(e, "batch launch");
  }
  if (!b->exec) {
    hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "graph capture begin");
    e = launch_batch(b->launch, b->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(e != hipSuccess ? e : e2, "graph capture");
    }
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      drop_graph(b);
      return hip_fail(e, "graph instantiate");
    }
  }
  hipError_t e = hipGraphLaunch(b->exec, stream);
  return e == hipSuccess ? CS_OK : hip_fail(e, "graph launch");
}

}  // namespace

extern "C" cs_status cs_batch_create(const cs_batch_item* items, uint32_t count, cs_dtype key_type,
                                     cs_dtype weight_type, const cs_batch_options* opts, cs_batch** out) {
  if (!out) return fail(CS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!items || count == 0) return fail(CS_EINVAL, "empty batch");
  if (key_type != CS_U32 && key_type != CS_U64) return fail(CS_EINVAL, "key type must be CS_U32 or CS_U64");
  if (weight_type != CS_I32 && weight_type != CS_I64) return fail(CS_EINVAL, "weight type must be CS_I32 or CS_I64");
  const cs_sketch* s0 = items[0].sketch;
  for (uint32_t i = 0; i < count; ++i) {
    const cs_batch_item& it = items[i];
    if (!it.sketch) return fail(CS_EINVAL, "item %u has no sketch", i);
    if (it.n && (!it.keys || !it.weights)) return fail(CS_EINVAL, "item %u has NULL keys or weights", i);
    if (it.sketch->device != s0->device || it.sketch->prime != s0->prime || it.sketch->mode != s0->mode ||
        it.sketch->k != s0->k)
      return fail(CS_EINVAL, "item %u differs in device, prime, mode or k", i);
  }
  auto* b = new (std::nothrow) cs_batch();
  if (!b) return fail(CS_ENOMEM, "host allocation");
  b->items.assign(items, items + count);
  b->kb = key_type == CS_U32 ? 4 : 8;
  b->wb = weight_type == CS_I32 ? 4 : 8;
  b->prime = s0->prime == CS_P61 ? kPrime61 : kPrime89;
  b->mode = (int)s0->mode;
  b->k = (int)s0->k;
  b->device = s0->device;
  if (opts) b->opts = *opts;
  if (hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return fail(CS_EDEVICE, "capture stream");
  }
  cs_status st = build_plan(b);
  if (st != CS_OK) {
    cs_batch_destroy(b);
    return st;
  }
  *out = b;
  return CS_OK;
}

extern "C" cs_status cs_batch_update(cs_batch* b, hipStream_t stream) {
  if (!b) return fail(CS_EINVAL, "batch is NULL");
  if (!b->planned) {
    cs_status st = build_plan(b);
    if (st != CS_OK) return st;
  }
  return run_plan(b, stream, b->opts.use_graph >= 0);
}

extern "C" cs_status cs_batch_get_options(const cs_batch* b, cs_batch_options* out) {
  if (!b || !out) return fail(CS_EINVAL, "batch or out is NULL");
  *out = b->opts;
  return CS_OK;
}

extern "C" cs_status cs_batch_classes(const cs_batch* b, uint32_t* n_global, uint32_t* n_lds, uint32_t* n_rows,
                                      uint32_t* n_twopass) {
  if (!b) return fail(CS_EINVAL, "batch is NULL");
  if (n_global) *n_global = b->n_global;
  if (n_lds) *n_lds = b->n_lds;
  if (n_rows) *n_rows = b->n_rows;
  if (n_twopass) *n_twopass = b->n_twopass;
  return CS_OK;
}

namespace {

// A copy of every member's counters and flags in one device buffer, so that
// tuning trials leave the sketches as they were.
struct SavedTables {
  char* buf = nullptr;
  std::vector<std::pair<cs_sketch*, size_t>> at;  // sketch, offset of its table copy
};

size_t table_bytes(const cs_sketch* s) { return ((size_t)s->rows << s->log2m) * sizeof(int64_t); }

cs_status save_tables(const cs_batch* b, hipStream_t stream, SavedTables* sv) {
  std::vector<cs_sketch*> sks;
  for (const cs_batch_item& it : b->items) sks.push_back(it.sketch);
  std::sort(sks.begin(), sks.end());
  sks.erase(std::unique(sks.begin(), sks.end()), sks.end());
  size_t bytes = 0;
  for (cs_sketch* s : sks) {
    sv->at.emplace_back(s, bytes);
    bytes = align256(bytes + table_bytes(s) + sizeof(uint32_t));
  }
  hipError_t e = hipMalloc(&sv->buf, std::max<size_t>(bytes, 256));
  if (e != hipSuccess) {
    sv->buf = nullptr;
    (void)hipGetLastError();
    return fail(status_of(e), "autotune: %zu bytes of device memory to keep the members' counters", bytes);
  }
  for (const auto& [s, off] : sv->at) {
    e = hipMemcpyAsync(sv->buf + off, s->d_table, table_bytes(s), hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(sv->buf + off + table_bytes(s), s->d_flags, sizeof(uint32_t), hipMemcpyDeviceToDevice,
                         stream);
    if (e != hipSuccess) return hip_fail(e, "autotune: copying the members' counters");
  }
  return CS_OK;
}

cs_status restore_tables(SavedTables* sv, hipStream_t stream) {
  cs_status st = CS_OK;
  if (!sv->buf) return st;
  for (const auto& [s, off] : sv->at) {
    hipError_t e = hipMemcpyAsync(s->d_table, sv->buf + off, table_bytes(s), hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->d_flags, sv->buf + off + table_bytes(s), sizeof(uint32_t), hipMemcpyDeviceToDevice,
                         stream);
    if (e != hipSuccess) {
      st = hip_fail(e, "autotune: restoring the members' counters");
      break;
    }
  }
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess && st == CS_OK) st = hip_fail(e, "autotune: restoring the members' counters");
  (void)hipFree(sv->buf);
  sv->buf = nullptr;
  return st;
}

}  // namespace

extern "C" cs_status cs_batch_autotune(cs_batch* b, hipStream_t stream, cs_batch_options* chosen) {
  if (!b) return fail(CS_EINVAL, "batch is NULL");
  const cs_batch_options keep = b->opts;
  SavedTables saved;
  cs_status status = save_tables(b, stream, &saved);
  if (status != CS_OK) {
    (void)restore_tables(&saved, stream);
    return status;
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) {
    status = fail(CS_EDEVICE, "event creation");
  }
  // median of three timed updates after one warm-up
  auto measure = [&](const cs_batch_options& c, float* ms) -> cs_status {
    b->opts = c;
    cs_status st = build_plan(b);
    if (st == CS_OK) st = run_plan(b, stream, false);
    float t[3] = {0, 0, 0};
    for (int i = 0; i < 3 && st == CS_OK; ++i) {
      if (hipEventRecord(ev[0], stream) != hipSuccess) st = fail(CS_EDEVICE, "autotune timing");
      if (st == CS_OK) st = run_plan(b, stream, false);
      if (st == CS_OK && (hipEventRecord(ev[1], stream) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
                          hipEventElapsedTime(&t[i], ev[0], ev[1]) != hipSuccess))
        st = fail(CS_EDEVICE, "autotune timing");
    }
    std::sort(t, t + 3);
    *ms = t[1];
    return st;
  };
  float best = 1e30f;
  cs_batch_options best_opts = keep;
  auto consider = [&](const cs_batch_options& c) {
    if (status != CS_OK) return;
    float ms = 0;
    status = measure(c, &ms);
    if (status == CS_OK && ms < best) {
      best = ms;
      best_opts = c;
    }
  };
  // the class limits, every combination
  for (int rr : {1, -1})
    for (uint32_t lm : {8u, 20480u, 40960u, 65536u, 163840u})
      for (double df : {1.0 / 128, 0.125, 1.0}) {
        cs_batch_options c{};
        c.lds_table_max = lm;
        c.use_graph = keep.use_graph;
        c.direct_fraction = df;
        c.row_resident = rr;
        consider(c);
      }
  // then one knob at a time from the best so far
  for (uint32_t kpt : {2u, 4u, 8u}) {
    cs_batch_options c = best_opts;
    c.keys_per_thread = kpt;
    consider(c);
  }
  for (uint32_t ch : {1u << 15, 1u << 17}) {
    cs_batch_options c = best_opts;
    c.lds_chunk_keys = ch;
    consider(c);
  }
  for (int cb : {1, -1}) {
    cs_batch_options c = best_opts;
    c.combine = cb;
    consider(c);
  }
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  b->opts = status == CS_OK ? best_opts : keep;
  cs_status st2 = build_plan(b);
  if (status == CS_OK) status = st2;
  // the trials added into the tables: put back what they held
  st2 = restore_tables(&saved, stream);
  if (status == CS_OK) status = st2;
  if (chosen) *chosen = b->opts;
  return status;
}

extern "C" void cs_batch_destroy(cs_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  drop_plan(b);
  if (b->d_work) (void)hipFree(b->d_work);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
}
