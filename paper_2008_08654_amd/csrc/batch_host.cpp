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
  uint32_t n_global = 0, n_lds = 0, n_twopass = 0;
  bool planned = false;
  // graph
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

constexpr uint32_t kDefaultLdsMax = 65536;
constexpr uint32_t kMaxLdsTable = 160 * 1024;
constexpr uint32_t kDefaultChunk = 1u << 16;
constexpr uint64_t kRoundKeys = 1ull << 27;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

void drop_graph(cs_batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

void drop_plan(cs_batch* b) {
  drop_graph(b);
  if (b->d_lists) hipFree(b->d_lists);
  b->d_lists = nullptr;
  b->lists_bytes = 0;
  b->rounds.clear();
  b->planned = false;
}

// range width of the two-pass update (wave tiles: at most 16 ranges per row)
bool twopass_shape(const cs_sketch* s, uint32_t* log2g, uint32_t* log2r) {
  if (s->log2m > 18 || s->rows > 16) return false;
  uint32_t lr = s->log2m > 3 ? s->log2m - 3 : 0;
  lr = std::max(lr, kMinRangeLog2);
  lr = std::min(lr, kMaxRangeLog2);
  lr = std::min(lr, s->log2m);
  *log2r = lr;
  *log2g = s->log2m - lr;
  return (1u << *log2g) <= 16;
}

cs_status build_plan(cs_batch* b) {
  drop_plan(b);
  const DeviceInfo& dev = device_info(b->device);
  const uint32_t lds_max = b->opts.lds_table_max ? std::min(b->opts.lds_table_max, kMaxLdsTable) : kDefaultLdsMax;
  const uint64_t chunk = b->opts.lds_chunk_keys ? b->opts.lds_chunk_keys : kDefaultChunk;
  const bool combine = b->opts.combine >= 0;

  std::vector<BatchSketch> sks;
  std::vector<BatchLdsItem> lds_items, glb_items;
  struct Seg { BatchSegment s; uint32_t round; size_t rec_off, desc_off; };
  std::vector<Seg> segs;
  std::vector<size_t> round_bytes(1, 0);
  std::vector<uint64_t> round_keys(1, 0);
  std::vector<uint32_t> round_tiles(1, 0);
  uint32_t max_table = 0, max_span = 0, max_wave_lds = 0;
  b->n_global = b->n_lds = b->n_twopass = 0;

  for (const cs_batch_item& it : b->items) {
    if (it.n == 0) continue;
    cs_sketch* s = it.sketch;
    const uint64_t m = 1ull << s->log2m;
    const uint64_t cells = (uint64_t)s->rows << s->log2m;
    BatchSketch bs{it.keys, it.weights, it.n, (const uint4*)s->d_coeffs, (unsigned long long*)s->d_table,
                   s->d_flags, s->rows, s->log2m};
    if (it.n < m / 8) {  // a table flush would cost more than the direct atomics
      const uint32_t id = (uint32_t)sks.size();
      sks.push_back(bs);
      for (uint64_t o = 0; o < it.n; o += kDefaultChunk)
        glb_items.push_back(BatchLdsItem{id, 0, o, std::min(it.n, o + kDefaultChunk)});
      ++b->n_global;
    } else if (cells * 8 <= lds_max) {
      const uint32_t id = (uint32_t)sks.size();
      sks.push_back(bs);
      const uint64_t c = std::max<uint64_t>(chunk, 4 * cells);
      for (uint64_t o = 0; o < it.n; o += c) lds_items.push_back(BatchLdsItem{id, 0, o, std::min(it.n, o + c)});
      max_table = std::max<uint32_t>(max_table, (uint32_t)(cells * 8));
      ++b->n_lds;
    } else {
      uint32_t log2g, log2r;
      if (!twopass_shape(s, &log2g, &log2r))
        return fail(CS_EINVAL, "a member's table (rows %u, buckets 2^%u) is too large for the batched update",
                    s->rows, s->log2m);
      const uint32_t G = 1u << log2g;
      max_span = std::max<uint32_t>(max_span, 1u << log2r);
      max_wave_lds = std::max<uint32_t>(max_wave_lds, combine ? binw_lds_per_wave<true>(s->rows, G)
                                                              : binw_lds_per_wave<false>(s->rows, G));
      uint64_t off = 0;
      while (off < it.n) {
        uint32_t r = (uint32_t)round_keys.size() - 1;
        if (round_keys[r] >= kRoundKeys) {
          round_keys.push_back(0);
          round_bytes.push_back(0);
          round_tiles.push_back(0);
          ++r;
        }
        const uint64_t len = std::min(it.n - off, kRoundKeys - round_keys[r]);
        const uint32_t tiles = (uint32_t)((len + kWaveTile - 1) / kWaveTile);
        Seg sg{};
        sg.s = BatchSegment{(const char*)it.keys + off * b->kb, (const char*)it.weights + off * b->wb, len,
                            (const uint4*)s->d_coeffs, (unsigned long long*)s->d_table, s->d_flags, nullptr, nullptr,
                            s->rows, s->log2m, log2g, log2r, round_tiles[r], tiles};
        sg.round = r;
        sg.rec_off = round_bytes[r];
        round_bytes[r] = align256(round_bytes[r] + (size_t)tiles * s->rows * kWaveTile * 4);
        sg.desc_off = round_bytes[r];
        round_bytes[r] = align256(round_bytes[r] + (size_t)tiles * s->rows * (G + 1) * 4);
        round_keys[r] += len;
        round_tiles[r] += tiles;
        segs.push_back(sg);
        off += len;
      }
      ++b->n_twopass;
    }
  }

  // workspace: the largest round (rounds run one after another on the stream)
  size_t work = 0;
  for (size_t v : round_bytes) work = std::max(work, v);
  if (work > b->work_bytes) {
    if (b->d_work) hipFree(b->d_work);
    b->d_work = nullptr;
    b->work_bytes = 0;
    if (hipMalloc(&b->d_work, work) != hipSuccess) return fail(CS_ENOMEM, "batch workspace of %zu bytes", work);
    b->work_bytes = work;
  }
  // segments per round, in round order, with their pass-2 items
  std::vector<BatchSegment> seg_list;
  std::vector<BatchAccItem> acc_list;
  std::vector<uint32_t> seg_first(round_keys.size() + 1, 0), acc_first(round_keys.size() + 1, 0);
  for (uint32_t r = 0; r < round_keys.size(); ++r) {
    seg_first[r] = (uint32_t)seg_list.size();
    acc_first[r] = (uint32_t)acc_list.size();
    for (const Seg& sg : segs) {
      if (sg.round != r) continue;
      BatchSegment x = sg.s;
      x.recs = (uint32_t*)((char*)b->d_work + sg.rec_off);
      x.desc = (uint32_t*)((char*)b->d_work + sg.desc_off);
      const uint32_t local = (uint32_t)(seg_list.size() - seg_first[r]);
      seg_list.push_back(x);
      const uint64_t m = 1ull << x.log2m;
      const uint32_t parts = x.rows << x.log2g;
      const uint32_t slices = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(64, (uint64_t)x.tiles * 128 / m));
      for (uint32_t pt = 0; pt < parts; ++pt)
        for (uint32_t sl = 0; sl < slices; ++sl) acc_list.push_back(BatchAccItem{local, pt, sl, slices});
    }
  }
  seg_first[round_keys.size()] = (uint32_t)seg_list.size();
  acc_first[round_keys.size()] = (uint32_t)acc_list.size();

  // one device allocation for every list
  const size_t o_sk = 0;
  const size_t o_lds = align256(o_sk + sks.size() * sizeof(BatchSketch));
  const size_t o_glb = align256(o_lds + lds_items.size() * sizeof(BatchLdsItem));
  const size_t o_seg = align256(o_glb + glb_items.size() * sizeof(BatchLdsItem));
  const size_t o_acc = align256(o_seg + seg_list.size() * sizeof(BatchSegment));
  const size_t total = align256(o_acc + acc_list.size() * sizeof(BatchAccItem)) + 256;
  std::vector<char> host(total, 0);
  memcpy(host.data() + o_sk, sks.data(), sks.size() * sizeof(BatchSketch));
  memcpy(host.data() + o_lds, lds_items.data(), lds_items.size() * sizeof(BatchLdsItem));
  memcpy(host.data() + o_glb, glb_items.data(), glb_items.size() * sizeof(BatchLdsItem));
  memcpy(host.data() + o_seg, seg_list.data(), seg_list.size() * sizeof(BatchSegment));
  memcpy(host.data() + o_acc, acc_list.data(), acc_list.size() * sizeof(BatchAccItem));
  if (hipMalloc(&b->d_lists, total) != hipSuccess) return fail(CS_ENOMEM, "batch lists");
  b->lists_bytes = total;
  hipError_t e = hipMemcpy(b->d_lists, host.data(), total, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "batch lists upload");
  char* base = (char*)b->d_lists;
  for (uint32_t r = 0; r < round_keys.size(); ++r) {
    if (seg_first[r + 1] == seg_first[r]) continue;
    BatchRound rd{};
    rd.segs = (const BatchSegment*)(base + o_seg) + seg_first[r];
    rd.nsegs = seg_first[r + 1] - seg_first[r];
    rd.total_tiles = round_tiles[r];
    rd.acc_items = (const BatchAccItem*)(base + o_acc) + acc_first[r];
    rd.nacc = acc_first[r + 1] - acc_first[r];
    b->rounds.push_back(rd);
  }
  BatchLaunch& L = b->launch;
  L = BatchLaunch{};
  L.prime = b->prime;
  L.mode = b->mode;
  L.k = b->k;
  L.key_bytes = b->kb;
  L.weight_bytes = b->wb;
  L.dedup = combine;
  L.sketches = (const BatchSketch*)(base + o_sk);
  L.lds_item_list = (const BatchLdsItem*)(base + o_lds);
  L.lds_items = (uint32_t)lds_items.size();
  L.lds_bytes = std::max<uint32_t>(max_table, 8);
  const uint32_t lds_per_cu = std::max<uint32_t>(1, std::min<uint32_t>(8, kMaxLdsTable / L.lds_bytes));
  L.lds_blocks = std::max<uint32_t>(1, std::min<uint32_t>(L.lds_items, dev.cus * lds_per_cu));
  L.glb_item_list = (const BatchLdsItem*)(base + o_glb);
  L.glb_items = (uint32_t)glb_items.size();
  L.glb_blocks = std::max<uint32_t>(1, std::min<uint32_t>(L.glb_items, dev.cus * 8));
  L.round_list = b->rounds.data();
  L.rounds = (uint32_t)b->rounds.size();
  L.bin_lds_per_wave = std::max<uint32_t>(max_wave_lds, 16);
  L.bin_lds_bytes = (kBlock / 64) * L.bin_lds_per_wave;
  L.bin_blocks = dev.cus * 8;
  L.acc_lds_bytes = std::max<uint32_t>(max_span, 1) * 8;
  L.acc_blocks = dev.cus * std::max<uint32_t>(1, std::min<uint32_t>(2, kMaxLdsTable / L.acc_lds_bytes));
  BatchLaunch prep = L;
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
      if (g) hipGraphDestroy(g);
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

extern "C" cs_status cs_batch_classes(const cs_batch* b, uint32_t* n_global, uint32_t* n_lds, uint32_t* n_twopass) {
  if (!b) return fail(CS_EINVAL, "batch is NULL");
  if (n_global) *n_global = b->n_global;
  if (n_lds) *n_lds = b->n_lds;
  if (n_twopass) *n_twopass = b->n_twopass;
  return CS_OK;
}

extern "C" cs_status cs_batch_autotune(cs_batch* b, hipStream_t stream, cs_batch_options* chosen) {
  if (!b) return fail(CS_EINVAL, "batch is NULL");
  const cs_batch_options keep = b->opts;
  std::vector<cs_batch_options> cands;
  for (uint32_t lm : {40960u, 65536u, 163840u})
    for (uint32_t ch : {1u << 15, 1u << 17})
      for (int cb : {1, -1}) cands.push_back(cs_batch_options{lm, ch, cb, keep.use_graph});
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(CS_EDEVICE, "event creation");
  float best = 1e30f;
  cs_batch_options best_opts = keep;
  cs_status status = CS_OK;
  for (const cs_batch_options& c : cands) {
    b->opts = c;
    status = build_plan(b);
    if (status != CS_OK) break;
    status = run_plan(b, stream, false);  // warm-up
    if (status != CS_OK) break;
    hipEventRecord(e0, stream);
    status = run_plan(b, stream, false);
    if (status != CS_OK) break;
    hipEventRecord(e1, stream);
    if (hipEventSynchronize(e1) != hipSuccess) {
      status = fail(CS_EDEVICE, "autotune timing");
      break;
    }
    float ms = 0;
    hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) {
      best = ms;
      best_opts = c;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  b->opts = status == CS_OK ? best_opts : keep;
  cs_status st2 = build_plan(b);
  if (status == CS_OK) status = st2;
  // the trial runs added into the tables: zero them
  for (const cs_batch_item& it : b->items) {
    if (cs_reset(it.sketch, stream) != CS_OK && status == CS_OK) status = CS_EDEVICE;
  }
  if (hipStreamSynchronize(stream) != hipSuccess && status == CS_OK) status = fail(CS_EDEVICE, "autotune sync");
  if (chosen) *chosen = b->opts;
  return status;
}

extern "C" void cs_batch_destroy(cs_batch* b) {
  if (!b) return;
  hipDeviceSynchronize();
  drop_plan(b);
  if (b->d_work) hipFree(b->d_work);
  if (b->cap_stream) hipStreamDestroy(b->cap_stream);
  delete b;
}
