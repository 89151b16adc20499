// sketch_kernels.hpp -- launch interface between the host library and the
// Count Sketch / quotient-remainder kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "field.hpp"

namespace mcs {

constexpr int kPrime61 = 1;
constexpr int kPrime89 = 2;
constexpr int kPrime64c = 3;
constexpr int kTwoForOne = 0;
constexpr int kTwoForOneMsb = 1;
constexpr int kTwoPoly = 2;
constexpr int kArbR = 3;  // any number of buckets (Algorithm 8)

constexpr int kBlock = 256;          // 4 wave64s
constexpr int kKeysPerThread = 4;    // keys held in registers per thread per tile
constexpr uint32_t kMaxRows = 64;    // rows per sketch
constexpr uint32_t kMaxQueryRows = 64;
constexpr uint32_t kMaxLog2m = 30;

// sticky device flags
constexpr uint32_t kFlagDomain = 1u;
constexpr uint32_t kFlagOverflow = 2u;

constexpr int kVariantLds = 0;
constexpr int kVariantGlobal = 1;
constexpr int kVariantBinned = 2;
constexpr int kVariantRows = 3;

// row-resident update (tables of up to 2^16 buckets per row)
constexpr int kRowBlock = 1024;                     // 16 wave64s, one block per CU
constexpr int kRowKpt = 8;                          // keys per thread per tile
constexpr uint32_t kRowTile = kRowBlock * kRowKpt;  // keys per tile
constexpr uint32_t kRowMaxLog2m = 16;               // a row of 16-bit fields fits LDS
constexpr uint32_t kRowLdsBytes = 160 * 1024;       // LDS a block may hold
constexpr uint32_t kRowChunk = 32;                  // wave tiles a wave takes from a queue at once
constexpr uint32_t kRowXcds = 8;                    // XCDs of the GPU: key ranges and queues per row group
constexpr uint32_t kRowRanges = kRowXcds + 1;       // the XCDs' key ranges and one pool range

// two-pass (binned) update
constexpr int kBinKpt = 8;                          // keys per thread in a pass-1 tile
constexpr uint32_t kBinTile = kBlock * kBinKpt;     // keys per tile (block tiles)
constexpr uint32_t kProbeTiles = 64;               // 512-key windows sampled by the combining probe
constexpr uint32_t kWaveTile = 512;                 // keys per tile (wave tiles, <= 16 ranges per row)
constexpr uint32_t kMinRangeLog2 = 11;              // counters per partition: 2^11 .. 2^14 (int64 LDS in pass 2)
constexpr uint32_t kMaxRangeLog2 = 14;
constexpr int kAccBlock = 1024;                     // pass-2 block (16 wave64s)
constexpr uint32_t kMaxLog2g = 10;                  // at most 1024 ranges per row

struct UpdatePlan {
  int variant;
  uint32_t blocks;
  uint32_t lds_bytes;
  // binned variant
  uint32_t log2g;       // log2 of bucket ranges per row
  uint32_t log2r;       // log2 of buckets per range
  uint32_t tiles;       // tiles in this launch
  uint32_t acc_slices;  // pass-2 items per partition
  uint32_t acc_blocks;  // pass-2 persistent blocks
  uint32_t acc_lds_bytes;
  bool dedup;           // combine repeated keys of a tile before hashing
  bool combine_auto;    // probe the keys, then launch both pass-1 variants (dedup ignored)
  uint32_t lds_bytes_plain;  // pass-1 LDS of the variant without combining (combine_auto)
  uint32_t* probe;           // kProbeTiles * 2 words of device memory (combine_auto)
  bool wave_tiles;      // pass 1 with one tile per wave (k_bin_wave)
  uint32_t* recs;       // [tiles][rows][kBinTile]
  uint32_t* desc;       // [tiles][rows][G + 1]
  // row-resident variant
  uint32_t rpg;         // rows per row group (a divisor of rows)
  uint32_t range_blocks;  // per XCD, blocks that work on the XCD's range (a multiple of the groups; 0: all)
  uint32_t* queues;     // kRowRanges * kMaxRows work-queue counters (the sketch's)
};

// Row-resident update: block b holds the 16-bit fields of row group b mod
// groups (rpg rows of 2^log2m buckets); its waves take wave tiles from the
// queues of that group, their own XCD's key range first.
template <typename KeyT, typename WT>
struct RowArgs {
  const KeyT* keys;
  const WT* weights;
  uint64_t n;
  const uint4* coeffs;
  uint32_t rows;
  uint32_t log2m;
  uint32_t rpg;
  uint32_t groups;
  uint32_t tiles;
  unsigned long long* table;
  uint32_t* flags;
  uint32_t* queues;  // (xcds + 1) * groups counters, zero at launch
  uint32_t xcds;
  uint32_t range_blocks;  // see k_update_rows (0 in the batched kernel)
};

template <typename KeyT, typename WT>
struct UpdateArgs {
  const KeyT* keys;
  const WT* weights;
  uint64_t n;
  uint64_t keys_per_block;
  const uint4* coeffs;
  uint32_t rows;
  uint32_t log2m;
  unsigned long long* table;
  uint32_t* flags;
};

struct UpdateArgsAny {
  int prime, mode, k;
  int key_bytes, weight_bytes;
  const void* keys;
  const void* weights;
  uint64_t n;
  uint64_t keys_per_block;
  const uint4* coeffs;
  uint32_t rows;
  uint32_t log2m;
  unsigned long long* table;
  uint32_t* flags;
  template <typename KeyT, typename WT>
  UpdateArgs<KeyT, WT> as() const {
    return UpdateArgs<KeyT, WT>{(const KeyT*)keys, (const WT*)weights, n, keys_per_block, coeffs, rows, log2m,
                                table, flags};
  }
};

template <typename KeyT, typename WT>
struct BinArgs {
  const KeyT* keys;
  const WT* weights;
  uint64_t n;
  const uint4* coeffs;
  uint32_t rows;
  uint32_t log2m;
  uint32_t log2g;
  uint32_t log2r;
  uint32_t tiles;
  uint32_t* recs;
  uint32_t* desc;
  unsigned long long* table;
  uint32_t* flags;
  // When probe is set, the launch runs only if its combining choice is the
  // probe's (combine_pays); the other variant is launched beside it.
  const uint32_t* probe;
  uint32_t probe_tiles;
  uint32_t probe_permille;
};

struct AccArgs {
  const uint32_t* recs;
  const uint32_t* desc;
  uint32_t tiles;
  uint32_t rows;
  uint32_t log2m;
  uint32_t log2g;
  uint32_t log2r;
  uint32_t slices;
  uint32_t tile_keys;
  unsigned long long* table;
};

template <typename KeyT>
struct QueryArgs {
  const KeyT* keys;
  uint64_t n;
  const uint4* coeffs;
  uint32_t rows;
  uint32_t log2m;
  const int64_t* table;
  int64_t* out;
  uint32_t* flags;
};

struct QueryArgsAny {
  int prime, mode, k, key_bytes;
  const void* keys;
  uint64_t n;
  const uint4* coeffs;
  uint32_t rows;
  uint32_t log2m;
  const int64_t* table;
  int64_t* out;
  uint32_t* flags;
  template <typename KeyT>
  QueryArgs<KeyT> as() const {
    return QueryArgs<KeyT>{(const KeyT*)keys, n, coeffs, rows, log2m, table, out, flags};
  }
};

struct EstPartial {
  unsigned long long lo, hi;
  uint32_t big, pad;
};

// Group bounds of the two-pass workspace, range-major: bound g (0..G) of row
// `row` of tile `tile` sits at desc[(row * (G + 1) + g) * tiles + tile], so a
// pass-2 item (row, range) reads the bounds of consecutive tiles contiguously.
__host__ __device__ inline size_t desc_index(uint32_t row, uint32_t g, uint32_t G, uint32_t tiles, uint32_t tile) {
  return ((size_t)row * (G + 1) + g) * tiles + tile;
}

hipError_t launch_update(const UpdatePlan& plan, const UpdateArgsAny& a, hipStream_t st);

// one F2 estimate of a batch: partial-kernel blocks [first_block, first_block +
// rows * slices), results (median, rows values, flags) at out[out_offset...]
struct BatchEstItem {
  const int64_t* table;
  EstPartial* part;  // rows * slices partial sums (the sketch's own buffer)
  const uint32_t* flags;
  uint32_t rows, log2m, slices, first_block;
  uint64_t out_offset;
};
hipError_t launch_batch_estimate(const BatchEstItem* items, uint32_t nitems, uint32_t total_blocks, int64_t* out,
                                 uint32_t cus, hipStream_t st);

// ---------------------------------------------------------------------------
// batched update
// ---------------------------------------------------------------------------
struct BatchSketch {          // a sketch whose table fits LDS
  const void* keys;
  const void* weights;
  uint64_t n;
  const uint4* coeffs;
  unsigned long long* table;
  uint32_t* flags;
  uint32_t rows, log2m;
};
struct BatchLdsItem {         // keys [begin, end) of sketch `sketch`
  uint32_t sketch, pad;
  uint64_t begin, end;
};
struct BatchRowItem {         // batched row-resident update (k_batch_rows)
  uint32_t sketch;            // index into the sketch list
  uint32_t r0;                // first row of the item's row group
  uint32_t rpg;               // rows of the group; 0: every row, direct device atomics
  uint32_t spread;            // piece index | pieces << 16 (16 bits each): staggers the pieces' flushes
  uint64_t wt_begin, wt_end;  // wave tiles [wt_begin, wt_end) of the sketch's stream
};
struct BatchSegment {         // keys of one two-pass sketch handled in a round
  const void* keys;           // first key of the segment
  const void* weights;
  uint64_t n;
  const uint4* coeffs;
  unsigned long long* table;
  uint32_t* flags;
  uint32_t* recs;             // segment's records: [tiles][rows][kWaveTile]
  uint32_t* desc;             // segment's group offsets: [tiles][rows][G + 1]
  uint32_t rows, log2m, log2g, log2r;
  uint32_t tile_begin, tiles; // wave tiles [tile_begin, tile_begin + tiles) of the round
};
struct BatchAccItem {
  uint32_t segment, part, slice, slices;
};
struct BatchRound {           // host-side description of one pass-1/pass-2 round
  const BatchSegment* segs;
  uint32_t nsegs;
  uint32_t total_tiles;
  const BatchAccItem* acc_items;
  uint32_t nacc;
  uint32_t bin_blocks, acc_blocks;  // grids of the round (grid-stride kernels)
};
struct BatchLaunch {
  int prime, mode, k, key_bytes, weight_bytes;
  bool dedup;
  bool prepare_only;  // only set kernel attributes
  const BatchSketch* sketches;
  const BatchLdsItem* lds_item_list;
  uint32_t lds_items, lds_blocks, lds_bytes;
  const BatchLdsItem* glb_item_list;  // items of sketches updated with direct atomics
  uint32_t glb_items, glb_blocks;
  const BatchRowItem* row_item_list;  // row-resident and direct items, largest first
  uint32_t row_items, row_blocks;
  uint32_t* row_queue;                // the row items' queue counter (8 bytes, zeroed per launch)
  int row_kpt;                        // keys per lane of a wave tile of the row items: 4 or 8
  const BatchRound* round_list;  // host array
  uint32_t rounds;
  uint32_t bin_blocks, bin_lds_bytes, bin_lds_per_wave;
  uint32_t acc_blocks, acc_lds_bytes;
};
hipError_t launch_batch(const BatchLaunch& b, hipStream_t st);

// Calls set() once per device (thread-safe; two threads may both call it, which
// is harmless for idempotent attribute settings): a kernel attribute such as the
// dynamic-LDS limit above 64 KiB must be in place before the first launch.
template <typename F>
inline hipError_t once_per_device(std::atomic<uint64_t>& done, F set) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const uint64_t bit = 1ull << (dev & 63);
  if (done.load(std::memory_order_acquire) & bit) return hipSuccess;
  e = set();
  if (e == hipSuccess) done.fetch_or(bit, std::memory_order_acq_rel);
  return e;
}

// Launchers per (prime, mode), one pair instantiated per translation unit;
// launch_update / launch_query / launch_batch dispatch to them.
template <int PRIME, int MODE>
hipError_t launch_batch_pm(const BatchLaunch& b, hipStream_t st);
template <int PRIME, int MODE>
hipError_t launch_update_pm(const UpdatePlan& plan, const UpdateArgsAny& a, hipStream_t st);
template <int PRIME, int MODE>
hipError_t launch_query_pm(const QueryArgsAny& a, hipStream_t st);
// pass-2 launches and LDS attributes shared by every instantiation
hipError_t launch_accumulate(const AccArgs& c, uint32_t blocks, uint32_t lds_bytes, hipStream_t st);
hipError_t launch_batch_acc(const BatchRound& rd, uint32_t lds_bytes, hipStream_t st);
hipError_t set_accumulate_attribute();
hipError_t set_batch_acc_attribute();

// LDS bytes of one wave of the wave-tile pass 1:
//   [combining: keys u64[T] | weights i64[T]] | slots u32[2T] (records are
//   staged there) | ticket counters u32[rows*4G] (two per range, then the
//   spare ones), padded to 16 bytes.
// Each wave's region starts at wave * this stride, so the stride must keep the
// 8-byte key/weight arrays (64-bit LDS atomics need natural alignment) and the
// 16-byte staged copies aligned for every wave, whatever rows * G is.
template <bool DEDUP>
__host__ __device__ constexpr uint32_t binw_lds_per_wave(uint32_t rows, uint32_t G) {
  return (DEDUP ? kWaveTile * 16 : 0) + 2 * kWaveTile * 4 + ((rows * 4 * G * 4 + 15u) & ~15u);
}

// LDS bytes of the pass-1 kernel besides the per-row counters
template <bool DEDUP>
constexpr uint32_t bin_lds_fixed_bytes() {
  return (DEDUP ? (kBinTile * 8 + kBinTile * 8 + 2 * kBinTile * 4) : 0) + kBinTile * 4;
}
hipError_t launch_query(const QueryArgsAny& a, hipStream_t st);
hipError_t launch_estimate(const int64_t* table, uint32_t rows, uint32_t log2m, uint32_t slices, EstPartial* part,
                           int64_t* out, uint32_t* flags, hipStream_t st);
hipError_t launch_add_tables(unsigned long long* dst, const unsigned long long* src, uint64_t n, hipStream_t st);
hipError_t launch_fill_zero(unsigned long long* dst, uint64_t n, hipStream_t st);

// quotient / remainder
hipError_t launch_wide_divmod(uint32_t b, uint32_t c, uint32_t m, int method, const uint32_t* x, uint64_t n,
                              uint32_t* quot, uint32_t* rem, hipStream_t st);
hipError_t launch_bucket_map(int prime, bool fast, const uint64_t* v, uint64_t n, uint32_t r, uint32_t* out,
                             uint32_t* flags, uint32_t cus, hipStream_t st);
hipError_t launch_divmod(int prime, bool naive, const uint64_t* x, uint64_t n, uint64_t* quot, uint64_t* rem,
                         uint32_t* flags, hipStream_t st);

}  // namespace mcs
