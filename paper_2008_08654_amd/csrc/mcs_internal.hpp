// mcs_internal.hpp -- host-side internals shared by the C ABI implementation
// files (sketch object, device info, error helpers, launch planning).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "mcs.h"
#include "mcs_batch.h"
#include "sketch_kernels.hpp"

struct cs_sketch {
  uint32_t rows = 0;
  uint32_t log2m = 0;        // table row pitch is 2^log2m counters
  uint64_t buckets = 0;      // bucket count r (2^log2m except in CS_ARB_R)
  cs_prime prime = CS_P61;
  cs_mode mode = CS_TWO_FOR_ONE;
  uint32_t k = 4;
  int device = 0;
  std::vector<uint64_t> h_coeffs;  // p61: one word per coefficient; p89: two
  int64_t* d_table = nullptr;      // rows x 2^log2m, row-major
  uint64_t* d_coeffs = nullptr;    // uint4 records, [row][poly][i]
  uint32_t* d_flags = nullptr;     // sticky flags (kFlagDomain | kFlagOverflow)
  uint32_t* d_queues = nullptr;    // work queues of the row-resident update (kRowRanges * kMaxRows)
  void* d_est_part = nullptr;      // EstPartial[rows * est_slices]
  int64_t* d_est_out = nullptr;    // median, rows values, flags
  int64_t* h_est_out = nullptr;    // pinned copy of d_est_out
  uint32_t est_slices = 1;
  void* d_work = nullptr;          // workspace of the two-pass update (cs_reserve)
  size_t work_bytes = 0;
  int path = 0;                    // 0 auto, else forced cs_update path (CS_PATH_*)
  bool combine = true;             // two-pass update combines repeated keys of a tile
};

namespace mcs {

constexpr uint64_t kLdsTableMax = 64 * 1024;   // tables up to this size use the LDS single pass
constexpr uint64_t kLdsPerCu = 160 * 1024;
constexpr uint64_t kBinChunkKeys = 1ull << 27;  // keys per pass-1/pass-2 round of the binned update
constexpr uint64_t kMaxUpdateKeys = 1ull << 40;  // keys per cs_update call (tile counts fit 32 bits)
constexpr uint64_t kDefaultRoundKeys = 1ull << 20;  // two-pass round a new sketch reserves a workspace for

struct DeviceInfo {
  bool valid = false;
  int cus = 256;
  uint32_t lds_per_block = 65536;
};

const DeviceInfo& device_info(int dev);
cs_status fail(cs_status st, const char* fmt, ...);
// CS_OK, CS_ENOMEM for an out-of-memory error, else CS_EDEVICE.
cs_status status_of(hipError_t e);
// Sets the last-error message and returns status_of(e) (never CS_OK).
cs_status hip_fail(hipError_t e, const char* what);

// Rows per row group of the row-resident update: the largest divisor of rows
// whose 16-bit fields (rpg * 2^log2m * 2 bytes) fit a block's LDS; 0 when no
// row fits (more than 2^16 buckets).
uint32_t rows_per_group(uint32_t rows, uint32_t log2m);
UpdatePlan plan_update(const cs_sketch* s, uint64_t n);
// Enqueues the plan's launches; the two-pass path runs in rounds as large as
// `work` (work_bytes) holds.  Allocates nothing.
cs_status enqueue_update(cs_sketch* s, const UpdatePlan& plan, const void* keys, int kb, const void* weights, int wb,
                         uint64_t n, void* work, size_t work_bytes, hipStream_t stream);
// cs_create_ex without the default workspace (for sketches that cs_update
// never touches, such as the serving runtime's tenants).
cs_status create_unreserved(uint32_t rows, uint64_t buckets, cs_prime prime, uint64_t seed, cs_mode mode, uint32_t k,
                            cs_sketch** out);
// Status for device-reported flags (kFlagDomain takes precedence); sets the
// last-error message.
cs_status flags_status(uint32_t flags);
// Device bytes a sketch of this shape holds (table, coefficients, flags,
// estimate buffers), without the lazily allocated update workspace.
size_t sketch_device_bytes(uint32_t rows, uint32_t log2m, cs_mode mode, uint32_t k);

// ---------------------------------------------------------------------------
// Batched-update planning, shared by cs_batch and the serving runtime.
// batch_plan classifies the members and lays out the two-pass segments in
// rounds (each round's records and descriptors fit the workspace, rounds run
// one after another and reuse it); batch_emit then writes the device work
// lists for a list buffer at a given device address.
// ---------------------------------------------------------------------------
struct BatchPlanLimits {
  uint64_t round_keys = 1ull << 27;  // keys of two-pass segments per round
  size_t work_cap = ~(size_t)0;      // workspace bytes per round
  uint32_t cus = 256;                // compute units: row items are sized for this many blocks
};

struct BatchPlan {
  struct Seg {
    BatchSegment s;  // recs/desc filled by batch_emit
    uint32_t round;
    size_t rec_off, desc_off;
  };
  std::vector<BatchSketch> sks;
  std::vector<BatchLdsItem> lds_items, glb_items;
  std::vector<Seg> segs;  // in round order
  std::vector<BatchAccItem> acc_items;
  std::vector<BatchRowItem> row_items;  // row-resident and direct items, largest first
  uint32_t row_kpt = 8;
  std::vector<uint32_t> seg_first, acc_first;  // per round, plus one past the end
  std::vector<uint32_t> round_tiles;
  uint32_t max_table = 0, max_span = 0, max_wave_lds = 0;
  bool combine = true;
  uint32_t n_global = 0, n_lds = 0, n_rows = 0, n_twopass = 0;
  size_t work_bytes = 0;   // workspace the largest round needs
  size_t lists_bytes = 0;  // bytes of the device work lists
  size_t o_sk = 0, o_lds = 0, o_glb = 0, o_seg = 0, o_acc = 0, o_row = 0, o_queue = 0;
};

bool batch_twopass_shape(uint32_t rows, uint32_t log2m, uint32_t* log2g, uint32_t* log2r);
cs_status batch_plan(const cs_batch_item* items, size_t count, int kb, int wb, const cs_batch_options& opts,
                     const BatchPlanLimits& lim, BatchPlan* out);
// Fills host[0, plan.lists_bytes) with the lists as they must appear at device
// address d_lists, and the launch description (whose pointers refer to
// d_lists and d_work, except round_list, which points into *rounds).
void batch_emit(BatchPlan& plan, int prime, int mode, int k, int kb, int wb, const DeviceInfo& dev, char* d_lists,
                char* d_work, char* host, BatchLaunch* launch, std::vector<BatchRound>* rounds);

inline void release_workspace(cs_sketch* s) {
  if (s->d_work) (void)hipFree(s->d_work);
  s->d_work = nullptr;
  s->work_bytes = 0;
}

}  // namespace mcs
