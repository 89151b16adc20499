// mcs_internal.hpp -- host-side internals shared by the C ABI implementation
// files (sketch object, device info, error helpers, launch planning).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "mcs.h"
#include "sketch_kernels.hpp"

struct cs_sketch {
  uint32_t rows = 0;
  uint32_t log2m = 0;
  cs_prime prime = CS_P61;
  cs_mode mode = CS_TWO_FOR_ONE;
  uint32_t k = 4;
  int device = 0;
  std::vector<uint64_t> h_coeffs;  // p61: one word per coefficient; p89: two
  int64_t* d_table = nullptr;      // rows x 2^log2m, row-major
  uint64_t* d_coeffs = nullptr;    // uint4 records, [row][poly][i]
  uint32_t* d_flags = nullptr;     // sticky flags (kFlagDomain | kFlagOverflow)
  void* d_est_part = nullptr;      // EstPartial[rows * est_slices]
  int64_t* d_est_out = nullptr;    // median, rows values, flags
  int64_t* h_est_out = nullptr;    // pinned copy of d_est_out
  uint32_t est_slices = 1;
  void* d_work = nullptr;          // workspace of the two-pass update (bins)
  size_t work_bytes = 0;
  int path = 0;                    // 0 auto, else forced cs_update path (CS_PATH_*)
  bool combine = true;             // two-pass update combines repeated keys of a tile
};

namespace mcs {

constexpr uint64_t kLdsTableMax = 64 * 1024;   // tables up to this size use the LDS single pass
constexpr uint64_t kLdsPerCu = 160 * 1024;
constexpr uint64_t kBinChunkKeys = 1ull << 27;  // keys per pass-1/pass-2 round of the binned update

struct DeviceInfo {
  bool valid = false;
  int cus = 256;
  uint32_t lds_per_block = 65536;
};

const DeviceInfo& device_info(int dev);
cs_status fail(cs_status st, const char* fmt, ...);
cs_status hip_fail(hipError_t e, const char* what);

UpdatePlan plan_update(const cs_sketch* s, uint64_t n);
cs_status enqueue_update(cs_sketch* s, const UpdatePlan& plan, const void* keys, int kb, const void* weights, int wb,
                         uint64_t n, hipStream_t stream);
inline void release_workspace(cs_sketch* s) {
  if (s->d_work) hipFree(s->d_work);
  s->d_work = nullptr;
  s->work_bytes = 0;
}

}  // namespace mcs
