// update_noalloc.cpp -- cs_update_noalloc (include/mcs_noalloc.h): the same
// update as cs_update, with the two-pass workspace taken from a fixed device
// array of the library instead of the sketch's, so that no call allocates.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "mcs.h"
#include "mcs_noalloc.h"
#include "mcs_internal.hpp"

using namespace mcs;

constexpr size_t kScratchBytes = (size_t)CS_NOALLOC_SCRATCH_BYTES;

// One copy per device, held from the library's load until the process ends.
// Host code never uses this name as an address: it is a host-side stand-in;
// the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of `scratch` on device `dev` (which must be current), looked
// up once per device.
void* scratch_address(int dev) {
  static std::mutex mu;
  static std::vector<void*> addr;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    addr[dev] = p;
  }
  return addr[dev];
}

}  // namespace

extern "C" cs_status cs_update_noalloc(cs_sketch* s, const void* keys, cs_dtype key_type, const void* weights,
                                       cs_dtype weight_type, uint64_t n, hipStream_t stream) {
  if (!s) return fail(CS_EINVAL, "sketch is NULL");
  if (key_type != CS_U32 && key_type != CS_U64) return fail(CS_EINVAL, "key type must be CS_U32 or CS_U64");
  if (weight_type != CS_I32 && weight_type != CS_I64) return fail(CS_EINVAL, "weight type must be CS_I32 or CS_I64");
  if (n == 0) return CS_OK;
  if (!keys || !weights) return fail(CS_EINVAL, "keys or weights is NULL");
  if (n > kMaxUpdateKeys) return fail(CS_EINVAL, "at most 2^40 keys per call");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != s->device) return fail(CS_EINVAL, "the sketch lives on device %d, device %d is current", s->device, dev);
  const UpdatePlan plan = plan_update(s, n);
  void* work = nullptr;
  if (plan.variant == kVariantBinned) {
    // one round of one tile must fit the array; larger inputs run in more rounds
    const uint64_t tk = plan.wave_tiles ? kWaveTile : kBinTile;
    const size_t one_tile = (size_t)s->rows * (tk + (1u << plan.log2g) + 1) * 4 + 2 * kProbeTiles * sizeof(uint32_t);
    if (one_tile > kScratchBytes)
      return fail(CS_EINVAL, "a round of this sketch needs %zu bytes, more than the %zu-byte scratch array", one_tile,
                  kScratchBytes);
    work = scratch_address(dev);
    if (!work) return fail(CS_EDEVICE, "scratch array address lookup failed");
  }
  return enqueue_update(s, plan, keys, key_type == CS_U32 ? 4 : 8, weights, weight_type == CS_I32 ? 4 : 8, n, work,
                        work ? kScratchBytes : 0, stream);
}
