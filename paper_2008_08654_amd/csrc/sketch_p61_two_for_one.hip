// sketch_p61_two_for_one.hip -- Count Sketch kernels for p = 2^61 - 1, two-for-one split (low-bit layout).
#include "sketch_device.hpp"

namespace mcs {

template hipError_t launch_batch_pm<kPrime61, kTwoForOne>(const BatchLaunch&, hipStream_t);
template hipError_t launch_update_pm<kPrime61, kTwoForOne>(const UpdatePlan&, const UpdateArgsAny&, hipStream_t);
template hipError_t launch_query_pm<kPrime61, kTwoForOne>(const QueryArgsAny&, hipStream_t);

}  // namespace mcs
