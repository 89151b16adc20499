// sketch_p89_two_for_one.hip -- Count Sketch kernels for p = 2^89 - 1, two-for-one split (low-bit layout).
#include "sketch_device.hpp"

namespace mcs {

template hipError_t launch_batch_pm<kPrime89, kTwoForOne>(const BatchLaunch&, hipStream_t);
template hipError_t launch_update_pm<kPrime89, kTwoForOne>(const UpdatePlan&, const UpdateArgsAny&, hipStream_t);
template hipError_t launch_query_pm<kPrime89, kTwoForOne>(const QueryArgsAny&, hipStream_t);

}  // namespace mcs
