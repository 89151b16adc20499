// sketch_p89_msb.hip -- Count Sketch kernels for p = 2^89 - 1, two-for-one split of Algorithm 3 as printed.
#include "sketch_device.hpp"

namespace mcs {

template hipError_t launch_batch_pm<kPrime89, kTwoForOneMsb>(const BatchLaunch&, hipStream_t);
template hipError_t launch_update_pm<kPrime89, kTwoForOneMsb>(const UpdatePlan&, const UpdateArgsAny&, hipStream_t);
template hipError_t launch_query_pm<kPrime89, kTwoForOneMsb>(const QueryArgsAny&, hipStream_t);

}  // namespace mcs
