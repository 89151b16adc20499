// sketch_p61_two_poly.hip -- Count Sketch kernels for p = 2^61 - 1, two polynomials per row.
#include "sketch_device.hpp"

namespace mcs {

template hipError_t launch_batch_pm<kPrime61, kTwoPoly>(const BatchLaunch&, hipStream_t);
template hipError_t launch_update_pm<kPrime61, kTwoPoly>(const UpdatePlan&, const UpdateArgsAny&, hipStream_t);
template hipError_t launch_query_pm<kPrime61, kTwoPoly>(const QueryArgsAny&, hipStream_t);

}  // namespace mcs
