// sketch_p89_two_poly.hip -- Count Sketch kernels for p = 2^89 - 1, two polynomials per row.
#include "sketch_device.hpp"

namespace mcs {

template hipError_t launch_batch_pm<kPrime89, kTwoPoly>(const BatchLaunch&, hipStream_t);
template hipError_t launch_update_pm<kPrime89, kTwoPoly>(const UpdatePlan&, const UpdateArgsAny&, hipStream_t);
template hipError_t launch_query_pm<kPrime89, kTwoPoly>(const QueryArgsAny&, hipStream_t);

}  // namespace mcs
