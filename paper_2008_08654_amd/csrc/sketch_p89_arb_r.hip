// sketch_p89_arb_r.hip -- Count Sketch kernels for p = 2^89 - 1, any bucket count (Algorithm 8).
#include "sketch_device.hpp"

namespace mcs {

template hipError_t launch_batch_pm<kPrime89, kArbR>(const BatchLaunch&, hipStream_t);
template hipError_t launch_update_pm<kPrime89, kArbR>(const UpdatePlan&, const UpdateArgsAny&, hipStream_t);
template hipError_t launch_query_pm<kPrime89, kArbR>(const QueryArgsAny&, hipStream_t);

}  // namespace mcs
