// sketch_p61_arb_r.hip -- Count Sketch kernels for p = 2^61 - 1, any bucket count (Algorithm 8).
#include "sketch_device.hpp"

namespace mcs {

template hipError_t launch_batch_pm<kPrime61, kArbR>(const BatchLaunch&, hipStream_t);
template hipError_t launch_update_pm<kPrime61, kArbR>(const UpdatePlan&, const UpdateArgsAny&, hipStream_t);
template hipError_t launch_query_pm<kPrime61, kArbR>(const QueryArgsAny&, hipStream_t);

}  // namespace mcs
