// Spot kernels of the forward model for subaperture size 10 (wfs_forward_kernels.h).
#include "wfs_forward_kernels.h"

namespace wfs {
template hipError_t launch_fwd_ns<10>(const FwdParams&, hipStream_t);
}  // namespace wfs
