// Spot kernels of the forward model for subaperture size 12 (wfs_forward_kernels.h).
#include "wfs_forward_kernels.h"

namespace wfs {
template hipError_t launch_fwd_ns<12>(const FwdParams&, hipStream_t);
}  // namespace wfs
