// Spot kernels of the forward model for subaperture size 11 (wfs_forward_kernels.h).
#include "wfs_forward_kernels.h"

namespace wfs {
template hipError_t launch_fwd_ns<11>(const FwdParams&, hipStream_t);
}  // namespace wfs
