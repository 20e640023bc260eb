// Spot kernels of the forward model for subaperture sizes 2 to 6 (wfs_forward_kernels.h).
#include "wfs_forward_kernels.h"

namespace wfs {
template hipError_t launch_fwd_ns<2>(const FwdParams&, hipStream_t);
template hipError_t launch_fwd_ns<3>(const FwdParams&, hipStream_t);
template hipError_t launch_fwd_ns<4>(const FwdParams&, hipStream_t);
template hipError_t launch_fwd_ns<5>(const FwdParams&, hipStream_t);
template hipError_t launch_fwd_ns<6>(const FwdParams&, hipStream_t);
}  // namespace wfs
