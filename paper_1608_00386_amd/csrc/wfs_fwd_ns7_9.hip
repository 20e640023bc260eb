// Spot kernels of the forward model for subaperture sizes 7 to 9 (wfs_forward_kernels.h).
#include "wfs_forward_kernels.h"

namespace wfs {
template hipError_t launch_fwd_ns<7>(const FwdParams&, hipStream_t);
template hipError_t launch_fwd_ns<8>(const FwdParams&, hipStream_t);
template hipError_t launch_fwd_ns<9>(const FwdParams&, hipStream_t);
}  // namespace wfs
