// FFT path of the Shack-Hartmann spot model (large subaperture fields, no elongation).
#pragma once

#include "wfs_otf.h"

namespace wfs {

inline bool fft_supported_impl(int n_sub, int n_fft, int bin) {
  (void)n_sub; (void)n_fft; (void)bin;
  return false;
}
inline int fft_lds_bytes_impl(int n_sub, int n_fft, int n_pix) {
  (void)n_sub; (void)n_fft; (void)n_pix;
  return 0;
}
__device__ __forceinline__ void fft_subap(const FwdParams& p, int task, int64_t step, char* smem) {
  (void)p; (void)task; (void)step; (void)smem;
}

}  // namespace wfs
