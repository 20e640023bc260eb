// Interaction-matrix calibration (Sec. 2.5 of the paper).
//
// Calibration registers the slopes of one actuator poke at a time through the sensor model.
// Here a batch of 2h realisations carries h pokes at +amplitude followed by the same h pokes
// at -amplitude (push-pull), so one batched forward call measures h columns; a second kernel
// forms each column as the central difference (s+ - s-) / (2 amplitude).  The control matrix
// built from it (Sec. 2.6) is set-up work in a library of its own (tlse.hip).
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace wfs {

constexpr int kCalBlock = 256;

// Realisation r < h holds actuator act0 + r at +amp, realisation h + r the same actuator at
// -amp (r < n_chunk; the rest hold no poke), on top of `base` (one realisation) or zero.
__global__ __launch_bounds__(kCalBlock) void calib_poke_kernel(float* __restrict__ layers,
                                                               const float* __restrict__ base,
                                                               int64_t stride, int32_t h,
                                                               int64_t act0, int32_t n_chunk,
                                                               float amp) {
  const int64_t total = 2 * (int64_t)h * stride;
  for (int64_t i = (int64_t)blockIdx.x * kCalBlock + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kCalBlock) {
    const int64_t r = i / stride, e = i - r * stride;
    const int64_t j = r < h ? r : r - h;
    float v = base ? base[e] : 0.0f;
    if (j < n_chunk && e == act0 + j) v += r < h ? amp : -amp;
    layers[i] = v;
  }
}

// Row j of the interaction matrix (slopes of actuator j): (s[j] - s[h + j]) / (2 amp).
__global__ __launch_bounds__(kCalBlock) void calib_diff_kernel(const float* __restrict__ s,
                                                               int32_t h, int32_t n_slopes,
                                                               float two_amp,
                                                               float* __restrict__ im,
                                                               int64_t ld_im) {
  const int32_t j = blockIdx.y;
  const float* sp = s + (int64_t)j * n_slopes;
  const float* sm = s + (int64_t)(h + j) * n_slopes;
  float* d = im + (int64_t)j * ld_im;
  for (int32_t k = blockIdx.x * kCalBlock + threadIdx.x; k < n_slopes;
       k += gridDim.x * kCalBlock)
    d[k] = (sp[k] - sm[k]) / two_amp;
}

hipError_t calib_poke(float* layers, const float* base, int64_t stride, int32_t h, int64_t act0,
                      int32_t n_chunk, float amp, hipStream_t st) {
  const int64_t total = 2 * (int64_t)h * stride;
  const int64_t blocks = (total + kCalBlock - 1) / kCalBlock;
  const int grid = (int)(blocks < 65536 ? blocks : 65536);
  calib_poke_kernel<<<grid, kCalBlock, 0, st>>>(layers, base, stride, h, act0, n_chunk, amp);
  return hipGetLastError();
}

hipError_t calib_diff(const float* slopes, int32_t h, int32_t n_slopes, int32_t n_chunk,
                      float amp, float* im, int64_t ld_im, hipStream_t st) {
  const int gx = (n_slopes + kCalBlock - 1) / kCalBlock;
  calib_diff_kernel<<<dim3(gx < 64 ? gx : 64, n_chunk), kCalBlock, 0, st>>>(
      slopes, h, n_slopes, 2.0f * amp, im, ld_im);
  return hipGetLastError();
}

}  // namespace wfs
