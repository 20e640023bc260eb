// Interaction-matrix calibration and the regularised least-squares control matrix
// (Sec. 2.5 and Sec. 2.6 of the paper).
//
// Calibration registers the slopes of one actuator poke at a time through the sensor model.
// Here a batch of 2h realisations carries h pokes at +amplitude followed by the same h pokes
// at -amplitude (push-pull), so one batched forward call measures h columns; a second kernel
// forms each column as the central difference (s+ - s-) / (2 amplitude).
//
// The control matrix is the least-squares estimator with a diagonal (per-actuator weighted)
// Tikhonov term, R = (D^T D + eps mean(diag D^T D) W)^(-1) D^T for the interaction matrix D,
// built once from library dense linear algebra (rocBLAS syrk and trsm, rocSOLVER Cholesky):
// it is set-up work, outside the per-frame path.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <stdint.h>
#include <stdio.h>

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

// G[j][j] += eps * mean(diag G) * w[j] (w = 1 when null): one workgroup, a fixed-order sum.
__global__ __launch_bounds__(1024) void tlse_regularise_kernel(float* __restrict__ G, int32_t m,
                                                               float eps,
                                                               const float* __restrict__ w) {
  __shared__ double part[1024];
  double acc = 0.0;
  for (int32_t j = threadIdx.x; j < m; j += 1024) acc += G[(int64_t)j * m + j];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  const float lam = (float)((double)eps * part[0] / (double)m);
  for (int32_t j = threadIdx.x; j < m; j += 1024)
    G[(int64_t)j * m + j] += lam * (w ? w[j] : 1.0f);
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

static const char* rb_msg(rocblas_status s, const char* what) {
  static thread_local char buf[160];
  snprintf(buf, sizeof buf, "%s: %s", what, rocblas_status_to_string(s));
  return buf;
}

// R (n_s x m column-major, ld_r) = D (D^T D + lambda W)^(-1) for D = im (n_s x m column-major,
// ld_im), i.e. row-major R[m][n_s] = (D^T D + lambda W)^(-1) D^T.  work: m*m floats (the
// Gram matrix, then its Cholesky factor) followed by one int.  Returns null on success, else a
// message; *info receives rocSOLVER's potrf info (0, or the order of the first non-positive
// leading minor).  Synchronises the stream.
const char* tlse_run(const float* im, int32_t m, int32_t n_s, int64_t ld_im, float eps,
                     const float* w, float* R, int64_t ld_r, float* work, hipStream_t st,
                     int* info) {
  rocblas_handle h = nullptr;
  const char* err = nullptr;
  rocblas_status s = rocblas_create_handle(&h);
  if (s != rocblas_status_success) return rb_msg(s, "rocblas_create_handle");
  float* G = work;
  rocblas_int* d_info = reinterpret_cast<rocblas_int*>(work + (int64_t)m * m);
  const float one = 1.0f, zero = 0.0f;
  hipError_t e;
  do {
    if ((s = rocblas_set_stream(h, st)) != rocblas_status_success) {
      err = rb_msg(s, "rocblas_set_stream");
      break;
    }
    // lower triangle of G = D^T D
    s = rocblas_ssyrk(h, rocblas_fill_lower, rocblas_operation_transpose, m, n_s, &one, im,
                      (rocblas_int)ld_im, &zero, G, m);
    if (s != rocblas_status_success) {
      err = rb_msg(s, "rocblas_ssyrk");
      break;
    }
    tlse_regularise_kernel<<<1, 1024, 0, st>>>(G, m, eps, w);
    if ((e = hipGetLastError()) != hipSuccess) {
      err = hipGetErrorString(e);
      break;
    }
    // G + lambda W = L L^T
    if ((s = rocsolver_spotrf(h, rocblas_fill_lower, m, G, m, d_info)) !=
        rocblas_status_success) {
      err = rb_msg(s, "rocsolver_spotrf");
      break;
    }
    if (R != im) {
      e = hipMemcpy2DAsync(R, ld_r * sizeof(float), im, ld_im * sizeof(float),
                           (size_t)n_s * sizeof(float), m, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) {
        err = hipGetErrorString(e);
        break;
      }
    }
    // R <- D L^-T, then R <- R L^-1 = D (L L^T)^-1
    s = rocblas_strsm(h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                      rocblas_diagonal_non_unit, n_s, m, &one, G, m, R, (rocblas_int)ld_r);
    if (s != rocblas_status_success) {
      err = rb_msg(s, "rocblas_strsm");
      break;
    }
    s = rocblas_strsm(h, rocblas_side_right, rocblas_fill_lower, rocblas_operation_none,
                      rocblas_diagonal_non_unit, n_s, m, &one, G, m, R, (rocblas_int)ld_r);
    if (s != rocblas_status_success) {
      err = rb_msg(s, "rocblas_strsm");
      break;
    }
    rocblas_int hinfo = 0;
    if ((e = hipMemcpyAsync(&hinfo, d_info, sizeof hinfo, hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess) {
      err = hipGetErrorString(e);
      break;
    }
    *info = hinfo;
  } while (false);
  rocblas_destroy_handle(h);
  return err;
}

}  // namespace wfs
