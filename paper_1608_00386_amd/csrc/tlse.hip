// Control matrix from an interaction matrix (Sec. 2.6 of the paper): the least-squares
// estimator with a diagonal (per-actuator weighted) Tikhonov term,
// R = (D^T D + eps mean(diag D^T D) W)^(-1) D^T for the interaction matrix D, built once from
// library dense linear algebra (rocBLAS syrk and trsm, rocSOLVER Cholesky).  It is set-up
// work outside the per-frame path, so it lives in a library of its own (libwfs_tlse.so, the
// only one that links rocBLAS and rocSOLVER); its errors go to libwfs's wfs_last_error.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cmath>
#include <cstdarg>
#include <stdint.h>
#include <stdio.h>

#include "../../include/wfs_tlse.h"

namespace wfs {
int set_error(int code, const char* msg);  // libwfs: the message wfs_last_error returns

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
static const char* tlse_run(const float* im, int32_t m, int32_t n_s, int64_t ld_im, float eps,
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

static int tlse_fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int tlse_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return wfs::set_error(code, buf);
}

extern "C" {

int wfs_tlse(const float* im, int32_t m, int32_t n_s, int64_t ld_im, float eps,
             const float* weights, float* R, int64_t ld_r, float* work, int64_t work_floats,
             void* stream) {
  if (!im || !R || !work) return tlse_fail(WFS_EINVAL, "wfs_tlse: null im, R or work");
  if (m < 1 || n_s < 1) return tlse_fail(WFS_EINVAL, "wfs_tlse: m=%d n_s=%d must be >= 1", m, n_s);
  if (m > 46000) return tlse_fail(WFS_EINVAL, "wfs_tlse: m=%d > 46000 actuators", m);
  if (ld_im < n_s || ld_r < n_s || ld_im > INT32_MAX || ld_r > INT32_MAX)
    return tlse_fail(WFS_EINVAL, "wfs_tlse: ld_im=%lld and ld_r=%lld must lie in [n_s=%d, 2^31)",
                (long long)ld_im, (long long)ld_r, n_s);
  if (R == im && ld_r != ld_im)
    return tlse_fail(WFS_EINVAL, "wfs_tlse: in place (R == im) needs ld_r == ld_im");
  if (!std::isfinite(eps) || eps < 0.0f)
    return tlse_fail(WFS_EINVAL, "wfs_tlse: eps must be finite and >= 0");
  const int64_t need = (int64_t)m * m + 64;
  if (work_floats < need)
    return tlse_fail(WFS_EINVAL, "wfs_tlse: work holds %lld floats, needs %lld",
                (long long)work_floats, (long long)need);
  int info = 0;
  const char* err = wfs::tlse_run(im, m, n_s, ld_im, eps, weights, R, ld_r, work,
                             (hipStream_t)stream, &info);
  if (err) return tlse_fail(WFS_EDEVICE, "wfs_tlse: %s", err);
  if (info != 0)
    return tlse_fail(WFS_EINVAL,
                "wfs_tlse: the regularised normal matrix is not positive definite (leading "
                "minor %d): raise eps or the weights", info);
  return WFS_OK;
}

}  // extern "C"
