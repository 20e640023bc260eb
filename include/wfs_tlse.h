/*
 * libwfs_tlse -- the control matrix (Sec. 2.6 of the paper), one-off set-up work kept out of
 * libwfs so that the per-frame path carries no dense-linear-algebra dependency: this library
 * alone links rocBLAS and rocSOLVER, and needs libwfs (error codes and wfs_last_error).
 */
#ifndef WFS_TLSE_H
#define WFS_TLSE_H

#include <stdint.h>

#include "wfs.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * wfs_tlse -- control matrix from an interaction matrix (Sec. 2.6: least-squares estimator,
 *   with a regularisation coefficient and per-actuator weights that set how the correction is
 *   shared between the DMs):  R = (D^T D + lambda diag(w))^-1 D^T,  lambda = eps * mean of
 *   diag(D^T D), where D[k][j] = im[j][k] (n_s slopes x m actuators).  im: device [m][ld_im]
 *   as wfs_calibrate writes it.  weights: device [m], >= 0, or NULL (all 1).  R: device
 *   [m][ld_r], row-major as recon_apply takes it; R == im (in place, ld_r == ld_im) is
 *   allowed.  work: device, >= m*m + 64 floats.  Set-up work: rocBLAS syrk and trsm with a
 *   rocSOLVER Cholesky factorisation, FP32; synchronises `stream`.  Errors as libwfs's calls
 *   (the message through wfs_last_error).  Returns WFS_EINVAL when
 *   the regularised matrix is not positive definite (eps = 0 with a rank-deficient D).
 */
int wfs_tlse(const float* im, int32_t m, int32_t n_s, int64_t ld_im, float eps,
             const float* weights, float* R, int64_t ld_r, float* work, int64_t work_floats,
             void* stream);

#ifdef __cplusplus
}
#endif

#endif /* WFS_TLSE_H */
