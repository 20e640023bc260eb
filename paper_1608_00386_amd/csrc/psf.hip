// Point-spread functions and Strehl ratios of the residual wavefront (Sec. 2.8 of the paper:
// PSFs at user wavelengths and pixel scales, on the GPU; Strehl ratio from the PSF or, by the
// Marechal approximation, from the history of the residual wavefront).
//
// Per frame, star and wavelength: residual phase on the full pupil grid (the layers and DM
// grids projected along the star's direction at infinity, bilinear, as for the sensors),
// field A exp(i kappa phi) zero-padded to N x N, its 2-D DFT, and |F|^2 / (N^2 sum A^2) added to
// a long-exposure image (unit sum per frame, zero frequency at pixel (N/2, N/2)).  The 2-D DFT
// is two passes over HBM: a row pass (one workgroup per pupil row: phase, field and an N-point
// FFT in LDS; only the n_pup non-zero rows exist) and a column pass (a few adjacent columns per
// workgroup, FFT in LDS, intensity accumulated in place).  Both FFTs are the Stockham
// radix-16 (+ one radix-2, 4 or 8 stage) transforms of lds_fft.h, compiled per log2 N, on
// bank-conflict-free padded LDS; their twiddle table is computed in double precision on the
// host (staged in LDS by the column pass).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/wfs.h"
#include "lds_fft.h"
#include "wfs_common.h"

namespace wfs {
int set_error(int code, const char* msg);

constexpr int kPsfBlock = 256;
constexpr int kPsfPoints = 4096;     // largest transform (and one row-pass workgroup's LDS)
constexpr int kPsfColPoints = 16384; // LDS points of a column-pass workgroup (C columns x N)
constexpr int kPsfColLds = 160 * 1024;  // its LDS bytes at most: C pitch + N - 1 float2
constexpr int kPsfRowLds = fft_span(kPsfPoints) * 8;  // one padded row
constexpr int kPsfMinLog2 = 4, kPsfMaxLog2 = 12;
constexpr int kPsfMaxLambda = 16;
constexpr int kPsfMaxStars = 256;

// u = ax*i + bx0 + step*dbx (column i), v = ay*j + by0 + step*dby (row j) in layer pixels.
struct PsfAff {
  double ax, bx0, dbx, ay, by0, dby;
};

struct PsfParams {
  const float* layers;
  const DevLayer* lay;
  const PsfAff* aff;     // [n_stars][n_layers]
  const uint8_t* mask;   // [n_pup][n_pup] pupil amplitude (0 / 1)
  const float2* tw;      // the N - 1 twiddles of lds_fft, stage after stage
  float2* T;             // [n_stars][n_pup][N] row transforms
  double* part;          // [n_stars][n_pup][2]: row sums of A phi and A phi^2 (reference wavelength)
  float* psf;            // this wavelength's [n_stars][N][N]
  int64_t step;
  int32_t n_layers, n_stars, n_pup, N, log2N, cols;
  float kappa, scale;
  int32_t write_part;
};

// Per-layer parameters of one pupil row, staged in LDS by the workgroup: the row tap (fixed
// for the row), the column affine map, and how the two layer rows are read (flags: kRowStaged
// = copied to LDS first, kRowVec4 = with 16-byte loads).
struct RowLayer {
  double a, b, inv_n;
  int64_t offset;
  int32_t n, boundary, r0, r1;
  float w0, w1, weight;
  int32_t flags;
};
constexpr int kRowStaged = 1, kRowVec4 = 2;

// Row pass: workgroup (row y, star s).  Phase of the pupil row, field, N-point FFT, row of T
// stored in C-column tiles: T[s][k / C][y][k % C], so the column pass reads whole tiles.
// The phase is a bilinear gather of every layer; when the pupil row is one pass of the
// threads and two rows of a layer fit twice in the FFT buffer (free until the field is
// written), the two layer rows of the pupil row's row tap are first copied to LDS with
// coalesced loads (double-buffered by layer, one barrier a layer) and the stencils read LDS:
// about a sixth of the load instructions of the per-pixel gather, the same arithmetic.
template <int LOG2N>
__global__ __launch_bounds__(kPsfBlock) void psf_rows_kernel(PsfParams p) {
  extern __shared__ __align__(16) float2 sh[];
  __shared__ double red[2][kPsfBlock];
  __shared__ RowLayer rl[kMaxLayers];
  constexpr int N = 1 << LOG2N;
  const int y = blockIdx.x, s = blockIdx.y, tid = threadIdx.x;
  const int n = p.n_pup, C = p.cols, lc = __builtin_ctz(C);  // C: a power of two
  if (tid < p.n_layers) {
    const DevLayer L = p.lay[tid];
    const PsfAff A = p.aff[s * p.n_layers + tid];
    const double stepd = (double)p.step;
    const Tap ry = make_tap(fma(A.ay, (double)y, A.by0) + stepd * A.dby, L.ny, L.inv_ny,
                            L.boundary, L.nx);
    RowLayer r;
    r.a = A.ax;
    r.b = A.bx0 + stepd * A.dbx;
    r.inv_n = L.inv_nx;
    r.offset = L.offset;
    r.n = L.nx;
    r.boundary = L.boundary;
    r.r0 = ry.i0;
    r.r1 = ry.i1;
    r.w0 = ry.w0;
    r.w1 = ry.w1;
    r.weight = L.weight;
    r.flags = 0;
    if (n <= 4 * kPsfBlock && 4 * L.nx <= 2 * fft_span(N)) {
      r.flags = kRowStaged;
      const uintptr_t a0 = reinterpret_cast<uintptr_t>(p.layers + L.offset);
      if ((L.nx & 3) == 0 && (a0 & 15) == 0 && (fft_span(N) & 3) == 0) r.flags |= kRowVec4;
    }
    rl[tid] = r;
  }
  __syncthreads();
  double s1 = 0.0, s2 = 0.0;
  // pupil pixels in blocks of kPix per thread: layers outer, pixels inner, so each layer's
  // parameters are read once per block and its 4 kPix taps load back to back
  constexpr int kPix = 4;
  for (int x0 = 0; x0 < n; x0 += kPix * kPsfBlock) {
    float phi[kPix];
    bool lit[kPix];
#pragma unroll
    for (int j = 0; j < kPix; ++j) {
      const int x = x0 + tid + j * kPsfBlock;
      lit[j] = x < n && p.mask[(int64_t)y * n + x];
      phi[j] = 0.0f;
    }
    int ks = 0;  // staged layers so far (workgroup-uniform)
    for (int l = 0; l < p.n_layers; ++l) {
      const RowLayer r = rl[l];
      const Tap ry{r.r0, r.r1, r.w0, r.w1};
      const float* g = p.layers + r.offset;
      if (r.flags & kRowStaged) {  // workgroup-uniform
        // rows ry.i0 / nx and ry.i1 / nx of the layer -> buffer ks % 2, each buffer half of
        // the FFT region (its last readers, the staged layer before the previous one, are
        // behind the previous staged layer's barrier)
        float* b0 = reinterpret_cast<float*>(sh) + (ks++ & 1) * fft_span(N);
        float* b1 = b0 + r.n;
        if (r.flags & kRowVec4) {
          const float4* g0 = reinterpret_cast<const float4*>(g + ry.i0);
          const float4* g1 = reinterpret_cast<const float4*>(g + ry.i1);
          for (int c = tid; c < (r.n >> 2); c += kPsfBlock) {
            reinterpret_cast<float4*>(b0)[c] = g0[c];
            reinterpret_cast<float4*>(b1)[c] = g1[c];
          }
        } else {
          for (int c = tid; c < r.n; c += kPsfBlock) {
            b0[c] = g[ry.i0 + c];
            b1[c] = g[ry.i1 + c];
          }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kPix; ++j) {
          if (lit[j]) {
            const int x = x0 + tid + j * kPsfBlock;
            const Tap cx = make_tap(fma(r.a, (double)x, r.b), r.n, r.inv_n, r.boundary, 1);
            const float v00 = b0[cx.i0], v01 = b0[cx.i1], v10 = b1[cx.i0], v11 = b1[cx.i1];
            const float v = ry.w0 * fmaf(cx.w0, v00, cx.w1 * v01) +
                            ry.w1 * fmaf(cx.w0, v10, cx.w1 * v11);  // as bilinear()
            phi[j] = fmaf(r.weight, v, phi[j]);
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < kPix; ++j) {
          if (lit[j]) {
            const int x = x0 + tid + j * kPsfBlock;
            const Tap cx = make_tap(fma(r.a, (double)x, r.b), r.n, r.inv_n, r.boundary, 1);
            phi[j] = fmaf(r.weight, bilinear(g, cx, ry), phi[j]);
          }
        }
      }
    }
    __syncthreads();  // the staged rows are read before the field overwrites the buffer
#pragma unroll
    for (int j = 0; j < kPix; ++j) {
      const int x = x0 + tid + j * kPsfBlock;
      float2 e = make_float2(0.0f, 0.0f);
      if (lit[j]) {
        s1 += (double)phi[j];
        s2 += (double)phi[j] * (double)phi[j];
        float sn, cs;
        sincosf(p.kappa * phi[j], &sn, &cs);
        e = make_float2(cs, sn);
      }
      if (x < N) sh[fft_pad(x)] = e;
    }
  }
  for (int x = n + tid; x < N; x += kPsfBlock) {  // zero padding beyond the pupil
    if (x >= ((n + kPix * kPsfBlock - 1) / (kPix * kPsfBlock)) * kPix * kPsfBlock)
      sh[fft_pad(x)] = make_float2(0.0f, 0.0f);
  }
  if (p.write_part) {  // fixed-order tree: deterministic row sums
    red[0][tid] = s1;
    red[1][tid] = s2;
    __syncthreads();
    for (int w = kPsfBlock / 2; w > 0; w >>= 1) {
      if (tid < w) {
        red[0][tid] += red[0][tid + w];
        red[1][tid] += red[1][tid + w];
      }
      __syncthreads();
    }
    if (tid == 0) {
      double* o = p.part + ((int64_t)s * n + y) * 2;
      o[0] = red[0][0];
      o[1] = red[1][0];
    }
  }
  __syncthreads();
  lds_fft<LOG2N, N, kPsfBlock>(sh, 1, fft_span(N), p.tw);
  float2* out = p.T + (int64_t)s * n * N + (int64_t)y * C;
  for (int x = tid; x < N; x += kPsfBlock) {
    const int kt = x >> lc;
    out[(int64_t)kt * n * C + (x - kt * C)] = sh[fft_pad(x)];
  }
}

// Column pass: workgroup (C adjacent columns, star s), blocks renumbered so that neighbouring
// column groups share an XCD (and its L2 lines of T).  Zero rows beyond the pupil are implicit.
constexpr int kPsfColBlock = 1024;  // 16 waves: the column pass is LDS-latency bound

template <int LOG2N>
__global__ __launch_bounds__(kPsfColBlock) void psf_cols_kernel(PsfParams p) {
  extern __shared__ float2 sh[];
  constexpr int N = 1 << LOG2N;
  const int tid = threadIdx.x;
  const int C = p.cols, lc = __builtin_ctz(C), n = p.n_pup, ld = fft_pitch(N, C);
  const int groups = N >> lc;
  const int lb = xcd_logical_block(blockIdx.x, groups * p.n_stars);
  const int s = lb / groups, k0 = (lb - s * groups) * C;
  const float2* src = p.T + (int64_t)s * n * N + (int64_t)k0 * n;  // tile k0 / C: [n][C]
  float2* tws = sh + C * ld;  // the twiddle table, staged in LDS after the data
  for (int i = tid; i < C * N; i += kPsfColBlock) {
    const int c = i & (C - 1), y = i >> lc;
    sh[c * ld + fft_pad(y)] = y < n ? src[i] : make_float2(0.0f, 0.0f);
  }
  for (int i = tid; i < N - 1; i += kPsfColBlock) tws[i] = p.tw[i];
  __syncthreads();
  lds_fft<LOG2N, kPsfColPoints, kPsfColBlock>(sh, C, ld, tws);
  // intensities from LDS, then every read of the long-exposure image before any write (one
  // memory latency per thread instead of one per pixel)
  float* __restrict__ dst = p.psf + (int64_t)s * N * N;
  const int h = N >> 1;
  constexpr int kPer = kPsfColPoints / kPsfColBlock;
  float val[kPer];
  int64_t at[kPer];
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int i = tid + r * kPsfColBlock;
    if (i < C * N) {
      const int c = i & (C - 1), v = i >> lc;
      const float2 f = sh[c * ld + fft_pad(v)];
      val[r] = (f.x * f.x + f.y * f.y) * p.scale;
      at[r] = (int64_t)((v + h) & (N - 1)) * N + ((k0 + c + h) & (N - 1));
    }
  }
  float old[kPer];
#pragma unroll
  for (int r = 0; r < kPer; ++r)
    if (tid + r * kPsfColBlock < C * N) old[r] = dst[at[r]];
#pragma unroll
  for (int r = 0; r < kPer; ++r)
    if (tid + r * kPsfColBlock < C * N) dst[at[r]] = old[r] + val[r];
}

struct PsfVarParams {
  const double* part;
  double* phase_var;  // [n_lambda][n_stars]
  int32_t n_pup, n_stars, n_lambda;
  double inv_lit;
  float kappa2[kPsfMaxLambda];
};

// Piston-removed pupil variance of this frame's phase, per star (one workgroup each: strided
// row sums, then a fixed-order tree), added at every wavelength.
__global__ __launch_bounds__(kPsfBlock) void psf_var_kernel(PsfVarParams q) {
  __shared__ double red[2][kPsfBlock];
  const int s = blockIdx.x, tid = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int y = tid; y < q.n_pup; y += kPsfBlock) {
    a += q.part[((int64_t)s * q.n_pup + y) * 2];
    b += q.part[((int64_t)s * q.n_pup + y) * 2 + 1];
  }
  red[0][tid] = a;
  red[1][tid] = b;
  __syncthreads();
  for (int w = kPsfBlock / 2; w > 0; w >>= 1) {
    if (tid < w) {
      red[0][tid] += red[0][tid + w];
      red[1][tid] += red[1][tid + w];
    }
    __syncthreads();
  }
  if (tid < q.n_lambda) {
    const double m = red[0][0] * q.inv_lit;
    const double var = red[1][0] * q.inv_lit - m * m;
    q.phase_var[tid * q.n_stars + s] += (double)q.kappa2[tid] * var;
  }
}

struct PsfStrehlParams {
  const float* psf;
  const double* phase_var;
  float* sr_psf;
  float* sr_marechal;
  int32_t n_stars, n_lambda;
  double inv_frames;
  int64_t off[kPsfMaxLambda];   // first float of wavelength l's images
  int32_t N[kPsfMaxLambda];
  double inv_peak[kPsfMaxLambda];  // N^2 / sum A: inverse of the diffraction-limited peak
};

__global__ __launch_bounds__(kPsfBlock) void psf_strehl_kernel(PsfStrehlParams q) {
  const int i = blockIdx.x * kPsfBlock + threadIdx.x;
  if (i >= q.n_lambda * q.n_stars) return;
  const int l = i / q.n_stars, s = i - l * q.n_stars;
  const int N = q.N[l], h = N >> 1;
  if (q.sr_psf && q.psf) {
    const float c = q.psf[q.off[l] + (int64_t)s * N * N + (int64_t)h * N + h];
    q.sr_psf[i] = (float)((double)c * q.inv_frames * q.inv_peak[l]);
  }
  if (q.sr_marechal && q.phase_var)
    q.sr_marechal[i] = (float)exp(-q.phase_var[i] * q.inv_frames);
}

}  // namespace wfs

using namespace wfs;

struct psf_plan_s {
  int device = 0;
  int32_t n_layers = 0, n_stars = 0, n_pup = 0, n_lambda = 0;
  int64_t layer_stride = 0, n_lit = 0, psf_floats = 0;
  std::vector<int32_t> N, log2N, cols;
  std::vector<float> kappa;
  std::vector<int64_t> psf_off, tw_off;
  DevLayer* lay = nullptr;
  PsfAff* aff = nullptr;
  uint8_t* mask = nullptr;
  float2* tw = nullptr;
  float2* T = nullptr;
  double* part = nullptr;
};

static int psf_fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int psf_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return set_error(code, buf);
}

static int psf_hip(hipError_t e, const char* what) {
  return psf_fail(e == hipErrorOutOfMemory ? WFS_ENOMEM : WFS_EDEVICE, "%s: %s", what,
                  hipGetErrorString(e));
}

static void psf_free(psf_plan_t P) {
  if (!P) return;
  (void)hipFree(P->lay);
  (void)hipFree(P->aff);
  (void)hipFree(P->mask);
  (void)hipFree(P->tw);
  (void)hipFree(P->T);
  (void)hipFree(P->part);
  delete P;
}

// Calls f(std::integral_constant<int, log2 N>) for a transform size of the plan.
template <class F>
static void psf_dispatch(int log2N, F&& f) {
  switch (log2N) {
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 9: f(std::integral_constant<int, 9>{}); break;
    case 10: f(std::integral_constant<int, 10>{}); break;
    case 11: f(std::integral_constant<int, 11>{}); break;
    default: f(std::integral_constant<int, 12>{}); break;
  }
}

template <class T>
static hipError_t upload(T** dst, const std::vector<T>& v) {
  hipError_t e = hipMalloc((void**)dst, v.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

extern "C" {

int psf_plan(const wfs_layer_desc* layers, int32_t n_layers, int64_t layer_stride,
             const double* star_theta_xy, int32_t n_stars, double pupil_d_m, double obs_d_m,
             int32_t n_pup, const double* lambda_m, const int32_t* n_fft, int32_t n_lambda,
             double lambda_ref_m, double dt_s, psf_plan_t* out) {
  if (!out) return psf_fail(WFS_EINVAL, "psf_plan: null out");
  *out = nullptr;
  if (!layers || !star_theta_xy || !lambda_m || !n_fft)
    return psf_fail(WFS_EINVAL, "psf_plan: null argument");
  if (n_layers < 1 || n_layers > kMaxLayers)
    return psf_fail(WFS_EINVAL, "psf_plan: n_layers=%d outside [1, %d]", n_layers, kMaxLayers);
  if (n_stars < 1 || n_stars > kPsfMaxStars)
    return psf_fail(WFS_EINVAL, "psf_plan: n_stars=%d outside [1, %d]", n_stars, kPsfMaxStars);
  if (n_lambda < 1 || n_lambda > kPsfMaxLambda)
    return psf_fail(WFS_EINVAL, "psf_plan: n_lambda=%d outside [1, %d]", n_lambda,
                    kPsfMaxLambda);
  if (n_pup < 2 || n_pup > kPsfPoints)
    return psf_fail(WFS_EINVAL, "psf_plan: n_pup=%d outside [2, %d]", n_pup, kPsfPoints);
  if (!(pupil_d_m > 0) || !std::isfinite(pupil_d_m) || !(obs_d_m >= 0) || obs_d_m >= pupil_d_m)
    return psf_fail(WFS_EINVAL, "psf_plan: pupil %g m, obstruction %g m", pupil_d_m, obs_d_m);
  if (!(lambda_ref_m > 0) || !std::isfinite(lambda_ref_m) || !(dt_s >= 0) ||
      !std::isfinite(dt_s))
    return psf_fail(WFS_EINVAL, "psf_plan: lambda_ref_m > 0 and dt_s >= 0 required");
  if (layer_stride < 1) return psf_fail(WFS_EINVAL, "psf_plan: layer_stride < 1");
  for (int l = 0; l < n_layers; ++l) {
    const wfs_layer_desc& L = layers[l];
    if (L.nx < 2 || L.ny < 2 || (int64_t)L.nx * L.ny > (1LL << 29))
      return psf_fail(WFS_EINVAL, "psf_plan: layer %d grid %dx%d", l, L.nx, L.ny);
    if (L.offset < 0 || L.offset + (int64_t)L.nx * L.ny > layer_stride)
      return psf_fail(WFS_EINVAL, "psf_plan: layer %d outside the stride", l);
    if (!(L.pitch_m > 0) || !std::isfinite(L.pitch_m) || !std::isfinite(L.alt_m) ||
        L.alt_m < 0 || !std::isfinite(L.vx_mps) || !std::isfinite(L.vy_mps) ||
        !std::isfinite(L.weight) || (L.boundary != 0 && L.boundary != 1))
      return psf_fail(WFS_EINVAL, "psf_plan: layer %d geometry", l);
  }
  for (int s = 0; s < 2 * n_stars; ++s)
    if (!std::isfinite(star_theta_xy[s])) return psf_fail(WFS_EINVAL, "psf_plan: star angle");
  for (int l = 0; l < n_lambda; ++l) {
    const int32_t N = n_fft[l];
    if (!(lambda_m[l] > 0) || !std::isfinite(lambda_m[l]))
      return psf_fail(WFS_EINVAL, "psf_plan: lambda %d must be > 0", l);
    if (N < 16 || N > kPsfPoints || (N & (N - 1)) || N < n_pup)
      return psf_fail(WFS_EINVAL,
                      "psf_plan: n_fft[%d]=%d must be a power of two in [max(16, n_pup=%d), %d]",
                      l, N, n_pup, kPsfPoints);
  }
  psf_plan_t P = new psf_plan_s();
  hipError_t e = hipGetDevice(&P->device);
  if (e != hipSuccess) {
    psf_free(P);
    return psf_hip(e, "psf_plan");
  }
  P->n_layers = n_layers;
  P->n_stars = n_stars;
  P->n_pup = n_pup;
  P->n_lambda = n_lambda;
  P->layer_stride = layer_stride;
  // pupil: pixel centres x_i = (i + 1/2 - n/2) dx; A = 1 for obs/2 <= r <= D/2
  const double dx = pupil_d_m / n_pup;
  std::vector<uint8_t> mask((size_t)n_pup * n_pup);
  for (int j = 0; j < n_pup; ++j)
    for (int i = 0; i < n_pup; ++i) {
      const double xx = (i + 0.5 - n_pup / 2.0) * dx, yy = (j + 0.5 - n_pup / 2.0) * dx;
      const double r = std::hypot(xx, yy);
      const bool lit = r >= obs_d_m / 2.0 && r <= pupil_d_m / 2.0;
      mask[(size_t)j * n_pup + i] = lit;
      P->n_lit += lit;
    }
  if (P->n_lit == 0) {
    psf_free(P);
    return psf_fail(WFS_EINVAL, "psf_plan: no lit pupil pixel");
  }
  std::vector<DevLayer> lay(n_layers);
  std::vector<PsfAff> aff((size_t)n_stars * n_layers);
  for (int l = 0; l < n_layers; ++l) {
    const wfs_layer_desc& L = layers[l];
    lay[l] = DevLayer{L.offset, L.nx, L.ny, L.weight, L.boundary, 1.0 / L.nx, 1.0 / L.ny};
    for (int s = 0; s < n_stars; ++s) {
      // a star at infinity: X = x + theta h - v t, u = X / pitch + nx/2 - 1/2
      const double tx = star_theta_xy[2 * s], ty = star_theta_xy[2 * s + 1];
      PsfAff& A = aff[(size_t)s * n_layers + l];
      A.ax = dx / L.pitch_m;
      A.bx0 = ((0.5 - n_pup / 2.0) * dx + tx * L.alt_m) / L.pitch_m + L.nx / 2.0 - 0.5;
      A.dbx = -L.vx_mps * dt_s / L.pitch_m;
      A.ay = dx / L.pitch_m;
      A.by0 = ((0.5 - n_pup / 2.0) * dx + ty * L.alt_m) / L.pitch_m + L.ny / 2.0 - 0.5;
      A.dby = -L.vy_mps * dt_s / L.pitch_m;
    }
  }
  std::vector<float2> tw;
  int32_t Nmax = 0;
  for (int l = 0; l < n_lambda; ++l) {
    const int32_t N = n_fft[l];
    int lg = 0;
    while ((1 << lg) < N) ++lg;
    P->N.push_back(N);
    P->log2N.push_back(lg);
    // C padded columns of N points plus the N - 1 twiddles must fit the 160 KB of LDS
    P->cols.push_back(N >= 4096 ? 2 : std::min(16, kPsfColPoints / N));
    P->kappa.push_back((float)(lambda_ref_m / lambda_m[l]));
    P->psf_off.push_back(P->psf_floats);
    P->psf_floats += (int64_t)n_stars * N * N;
    P->tw_off.push_back((int64_t)tw.size());
    for (int m = 0; m < N - 1; ++m) {
      const double a = -2.0 * M_PI * (double)fft_tw_angle(lg, m) / (double)N;
      tw.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
    }
    Nmax = std::max(Nmax, N);
  }
  // the column pass holds more than the default 64 KB of LDS (data, padding and twiddles)
  e = hipSuccess;
  for (int lg = kPsfMinLog2; lg <= kPsfMaxLog2 && e == hipSuccess; ++lg) {
    psf_dispatch(lg, [&](auto L) {
      constexpr int LG = decltype(L)::value;
      if ((e = hipFuncSetAttribute((const void*)psf_cols_kernel<LG>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, kPsfColLds)) ==
          hipSuccess)
        e = hipFuncSetAttribute((const void*)psf_rows_kernel<LG>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, kPsfRowLds);
    });
  }
  if (e != hipSuccess) {
    psf_free(P);
    return psf_hip(e, "psf_plan: column-pass LDS");
  }
  if ((e = upload(&P->lay, lay)) != hipSuccess || (e = upload(&P->aff, aff)) != hipSuccess ||
      (e = upload(&P->mask, mask)) != hipSuccess || (e = upload(&P->tw, tw)) != hipSuccess ||
      (e = hipMalloc((void**)&P->T, (size_t)n_stars * n_pup * Nmax * sizeof(float2))) !=
          hipSuccess ||
      (e = hipMalloc((void**)&P->part, (size_t)n_stars * n_pup * 2 * sizeof(double))) !=
          hipSuccess) {
    psf_free(P);
    return psf_hip(e, "psf_plan: device tables");
  }
  *out = P;
  return WFS_OK;
}

int psf_plan_info(psf_plan_t P, int64_t* psf_floats, int64_t* psf_offsets, int64_t* n_lit) {
  if (!P) return psf_fail(WFS_EINVAL, "psf_plan_info: null plan");
  if (psf_floats) *psf_floats = P->psf_floats;
  if (psf_offsets)
    for (int l = 0; l < P->n_lambda; ++l) psf_offsets[l] = P->psf_off[l];
  if (n_lit) *n_lit = P->n_lit;
  return WFS_OK;
}

int psf_plan_destroy(psf_plan_t P) {
  if (!P) return psf_fail(WFS_EINVAL, "psf_plan_destroy: null plan");
  hipError_t e = hipDeviceSynchronize();
  psf_free(P);
  if (e != hipSuccess) return psf_hip(e, "psf_plan_destroy");
  return WFS_OK;
}

int psf_accumulate(psf_plan_t P, const float* layers, int64_t step, float* psf,
                   double* phase_var, void* stream) {
  if (!P) return psf_fail(WFS_EINVAL, "psf_accumulate: null plan");
  if (!layers || !psf) return psf_fail(WFS_EINVAL, "psf_accumulate: null layers or psf");
  if (step < 0) return psf_fail(WFS_EINVAL, "psf_accumulate: step=%lld < 0", (long long)step);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return psf_hip(e, "psf_accumulate");
  if (dev != P->device)
    return psf_fail(WFS_EINVAL, "psf_accumulate: current device %d is not the plan's %d", dev,
                    P->device);
  hipStream_t st = (hipStream_t)stream;
  for (int l = 0; l < P->n_lambda; ++l) {
    PsfParams p{};
    p.layers = layers;
    p.lay = P->lay;
    p.aff = P->aff;
    p.mask = P->mask;
    p.tw = P->tw + P->tw_off[l];
    p.T = P->T;
    p.part = P->part;
    p.psf = psf + P->psf_off[l];
    p.step = step;
    p.n_layers = P->n_layers;
    p.n_stars = P->n_stars;
    p.n_pup = P->n_pup;
    p.N = P->N[l];
    p.log2N = P->log2N[l];
    p.cols = P->cols[l];
    p.kappa = P->kappa[l];
    p.scale = (float)(1.0 / ((double)p.N * p.N * (double)P->n_lit));
    p.write_part = (l == 0 && phase_var) ? 1 : 0;
    psf_dispatch(p.log2N, [&](auto L) {
      psf_rows_kernel<decltype(L)::value><<<dim3(P->n_pup, P->n_stars), kPsfBlock,
                                            (size_t)fft_span(p.N) * sizeof(float2), st>>>(p);
    });
    if ((e = hipGetLastError()) != hipSuccess) return psf_hip(e, "psf_accumulate: rows");
    if (p.write_part) {
      PsfVarParams q{};
      q.part = P->part;
      q.phase_var = phase_var;
      q.n_pup = P->n_pup;
      q.n_stars = P->n_stars;
      q.n_lambda = P->n_lambda;
      q.inv_lit = 1.0 / (double)P->n_lit;
      for (int m = 0; m < P->n_lambda; ++m) q.kappa2[m] = P->kappa[m] * P->kappa[m];
      psf_var_kernel<<<P->n_stars, kPsfBlock, 0, st>>>(q);
      if ((e = hipGetLastError()) != hipSuccess) return psf_hip(e, "psf_accumulate: variance");
    }
    const int blocks = (p.N / p.cols) * P->n_stars;
    const size_t lds = ((size_t)p.cols * fft_pitch(p.N, p.cols) + p.N - 1) * sizeof(float2);
    psf_dispatch(p.log2N, [&](auto L) {
      psf_cols_kernel<decltype(L)::value><<<blocks, kPsfColBlock, lds, st>>>(p);
    });
    if ((e = hipGetLastError()) != hipSuccess) return psf_hip(e, "psf_accumulate: columns");
  }
  return WFS_OK;
}

int psf_strehl(psf_plan_t P, const float* psf, const double* phase_var, int64_t n_frames,
               float* sr_psf, float* sr_marechal, void* stream) {
  if (!P) return psf_fail(WFS_EINVAL, "psf_strehl: null plan");
  if (n_frames < 1) return psf_fail(WFS_EINVAL, "psf_strehl: n_frames=%lld < 1",
                                    (long long)n_frames);
  if ((sr_psf && !psf) || (sr_marechal && !phase_var) || (!sr_psf && !sr_marechal))
    return psf_fail(WFS_EINVAL, "psf_strehl: outputs need their inputs (psf, phase_var)");
  PsfStrehlParams q{};
  q.psf = psf;
  q.phase_var = phase_var;
  q.sr_psf = sr_psf;
  q.sr_marechal = sr_marechal;
  q.n_stars = P->n_stars;
  q.n_lambda = P->n_lambda;
  q.inv_frames = 1.0 / (double)n_frames;
  for (int l = 0; l < P->n_lambda; ++l) {
    q.off[l] = P->psf_off[l];
    q.N[l] = P->N[l];
    q.inv_peak[l] = (double)P->N[l] * P->N[l] / (double)P->n_lit;
  }
  const int n = P->n_lambda * P->n_stars;
  psf_strehl_kernel<<<(n + kPsfBlock - 1) / kPsfBlock, kPsfBlock, 0, (hipStream_t)stream>>>(q);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return psf_hip(e, "psf_strehl");
  return WFS_OK;
}

}  // extern "C"
