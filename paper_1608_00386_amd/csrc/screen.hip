// Phase screens on the GPU (Sec. 2.1 of the paper: the atmosphere is a set of phase screens
// made by filtering random noise in the Fourier domain with a Kolmogorov or von Karman phase
// spectrum, parameterised by r0 and L0).
//
//   phi = Re( sum_k W_k sqrt(PSD(f_k)) df exp(+2 pi i k.x / n) ),  W = a + i b, a, b ~ N(0, 1),
//   PSD(f) = 0.023 r0^(-5/3) (f^2 + L0^-2)^(-11/6)  (L0 = infinity: Kolmogorov), f = 0 zeroed,
//
// on an n x n periodic grid of pitch dx (df = 1 / (n dx)).  The noise is Philox4x32-10 keyed by
// the seed, one block per Fourier sample (counter: sample index, stream id), Box-Muller on its
// first two words.  The unnormalised inverse DFT is the forward one of the conjugate; it runs
// as the PSF module's two passes: rows (noise, filter and an n-point FFT in LDS, written in
// C-column tiles) and columns (FFT in LDS, real part out); each workgroup forms its own
// twiddles in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "../../include/wfs.h"
#include "lds_fft.h"
#include "wfs_common.h"

namespace wfs {
int set_error(int code, const char* msg);

constexpr int kScrBlock = 256;
constexpr int kScrMaxN = 4096;
constexpr int kScrColPoints = 16384;
constexpr int kScrColBlock = 1024;

struct ScreenParams {
  float2* T;            // [n / C][n][C] row transforms
  float* out;           // [n][n]
  int32_t n, log2n, cols;
  float c_psd;          // 0.023 r0^(-5/3)
  float inv_l02;        // L0^-2 (0: Kolmogorov)
  float inv_ndx;        // df = 1 / (n dx), cycles per metre per frequency index
  uint32_t seed_lo, seed_hi, sid_lo, sid_hi;
};

// The n - 1 twiddles of lds_fft into LDS (FP32 sincospi: about one ulp).
template <int LOG2N>
__device__ __forceinline__ void screen_twiddles(float2* tws, int nthreads) {
  constexpr int n = 1 << LOG2N;
  for (int m = threadIdx.x; m < n - 1; m += nthreads) {
    float sn, cs;
    sincospif(-2.0f * (float)fft_tw_angle(LOG2N, m) / (float)n, &sn, &cs);
    tws[m] = make_float2(cs, sn);
  }
}

// Row pass: workgroup per row ky of the spectrum.
template <int LOG2N>
__global__ __launch_bounds__(kScrBlock) void screen_rows_kernel(ScreenParams p) {
  extern __shared__ float2 sh[];
  constexpr int n = 1 << LOG2N;
  const int ky = blockIdx.x, tid = threadIdx.x, C = p.cols, lc = __builtin_ctz(C);
  const int iy = ky < n / 2 ? ky : ky - n;  // frequency index in [-n/2, n/2)
  const float fy = (float)iy * p.inv_ndx;
  for (int kx = tid; kx < n; kx += kScrBlock) {
    const int ix = kx < n / 2 ? kx : kx - n;
    const float fx = (float)ix * p.inv_ndx;
    const float f2 = fx * fx + fy * fy;
    float amp = 0.0f;
    if (kx | ky) {
      // sqrt(PSD) df = sqrt(c) (f^2 + L0^-2)^(-11/12) df
      amp = sqrtf(p.c_psd) * exp2f(-11.0f / 12.0f * log2f(f2 + p.inv_l02)) * p.inv_ndx;
    }
    const uint32_t idx = (uint32_t)ky * (uint32_t)n + (uint32_t)kx;
    const uint4 w = philox4x32_10(make_uint4(idx, 0u, p.sid_lo, p.sid_hi), p.seed_lo, p.seed_hi);
    const float r = sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u24(w.x)));
    float sn, cs;
    sincos_rev(u24(w.y), &sn, &cs);
    // conjugate spectrum: the forward transform of conj(S) is conj of the inverse of S
    sh[fft_pad(kx)] = make_float2(r * cs * amp, -(r * sn * amp));
  }
  float2* tws = sh + fft_span(n);  // the twiddles, after the row
  screen_twiddles<LOG2N>(tws, kScrBlock);
  __syncthreads();
  lds_fft<LOG2N, n, kScrBlock>(sh, 1, fft_span(n), tws);
  float2* o = p.T + (int64_t)ky * C;
  for (int x = tid; x < n; x += kScrBlock) {
    const int kt = x >> lc;
    o[(int64_t)kt * n * C + (x - kt * C)] = sh[fft_pad(x)];
  }
}

// Column pass: C adjacent columns per workgroup; the screen is the real part.
template <int LOG2N>
__global__ __launch_bounds__(kScrColBlock) void screen_cols_kernel(ScreenParams p) {
  extern __shared__ float2 sh[];
  constexpr int n = 1 << LOG2N;
  const int tid = threadIdx.x, C = p.cols, lc = __builtin_ctz(C), ld = fft_pitch(n, C);
  const int groups = n >> lc;
  const int g = xcd_logical_block(blockIdx.x, groups);
  const int x0 = g * C;
  const float2* src = p.T + (int64_t)x0 * n;  // tile x0 / C: [n][C]
  float2* tws = sh + C * ld;
  for (int i = tid; i < C * n; i += kScrColBlock) {
    const int c = i & (C - 1), y = i >> lc;
    sh[c * ld + fft_pad(y)] = src[i];
  }
  screen_twiddles<LOG2N>(tws, kScrColBlock);
  __syncthreads();
  lds_fft<LOG2N, kScrColPoints, kScrColBlock>(sh, C, ld, tws);
  for (int i = tid; i < C * n; i += kScrColBlock) {
    const int c = i & (C - 1), y = i >> lc;
    p.out[(int64_t)y * n + x0 + c] = sh[c * ld + fft_pad(y)].x;
  }
}

}  // namespace wfs

using namespace wfs;

static int scr_fail(int code, const char* msg) { return set_error(code, msg); }

// Calls f(std::integral_constant<int, log2 n>) for a screen size 16 <= n <= 4096.
template <class F>
static void scr_dispatch(int log2n, F&& f) {
  switch (log2n) {
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

extern "C" {

int screen_generate(int32_t n, double pitch_m, double r0_m, double L0_m, uint64_t seed,
                    uint64_t stream_id, float* screen, float* work, int64_t work_floats,
                    void* stream) {
  if (!screen || !work) return scr_fail(WFS_EINVAL, "screen_generate: null screen or work");
  if (n < 16 || n > kScrMaxN || (n & (n - 1)))
    return scr_fail(WFS_EINVAL, "screen_generate: n must be a power of two in [16, 4096]");
  if (!(pitch_m > 0) || !std::isfinite(pitch_m) || !(r0_m > 0) || !std::isfinite(r0_m) ||
      !(L0_m > 0))
    return scr_fail(WFS_EINVAL, "screen_generate: pitch, r0 and L0 must be > 0");
  if (work_floats < 2 * (int64_t)n * n)
    return scr_fail(WFS_EINVAL, "screen_generate: work must hold 2 n^2 floats");
  int log2n = 0;
  while ((1 << log2n) < n) ++log2n;
  // columns per column-pass workgroup: enough workgroups to cover the 256 CUs (n / C >= 256
  // where n allows), C (n + 1) + n points within the 160 KB of LDS
  const int cols = n >= 4096 ? 2 : std::max(2, std::min(n / 256, kScrColPoints / n));
  hipError_t e;
  static std::once_flag lds_once;
  static hipError_t lds_err = hipSuccess;
  std::call_once(lds_once, [] {
    for (int lg = 4; lg <= 12 && lds_err == hipSuccess; ++lg)
      scr_dispatch(lg, [&](auto L) {  // columns and twiddles, or a 4096-point row and its
                                      // twiddles, hold more than the default 64 KB of LDS
        lds_err = hipFuncSetAttribute((const void*)screen_cols_kernel<decltype(L)::value>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (lds_err == hipSuccess)
          lds_err = hipFuncSetAttribute((const void*)screen_rows_kernel<decltype(L)::value>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      });
  });
  if (lds_err != hipSuccess) return scr_fail(WFS_EDEVICE, hipGetErrorString(lds_err));
  hipStream_t st = (hipStream_t)stream;
  ScreenParams p{};
  p.T = reinterpret_cast<float2*>(work);
  p.out = screen;
  p.n = n;
  p.log2n = log2n;
  p.cols = cols;
  p.c_psd = (float)(0.023 * std::pow(r0_m, -5.0 / 3.0));
  p.inv_l02 = std::isfinite(L0_m) ? (float)(1.0 / (L0_m * L0_m)) : 0.0f;
  p.inv_ndx = (float)(1.0 / (n * pitch_m));
  p.seed_lo = (uint32_t)seed;
  p.seed_hi = (uint32_t)(seed >> 32);
  p.sid_lo = (uint32_t)stream_id;
  p.sid_hi = (uint32_t)(stream_id >> 32);
  const size_t row_lds = ((size_t)fft_span(n) + n - 1) * sizeof(float2);
  scr_dispatch(log2n, [&](auto L) {
    screen_rows_kernel<decltype(L)::value><<<n, kScrBlock, row_lds, st>>>(p);
  });
  if ((e = hipGetLastError()) != hipSuccess) return scr_fail(WFS_EDEVICE, hipGetErrorString(e));
  const size_t lds = ((size_t)cols * fft_pitch(n, cols) + n - 1) * sizeof(float2);
  scr_dispatch(log2n, [&](auto L) {
    screen_cols_kernel<decltype(L)::value><<<n / cols, kScrColBlock, lds, st>>>(p);
  });
  if ((e = hipGetLastError()) != hipSuccess) return scr_fail(WFS_EDEVICE, hipGetErrorString(e));
  return WFS_OK;
}

}  // extern "C"
