// Forward Shack-Hartmann sensor kernels for gfx950 (CDNA4).
//
// One launch serves every sensor of a plan for every realisation at one time step:
//   blocks [0, fft_blocks)   : FFT path, one subaperture per 256-thread workgroup (large fields)
//   blocks [fft_blocks, ...) : lag-domain path, one subaperture per 64-lane wavefront at a time
//
// The lag-domain path (wfs_otf.h) forms each binned spot from the field autocorrelation; the
// FFT path (wfs_fft.h) from zero-padded transforms.  Both end in the same noise + centre of
// gravity stage.

#include "wfs_otf.h"
#include "wfs_fft.h"

namespace wfs {

// ------------------------------------------------------------------------------------------
// The launch
// ------------------------------------------------------------------------------------------

template <int NS>
__global__ __launch_bounds__(kBlock) void wfs_forward_kernel(FwdParams p) {
  extern __shared__ __align__(16) char smem[];
  const int64_t step = current_step(p);
  const int i = blockIdx.x;
  if (i < p.fft_blocks) {
    fft_subap(p, i, step, smem);
    return;
  }
  const int n = gridDim.x - p.fft_blocks;
  const int ib = i - p.fft_blocks;
  const int L = p.xcd_remap ? xcd_logical_block(ib, n) : ib;
  const int wave = threadIdx.x >> 6;
  char* wsm = smem + wave * p.lds_per_wave;
  const int total = p.otf.per_real * p.batch;
  const int t0 = (L * kWavesPerBlock + wave) * p.subaps_per_wave;
  for (int k = 0; k < p.subaps_per_wave; ++k) {
    const int t = t0 + k;
    if (t >= total) break;
    otf_subap<NS>(p, t, step, wsm);
  }
}

// wfs_project: phase (radians at the sensor wavelength) of every pixel of every valid
// subaperture; thread per pixel.
__global__ __launch_bounds__(kBlock) void wfs_project_kernel(FwdParams p, float* phase,
                                                              int64_t per_real) {
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t total = per_real * p.batch;
  if (gid >= total) return;
  const int b = (int)(gid / per_real);
  int64_t r = gid - (int64_t)b * per_real;
  int sid = 0;
  while (sid + 1 < p.n_sensors && r >= p.sen[sid + 1].phase_off) ++sid;
  const DevSensor S = p.sen[sid];
  r -= S.phase_off;
  const int ns = S.n_sub;
  const int v = (int)(r / (ns * ns));
  const int q = (int)(r - (int64_t)v * ns * ns);
  const DevSubap sb = p.sub[S.valid_off + v];
  const int ir = sb.a * ns + q / ns, ic = sb.b * ns + q % ns;
  const double stepd = (double)current_step(p);
  const float* lay_b = p.layers + (int64_t)b * p.layer_stride;
  float psi = 0.0f;
  for (int l = 0; l < p.n_layers; ++l) {
    const Tap cx = col_tap(p, sid, l, ic, stepd);
    const Tap ry = row_tap(p, sid, l, ir, stepd);
    psi = fmaf(p.lay[l].weight, bilinear(lay_b + p.lay[l].offset, cx, ry), psi);
  }
  phase[gid] = psi * S.kappa;
}

__global__ void wfs_step_kernel(int64_t* step_dev, int64_t value, int32_t add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step_dev = add ? *step_dev + value : value;
}

// ------------------------------------------------------------------------------------------
// Host-side launchers (called from wfs_host.cpp)
// ------------------------------------------------------------------------------------------

template <int NS>
static hipError_t launch_fwd(const FwdParams& p, hipStream_t st) {
  const int grid = p.fft_blocks + p.otf_blocks;
  if (grid == 0) return hipSuccess;
  const int lds = p.lds_per_wave * kWavesPerBlock;
  hipLaunchKernelGGL(wfs_forward_kernel<NS>, dim3(grid), dim3(kBlock), lds, st, p);
  return hipGetLastError();
}

hipError_t launch_forward(const FwdParams& p, int ns, hipStream_t st) {
  switch (ns) {
    case 2: return launch_fwd<2>(p, st);
    case 3: return launch_fwd<3>(p, st);
    case 4: return launch_fwd<4>(p, st);
    case 5: return launch_fwd<5>(p, st);
    case 6: return launch_fwd<6>(p, st);
    case 7: return launch_fwd<7>(p, st);
    case 8: return launch_fwd<8>(p, st);
    case 9: return launch_fwd<9>(p, st);
    case 10: return launch_fwd<10>(p, st);
    case 11: return launch_fwd<11>(p, st);
    case 12: return launch_fwd<12>(p, st);
    default: return hipErrorInvalidValue;
  }
}

int otf_lds_bytes(int ns, int n_layers, int n_pix) {
  return otf_lds_layout(ns, n_layers, n_pix).total;
}

hipError_t launch_project(const FwdParams& p, float* phase, int64_t per_real, hipStream_t st) {
  const int64_t total = per_real * p.batch;
  if (total == 0) return hipSuccess;
  const int grid = (int)((total + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(wfs_project_kernel, dim3(grid), dim3(kBlock), 0, st, p, phase, per_real);
  return hipGetLastError();
}

hipError_t launch_step(int64_t* step_dev, int64_t value, int add, hipStream_t st) {
  hipLaunchKernelGGL(wfs_step_kernel, dim3(1), dim3(64), 0, st, step_dev, value, add);
  return hipGetLastError();
}

}  // namespace wfs

namespace wfs {
bool fft_supported(int n_sub, int n_fft, int bin) { return fft_supported_impl(n_sub, n_fft, bin); }
int fft_lds_bytes(int n_sub, int n_fft, int n_pix) { return fft_lds_bytes_impl(n_sub, n_fft, n_pix); }
}  // namespace wfs
