// Forward Shack-Hartmann sensor model for gfx950 (CDNA4): the projection kernel, the device
// step counter and the host-side launchers.  The spot kernels (wfs_forward_kernels.h) are
// instantiated per subaperture size in the wfs_fwd_ns*.hip units, which compile in parallel.
//
// The lag-domain path (wfs_otf.h) forms each binned spot from the field autocorrelation; the
// FFT path (wfs_fft.h) from zero-padded transforms.  Both end in the same noise + centre of
// gravity stage.

#include "wfs_fft.h"
#include "wfs_otf.h"
#include "wfs_project.h"

namespace wfs {

__global__ __launch_bounds__(kBlock) void wfs_project_kernel(FwdParams p, float* phase) {
  extern __shared__ __align__(16) char smem[];
  const int blk = p.xcd_remap ? xcd_logical_block(blockIdx.x, gridDim.x) : blockIdx.x;
  project_block(p, blk, phase, (double)current_step(p), smem);
}

// Stencil entries of the staged footprint for the frames of one launch: block per (frame,
// sensor, layer, axis), thread per pupil index; frame f is at step current_step + f.  The
// window of a subaperture starts at the first tap of its pupil index of smallest coordinate,
// so each entry's offset in that window is known here (same arithmetic as the projection).
__global__ __launch_bounds__(kBlock) void wfs_foot_entries_kernel(FwdParams p, FootEnt* out) {
  const int per_frame = p.n_sensors * p.n_layers * 2;
  const int f = blockIdx.x / per_frame;
  const int r = blockIdx.x - f * per_frame;  // (sensor * n_layers + layer) * 2 + axis
  const DevSensor S = cload(p.sen, r / (2 * p.n_layers));
  if (S.foot_ncols == 0) return;  // no staged footprint (FFT-path sensor)
  const FootAxis X = p.foot_axis[r];
  const double stepd = (double)(current_step(p) + f);
  FootEnt* e = out + (int64_t)f * p.foot_ent_per_frame + X.ent_off;
  const int ns = S.n_sub;
  for (int i = threadIdx.x; i < S.n_pup; i += kBlock) {
    int i0, o;
    const double c = fma(X.a, (double)i, X.b0) + stepd * X.db;
    const float2 w = foot_axis_tap(c, X.n, X.inv_n, X.boundary, &i0);
    const int first = (i / ns) * ns;
    const int io = X.a >= 0.0 ? first : first + ns - 1;  // the window origin's pupil index
    (void)foot_axis_tap(fma(X.a, (double)io, X.b0) + stepd * X.db, X.n, X.inv_n, X.boundary,
                        &o);
    int rel = i0 - o;
    if (X.boundary == 0 && rel < 0) rel += X.n;
    e[i] = FootEnt{w.x * X.weight, w.y * X.weight, (X.koff + rel * X.kmul) * 4, i0};
  }
}

__global__ void wfs_step_kernel(int64_t* step_dev, int64_t value, int32_t add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step_dev = add ? *step_dev + value : value;
}

// ------------------------------------------------------------------------------------------
// Host-side launchers (called from wfs_host.cpp)
// ------------------------------------------------------------------------------------------

// spot kernels, instantiated per subaperture size in the wfs_fwd_ns*.hip units
template <int NS>
hipError_t launch_fwd_ns(const FwdParams& p, hipStream_t st);

static hipError_t launch_forward_ns(const FwdParams& p, int ns, hipStream_t st) {
  switch (ns) {
    case 2: return launch_fwd_ns<2>(p, st);
    case 3: return launch_fwd_ns<3>(p, st);
    case 4: return launch_fwd_ns<4>(p, st);
    case 5: return launch_fwd_ns<5>(p, st);
    case 6: return launch_fwd_ns<6>(p, st);
    case 7: return launch_fwd_ns<7>(p, st);
    case 8: return launch_fwd_ns<8>(p, st);
    case 9: return launch_fwd_ns<9>(p, st);
    case 10: return launch_fwd_ns<10>(p, st);
    case 11: return launch_fwd_ns<11>(p, st);
    case 12: return launch_fwd_ns<12>(p, st);
    default: return hipErrorInvalidValue;
  }
}

// FFT-path and lag-domain subapertures: by default in two launches, since the FFT path's
// registers and LDS would otherwise set the occupancy of every lag-domain wavefront.  The
// FFT-path blocks (large fields, one workgroup each, 48 KB of LDS) and the lag-domain blocks
// go to separate launches, so that the lag-domain waves keep their own occupancy; with a side
// stream the FFT-path launch runs concurrently (fork after everything already queued on st,
// join before anything queued after this call).  With fft_inline they share one launch.
hipError_t launch_forward(const FwdParams& p, int ns, hipStream_t st, const SideStream* side) {
  if (p.fft_inline || p.fft_blocks == 0 || (p.otf_blocks == 0 && p.proj_blocks == 0))
    return launch_forward_ns(p, ns, st);
  FwdParams a = p;
  a.otf_blocks = 0;
  a.proj_blocks = 0;
  FwdParams c = p;
  c.fft_blocks = 0;
  c.lds_per_wave = p.lds_per_wave_otf;
  hipError_t e;
  if (side && side->stream) {
    e = hipEventRecord(side->fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(side->stream, side->fork, 0);
    if (e == hipSuccess) e = launch_forward_ns(a, ns, side->stream);
    if (e == hipSuccess) e = launch_forward_ns(c, ns, st);
    if (e == hipSuccess) e = hipEventRecord(side->join, side->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, side->join, 0);
    return e;
  }
  e = launch_forward_ns(a, ns, st);
  if (e != hipSuccess) return e;
  return launch_forward_ns(c, ns, st);
}

int foot_pitch(int ns) { return otf_pitch(ns + 2); }

int otf_lds_bytes(int ns, int n_layers, int n_pix, bool with_taps, int foot_floats,
                  int lag_parts) {
  return otf_lds_layout(ns, n_layers, n_pix, with_taps, foot_floats, lag_parts).total;
}

int project_lds_bytes(int n_layers, int rows) {
  return n_layers * (kProjStrip + rows) * (int)sizeof(Tap);
}

int project_max_groups() { return kProjMaxGroups; }

int project_strip() { return kProjStrip; }
int project_rows() { return kProjRows; }

hipError_t launch_project(const FwdParams& p, float* phase, int lds, hipStream_t st) {
  const int64_t blocks = (int64_t)p.proj_per_real * p.batch;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(wfs_project_kernel, dim3((unsigned)blocks), dim3(kBlock), lds, st, p, phase);
  return hipGetLastError();
}

hipError_t launch_foot_entries(const FwdParams& p, FootEnt* out, int n_frames,
                               hipStream_t st) {
  const int64_t blocks = (int64_t)n_frames * p.n_sensors * p.n_layers * 2;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(wfs_foot_entries_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, p,
                     out);
  return hipGetLastError();
}

hipError_t launch_step(int64_t* step_dev, int64_t value, int add, hipStream_t st) {
  hipLaunchKernelGGL(wfs_step_kernel, dim3(1), dim3(64), 0, st, step_dev, value, add);
  return hipGetLastError();
}

}  // namespace wfs

namespace wfs {
bool fft_supported(int n_sub, int n_fft, int bin) { return fft_supported_impl(n_sub, n_fft, bin); }
int fft_wave_lds_bytes(int n_fft, int n_pix) { return fft_wave_lds_bytes_impl(n_fft, n_pix); }
}  // namespace wfs
