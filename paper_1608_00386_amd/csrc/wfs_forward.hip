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

// Projection (Sec. 2.2), also the first kernel of the split forward.  Coalesced column
// strips: block = (realisation, sensor, subaperture row a, chunk of proj_rows pixel rows,
// strip of kProjStrip pupil columns); thread = one pupil column and every kProjRowGroups-th
// row.  The column taps of the strip and the row taps of the chunk (FP64 coordinates) go to
// LDS once per block; then for each of its rows a thread issues the four stencil loads of
// five layers at once — consecutive threads read consecutive layer pixels.  Output: kappa*psi
// of every pixel of every valid subaperture, subaperture-major (the spot kernels' layout).
constexpr int kProjStrip = 64;
constexpr int kProjRowGroups = kBlock / kProjStrip;

__global__ __launch_bounds__(kBlock) void wfs_project_kernel(FwdParams p, float* phase) {
  extern __shared__ __align__(16) char smem[];
  const int blk = p.xcd_remap ? xcd_logical_block(blockIdx.x, gridDim.x) : blockIdx.x;
  int b, sid, task;
  task_of(p.proj, blk, b, sid, task);
  const DevSensor S = cload(p.sen, sid);
  const int packed = cload(p.proj_tasks, (int64_t)S.ptask_off + task);  // a | rc<<12 | strip<<20
  const int a = packed & 0xFFF, rc = (packed >> 12) & 0xFF, strip = packed >> 20;
  const int ns = S.n_sub, n2 = ns * ns, R = S.proj_rows;
  const int r0 = rc * R, nr = min(R, ns - r0);
  const int c0 = strip * kProjStrip;
  const int nl = p.n_layers;
  Tap* ctap = reinterpret_cast<Tap*>(smem);   // [nl][kProjStrip]
  Tap* rtap = ctap + nl * kProjStrip;         // [nl][R]
  const double stepd = (double)current_step(p);
  const int tx = threadIdx.x & (kProjStrip - 1), tg = threadIdx.x / kProjStrip;
  for (int l = tg; l < nl; l += kProjRowGroups) {  // column taps: one per thread per layer
    const DevLayer L = p.lay[l];
    const DevAffine A = p.aff[sid * nl + l];
    const double u = fma(A.ax, (double)(c0 + tx), A.bx0) + stepd * A.dbx;
    ctap[l * kProjStrip + tx] = make_tap(u, L.nx, L.inv_nx, L.boundary, 1);
  }
  for (int t = threadIdx.x; t < nl * nr; t += kBlock) {  // row taps of the chunk
    const int l = t / nr, r = t - l * nr;
    const DevLayer L = p.lay[l];
    const DevAffine A = p.aff[sid * nl + l];
    const double v = fma(A.ay, (double)(a * ns + r0 + r), A.by0) + stepd * A.dby;
    rtap[l * R + r] = make_tap(v, L.ny, L.inv_ny, L.boundary, L.nx);
  }
  __syncthreads();
  const int ic = c0 + tx;
  if (ic >= S.n_pup) return;
  const int bs = ic / ns, cx_in = ic - bs * ns;
  const int vsub = cload(p.subidx, (int64_t)S.subidx_off + a * S.n_sa + bs);
  if (vsub < 0) return;  // column of an unused subaperture
  const float* lay_b = p.layers + (int64_t)b * p.layer_stride;
  float* out = phase + (int64_t)b * p.phase_per_real + S.phase_off + (int64_t)vsub * n2 + cx_in;
  for (int r = tg; r < nr; r += kProjRowGroups) {
    float psi = 0.0f;
    constexpr int LC = 5;  // layers past the end repeat the last one with weight 0
    for (int l0 = 0; l0 < nl; l0 += LC) {
      float v[LC][4], wx0[LC], wx1[LC], wy0[LC], wy1[LC];
#pragma unroll
      for (int jj = 0; jj < LC; ++jj) {
        const int l = min(l0 + jj, nl - 1);
        const DevLayer L = cload(p.lay, l);  // wave-uniform: scalar base address
        const float wl = l0 + jj < nl ? L.weight : 0.0f;
        const float* gl = lay_b + L.offset;
        const Tap cx = ctap[l * kProjStrip + tx];
        const Tap ry = rtap[l * R + r];
        v[jj][0] = ld_idx(gl, (uint32_t)(ry.i0 + cx.i0));
        v[jj][1] = ld_idx(gl, (uint32_t)(ry.i0 + cx.i1));
        v[jj][2] = ld_idx(gl, (uint32_t)(ry.i1 + cx.i0));
        v[jj][3] = ld_idx(gl, (uint32_t)(ry.i1 + cx.i1));
        wx0[jj] = cx.w0;
        wx1[jj] = cx.w1;
        wy0[jj] = ry.w0 * wl;
        wy1[jj] = ry.w1 * wl;
      }
#pragma unroll
      for (int jj = 0; jj < LC; ++jj) {
        psi = fmaf(wy0[jj], fmaf(wx0[jj], v[jj][0], wx1[jj] * v[jj][1]), psi);
        psi = fmaf(wy1[jj], fmaf(wx0[jj], v[jj][2], wx1[jj] * v[jj][3]), psi);
      }
    }
    out[(r0 + r) * ns] = psi * S.kappa;
  }
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

int project_lds_bytes(int n_layers, int rows) {
  return n_layers * (kProjStrip + rows) * (int)sizeof(Tap);
}

int project_strip() { return kProjStrip; }

hipError_t launch_project(const FwdParams& p, float* phase, int lds, hipStream_t st) {
  const int64_t blocks = (int64_t)p.proj.per_real * p.batch;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(wfs_project_kernel, dim3((unsigned)blocks), dim3(kBlock), lds, st, p, phase);
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
