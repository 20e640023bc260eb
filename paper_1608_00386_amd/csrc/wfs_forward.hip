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

// Projection (Sec. 2.2), also the first kernel of the split forward: block = (realisation,
// sensor, group of proj_group consecutive valid subapertures or, for large subapertures, a
// chunk of proj_rows of their rows; ~512 pixels).  The stencil taps of the block's pupil
// columns and rows for every layer (FP64 coordinates) go to LDS once, then every thread
// gathers its pixels with the loads of eight layers in flight.  Output: kappa * psi of every
// pixel of every valid subaperture, subaperture-major (the spot kernels' input layout).
__global__ __launch_bounds__(kBlock) void wfs_project_kernel(FwdParams p, float* phase) {
  extern __shared__ __align__(16) char smem[];
  const int i = p.xcd_remap ? xcd_logical_block(blockIdx.x, gridDim.x) : blockIdx.x;
  int b, sid, task;
  task_of(p.proj, i, b, sid, task);
  const DevSensor S = cload(p.sen, sid);
  const int ns = S.n_sub, n2 = ns * ns, G = S.proj_group, R = S.proj_rows;
  const int chunks = (ns + R - 1) / R;
  const int g = task / chunks, rc = task - g * chunks;
  const int r0 = rc * R, nr = min(R, ns - r0);  // rows [r0, r0 + nr) of each subaperture
  const int v0 = g * G;
  const int nv = min(G, S.n_valid - v0);
  const int nl = p.n_layers, nt = ns + nr;      // taps per (subaperture, layer): cols + rows
  DevLayer* lay = reinterpret_cast<DevLayer*>(smem);
  DevAffine* aff = reinterpret_cast<DevAffine*>(smem + kMaxLayers * sizeof(DevLayer));
  Tap* taps = reinterpret_cast<Tap*>(smem + kMaxLayers * (sizeof(DevLayer) + sizeof(DevAffine)));
  for (int l = threadIdx.x; l < nl; l += kBlock) {
    lay[l] = p.lay[l];
    aff[l] = p.aff[sid * nl + l];
  }
  __syncthreads();
  const double stepd = (double)current_step(p);
  const int nvt = nv * nt;
  const float inv_nvt = 1.0f / (float)nvt, inv_nt = 1.0f / (float)nt;
  for (int t = threadIdx.x; t < nl * nvt; t += kBlock) {
    const int l = fdiv(t, nvt, inv_nvt);
    const int rem = t - l * nvt;
    const int gi = fdiv(rem, nt, inv_nt), k = rem - gi * nt;
    const DevSubap sb = p.sub[S.valid_off + v0 + gi];
    const DevLayer& L = lay[l];
    const DevAffine& A = aff[l];
    Tap tp;
    if (k < ns) {
      const double u = fma(A.ax, (double)(sb.b * ns + k), A.bx0) + stepd * A.dbx;
      tp = make_tap(u, L.nx, L.inv_nx, L.boundary, 1);
    } else {
      const double v = fma(A.ay, (double)(sb.a * ns + r0 + k - ns), A.by0) + stepd * A.dby;
      tp = make_tap(v, L.ny, L.inv_ny, L.boundary, L.nx);
    }
    taps[(gi * nl + l) * nt + k] = tp;
  }
  __syncthreads();
  const float* lay_b = p.layers + (int64_t)b * p.layer_stride;
  float* out = phase + (int64_t)b * p.phase_per_real + S.phase_off + (int64_t)v0 * n2 + r0 * ns;
  const int npx = nr * ns;  // pixels per subaperture in this block
  const float inv_npx = 1.0f / (float)npx, inv_ns = 1.0f / (float)ns;
  for (int px = threadIdx.x; px < nv * npx; px += kBlock) {
    const int gi = fdiv(px, npx, inv_npx);
    const int q = px - gi * npx;
    const int r = fdiv(q, ns, inv_ns), c = q - r * ns;  // row r within the chunk
    const Tap* tg = taps + gi * nl * nt;
    float psi = 0.0f;
    constexpr int LC = 8;
    for (int l0 = 0; l0 < nl; l0 += LC) {
      float v[LC][4], wx0[LC], wx1[LC], wy0[LC], wy1[LC];
#pragma unroll
      for (int jj = 0; jj < LC; ++jj) {
        const int l = l0 + jj;
        if (l < nl) {
          const DevLayer L = cload(p.lay, l);  // wave-uniform: scalar base address
          const float* gl = lay_b + L.offset;
          const Tap cx = tg[l * nt + c];
          const Tap ry = tg[l * nt + ns + r];
          v[jj][0] = ld_idx(gl, (uint32_t)(ry.i0 + cx.i0));
          v[jj][1] = ld_idx(gl, (uint32_t)(ry.i0 + cx.i1));
          v[jj][2] = ld_idx(gl, (uint32_t)(ry.i1 + cx.i0));
          v[jj][3] = ld_idx(gl, (uint32_t)(ry.i1 + cx.i1));
          wx0[jj] = cx.w0;
          wx1[jj] = cx.w1;
          wy0[jj] = ry.w0 * L.weight;
          wy1[jj] = ry.w1 * L.weight;
        }
      }
#pragma unroll
      for (int jj = 0; jj < LC; ++jj) {
        if (l0 + jj < nl) {
          psi = fmaf(wy0[jj], fmaf(wx0[jj], v[jj][0], wx1[jj] * v[jj][1]), psi);
          psi = fmaf(wy1[jj], fmaf(wx0[jj], v[jj][2], wx1[jj] * v[jj][3]), psi);
        }
      }
    }
    out[(int64_t)gi * n2 + q] = psi * S.kappa;
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

int project_lds_bytes(int n_sub, int n_layers, int group, int rows) {
  return kMaxLayers * (int)(sizeof(DevLayer) + sizeof(DevAffine)) +
         group * n_layers * (n_sub + rows) * (int)sizeof(Tap);
}

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
