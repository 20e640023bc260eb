// Projection of the layers onto the pupil pixels of valid subapertures (Sec. 2.2): one block
// of the projection kernel, also run inside the pipelined spot launch.
#pragma once

#include "wfs_common.h"

namespace wfs {

// Projection (Sec. 2.2), also the first kernel of the split forward.  Block = (realisation,
// sensor, kProjRows consecutive pupil rows, strip of kProjStrip pupil columns); thread = one
// pupil pixel.  The column taps of the strip and the row taps of the rows (FP64 coordinates)
// go to LDS once per block; each thread then has the stencil loads of up to kProjLC layers in
// flight at once (one memory round trip for up to kProjLC layers), consecutive threads reading
// consecutive layer pixels.  Output: the phase at the sensor wavelength of every pixel of every
// valid subaperture, subaperture-major (the spot kernels' layout).
constexpr int kProjStrip = 64;
constexpr int kProjRows = kBlock / kProjStrip;
constexpr int kProjLC = 10;

__device__ __forceinline__ void project_block(const FwdParams& p, int blk, float* phase, double stepd,
                              char* smem) {
  int b, sid, task;
  task_of(p.proj, blk, b, sid, task);
  const DevSensor S = cload(p.sen, sid);
  const int packed = cload(p.proj_tasks, (int64_t)S.ptask_off + task);  // row0 | strip << 16
  const int row0 = packed & 0xFFFF, c0 = (packed >> 16) * kProjStrip;
  const int ns = S.n_sub, n2 = ns * ns;
  const int nl = p.n_layers;
  Tap* ctap = reinterpret_cast<Tap*>(smem);   // [nl][kProjStrip]
  Tap* rtap = ctap + nl * kProjStrip;         // [nl][kProjRows]
  const int tx = threadIdx.x & (kProjStrip - 1);
  const int ty = __builtin_amdgcn_readfirstlane(threadIdx.x / kProjStrip);  // wave index
  const int ic = c0 + tx, ir = row0 + ty;
  int vsub = -1, a = 0, bs = 0;
  if (ic < S.n_pup && ir < S.n_pup) {  // issued first: in flight while the taps are computed
    a = ir / ns;
    bs = ic / ns;
    vsub = p.subidx[(int64_t)S.subidx_off + a * S.n_sa + bs];
  }
  // taps: wave w serves layers w, w + kProjRows, ...: one column tap per lane and the row
  // taps of the block's rows on the first lanes (layer tables through the scalar cache)
  for (int l = ty; l < nl; l += kProjRows) {
    const DevLayer L = cload(p.lay, l);
    const DevAffine A = cload(p.aff, (int64_t)sid * nl + l);
    const double u = fma(A.ax, (double)ic, A.bx0) + stepd * A.dbx;
    ctap[l * kProjStrip + tx] = make_tap(u, L.nx, L.inv_nx, L.boundary, 1);
    if (tx < kProjRows) {
      const double v = fma(A.ay, (double)(row0 + tx), A.by0) + stepd * A.dby;
      rtap[l * kProjRows + tx] = make_tap(v, L.ny, L.inv_ny, L.boundary, L.nx);
    }
  }
  __syncthreads();
  if (vsub < 0) return;  // outside the pupil grid or in an unused subaperture
  const float* lay_b = p.layers + (int64_t)b * p.layer_stride;
  float psi = 0.0f;
  for (int l0 = 0; l0 < nl; l0 += kProjLC) {
    // layers past the end repeat the last one with weight 0 (same addresses: cache hits)
    float v[kProjLC][4];
#pragma unroll
    for (int jj = 0; jj < kProjLC; ++jj) {
      const int l = min(l0 + jj, nl - 1);
      const float* gl = lay_b + cload(p.lay, l).offset;  // wave-uniform: scalar base address
      const Tap cx = ctap[l * kProjStrip + tx];
      const Tap ry = rtap[l * kProjRows + ty];
      v[jj][0] = ld_idx(gl, (uint32_t)(ry.i0 + cx.i0));
      v[jj][1] = ld_idx(gl, (uint32_t)(ry.i0 + cx.i1));
      v[jj][2] = ld_idx(gl, (uint32_t)(ry.i1 + cx.i0));
      v[jj][3] = ld_idx(gl, (uint32_t)(ry.i1 + cx.i1));
    }
    // all loads of the chunk are issued; the weights are read again from LDS so that they
    // do not hold registers while the loads are in flight
    asm volatile("" ::: "memory");
#pragma unroll
    for (int jj = 0; jj < kProjLC; ++jj) {
      const int l = min(l0 + jj, nl - 1);
      const float wl = l0 + jj < nl ? cload(p.lay, l).weight : 0.0f;
      const Tap cx = ctap[l * kProjStrip + tx];
      const Tap ry = rtap[l * kProjRows + ty];
      const float r0v = fmaf(cx.w0, v[jj][0], cx.w1 * v[jj][1]);
      const float r1v = fmaf(cx.w0, v[jj][2], cx.w1 * v[jj][3]);
      psi = fmaf(ry.w0 * wl, r0v, fmaf(ry.w1 * wl, r1v, psi));
    }
    if (l0 + kProjLC >= nl) break;
  }
  phase[(int64_t)b * p.phase_per_real + S.phase_off + (int64_t)vsub * n2 + (ir - a * ns) * ns +
        (ic - bs * ns)] = psi * S.kappa;
}

}  // namespace wfs
