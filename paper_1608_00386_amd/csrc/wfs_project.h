// Projection of the layers onto the pupil pixels of valid subapertures (Sec. 2.2): one block
// of the projection kernel, also run inside the pipelined spot launch.
#pragma once

#include "wfs_common.h"

namespace wfs {

// Block = (realisation, sensor, G groups of kProjRows consecutive pupil rows, strip of
// kProjStrip pupil columns) from one two-word descriptor (row0 | strip << 16, sensor |
// log2 G << 24; G is a tile choice of the plan: taller blocks share each column tap among
// more rows, shorter ones fill the chip with more blocks); thread = one pupil column and two
// rows of each group
// (ty and ty + kProjRows / 2, ty = wave).  The column taps of the strip and the row taps of
// the rows (FP64 coordinates, byte offsets) go to LDS once per block; each thread then has
// the stencil loads of both its pixels for kProjLC layers in flight at once, consecutive
// threads reading consecutive layer pixels.  Output: the phase at the sensor wavelength of
// every pixel of every valid subaperture, subaperture-major (the spot kernels' layout).
constexpr int kProjStrip = 64;
constexpr int kProjRows = 2 * kBlock / kProjStrip;
constexpr int kProjLC = 5;
constexpr int kProjMaxGroups = 4;

__device__ __forceinline__ float ld_byte(const float* base, uint32_t off) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + off);
}

// Column taps [nl][kProjStrip] and row taps [nl][rows] of one block into LDS: wave w serves
// layers w, w + 4, ...: one column tap per lane and the row taps on the first lanes (layer
// tables through the scalar cache).
__device__ __forceinline__ void project_taps(const FwdParams& p, int sid, int row0, int rows,
                                             int c0, double stepd, char* smem, const int ty,
                                             const int tx) {
  const int nl = p.n_layers;
  Tap* ctap = reinterpret_cast<Tap*>(smem);  // [nl][kProjStrip], byte offsets
  Tap* rtap = ctap + nl * kProjStrip;        // [nl][rows], byte offsets
  for (int l = ty; l < nl; l += kBlock / kProjStrip) {
    const DevLayer L = cload(p.lay, l);
    const DevAffine A = cload(p.aff, (int64_t)sid * nl + l);
    const double u = fma(A.ax, (double)(c0 + tx), A.bx0) + stepd * A.dbx;
    ctap[l * kProjStrip + tx] = make_tap(u, L.nx, L.inv_nx, L.boundary, 4);
    if (tx < rows) {
      const double v = fma(A.ay, (double)(row0 + tx), A.by0) + stepd * A.dby;
      rtap[l * rows + tx] = make_tap(v, L.ny, L.inv_ny, L.boundary, 4 * L.nx);
    }
  }
  __syncthreads();
}

// Phase sums of the thread's two pixels of row group g (rows ry0 and ry0 + kProjRows / 2 of
// the block's row taps).
__device__ __forceinline__ void project_pixels(const FwdParams& p, int b, int rows, int ry0,
                                               const char* smem, float psi[2], const int tx) {
  const int nl = p.n_layers;
  const Tap* ctap = reinterpret_cast<const Tap*>(smem);
  const Tap* rtap = ctap + nl * kProjStrip;
  const float* lay_b = p.layers + (int64_t)b * p.layer_stride;
  for (int l0 = 0; l0 < nl; l0 += kProjLC) {
    // layers past the end repeat the last one with weight 0 (same addresses: cache hits)
    float v[kProjLC][2][4];
#pragma unroll
    for (int jj = 0; jj < kProjLC; ++jj) {
      const int l = min(l0 + jj, nl - 1);
      const float* gl = lay_b + cload(p.lay, l).offset;  // wave-uniform: scalar base address
      const Tap cx = ctap[l * kProjStrip + tx];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const Tap ry = rtap[l * rows + ry0 + k * (kProjRows / 2)];
        v[jj][k][0] = ld_byte(gl, (uint32_t)(ry.i0 + cx.i0));
        v[jj][k][1] = ld_byte(gl, (uint32_t)(ry.i0 + cx.i1));
        v[jj][k][2] = ld_byte(gl, (uint32_t)(ry.i1 + cx.i0));
        v[jj][k][3] = ld_byte(gl, (uint32_t)(ry.i1 + cx.i1));
      }
    }
    // all loads of the chunk are issued; the weights are read again from LDS so that they
    // do not hold registers while the loads are in flight
    asm volatile("" ::: "memory");
#pragma unroll
    for (int jj = 0; jj < kProjLC; ++jj) {
      const int l = min(l0 + jj, nl - 1);
      const float wl = l0 + jj < nl ? cload(p.lay, l).weight : 0.0f;
      const Tap cx = ctap[l * kProjStrip + tx];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const Tap ry = rtap[l * rows + ry0 + k * (kProjRows / 2)];
        const float r0v = fmaf(cx.w0, v[jj][k][0], cx.w1 * v[jj][k][1]);
        const float r1v = fmaf(cx.w0, v[jj][k][2], cx.w1 * v[jj][k][3]);
        psi[k] = fmaf(ry.w0 * wl, r0v, fmaf(ry.w1 * wl, r1v, psi[k]));
      }
    }
  }
}

__device__ __forceinline__ void project_block(const FwdParams& p, int blk, float* phase,
                                              double stepd, char* smem) {
  const int b = blk / p.proj_per_real;
  const int2 d = cload(p.proj_desc, blk - b * p.proj_per_real);
  const int sid = d.y & 0xFFFFFF;
  const int row0 = d.x & 0xFFFF, c0 = (d.x >> 16) * kProjStrip;
  const int rows = kProjRows << (d.y >> 24);
  const int tx = threadIdx.x & (kProjStrip - 1);
  const int ty = __builtin_amdgcn_readfirstlane(threadIdx.x / kProjStrip);  // wave index
  const DevSensor S = cload(p.sen, sid);
  const int ns = S.n_sub;
  const int ic = c0 + tx;
  const int bs = fdiv(ic, ns, S.inv_nsub);
  project_taps(p, sid, row0, rows, c0, stepd, smem, ty, tx);
  float* out = phase + (int64_t)b * p.phase_per_real + S.phase_off;
  for (int g = 0; g < rows; g += kProjRows) {
    int ir[2], a[2], vsub[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {  // issued first: in flight while the loads are issued
      ir[k] = row0 + g + ty + k * (kProjRows / 2);
      a[k] = fdiv(ir[k], ns, S.inv_nsub);
      vsub[k] = (ic < S.n_pup && ir[k] < S.n_pup)
                    ? p.subidx[(int64_t)S.subidx_off + a[k] * S.n_sa + bs]
                    : -1;
    }
    float psi[2] = {0.0f, 0.0f};
    project_pixels(p, b, rows, g + ty, smem, psi, tx);
#pragma unroll
    for (int k = 0; k < 2; ++k)
      if (vsub[k] >= 0)
        out[(int64_t)vsub[k] * (ns * ns) + (ir[k] - a[k] * ns) * ns + (ic - bs * ns)] =
            psi[k] * S.kappa;
  }
}

}  // namespace wfs
