// Device helpers shared by the sensor kernels: wave synchronisation, block ordering,
// Philox4x32-10, layer-coordinate taps and the fused layer projection.
#pragma once

#include "wfs_internal.h"

namespace wfs {

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Order LDS traffic inside one wavefront (the wave is the only reader/writer of its region).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Workgroups are dispatched round-robin over the 8 XCDs (block i on XCD i % 8).  Renumber so
// that consecutive logical blocks share an XCD and therefore its L2: XCD x owns the logical
// range [x*q + min(x, r), ...) of n = 8q + r blocks.
__device__ __forceinline__ int xcd_logical_block(int i, int n) {
  const int x = i & 7, q = n >> 3, r = n & 7;
  return x * q + (x < r ? x : r) + (i >> 3);
}

// Read-only tables are read through the constant address space so that wave-uniform
// indices become scalar (SMEM) loads.
template <class T>
__device__ __forceinline__ T cload(const T* p, int64_t i) {
  static_assert(sizeof(T) % 4 == 0, "table rows are whole 32-bit words");
  typedef const __attribute__((address_space(4))) uint32_t* wptr;
  const wptr src = (wptr)(p + i);
  T out;
  uint32_t* o = reinterpret_cast<uint32_t*>(&out);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) o[k] = src[k];
  return out;
}

// Sum over the wavefront, returned to every lane: butterflies inside each row of 16 lanes
// with DPP (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror), then the
// four row totals.  No LDS traffic.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x141>(v);
  v += dpp_mov<0x140>(v);
  const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 0));
  const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16));
  const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
  const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 48));
  return (r0 + r1) + (r2 + r3);
}

// Philox4x32-10 (Salmon et al., SC'11): 10 rounds of two 32x32->64 multiplications with the
// published multipliers, Weyl key schedule between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;  // one 32x32->64 multiply each
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
                   (uint32_t)p0);
  }
  return c;
}

// sin(2 pi x) and cos(2 pi x) for x in revolutions (|x| small): the hardware transcendental
// unit (v_sin_f32 / v_cos_f32) takes its argument in revolutions.
__device__ __forceinline__ void sincos_rev(float x, float* s, float* c) {
  *s = __builtin_amdgcn_sinf(x);
  *c = __builtin_amdgcn_cosf(x);
}

// floor(q / d) for 0 <= q < 2^22, d >= 1, given inv_d = 1/d rounded: the float quotient is off
// by at most one, fixed by one compare.
__device__ __forceinline__ int fdiv(int q, int d, float inv_d) {
  int r = (int)((float)q * inv_d);
  const int m = r * d;
  r += (m > q) ? -1 : ((m + d <= q) ? 1 : 0);
  return r;
}

// Uniform in (0,1) from the top 24 bits of a word: ((w >> 8) + 1/2) 2^-24 (exact in fp32).
__device__ __forceinline__ float u24(uint32_t w) {
  return (float)(w >> 8) * 5.9604644775390625e-08f + 2.98023223876953125e-08f;
}

// Gaussian photon + read noise of two pixels from one Philox block (Box-Muller pairs
// (u0,u1) and (u2,u3)): b' = b + sqrt(max(b,0)) z1 + ro z2.
__device__ __forceinline__ void add_noise_pair(float& b0, float& b1, uint4 w, float ro) {
  // -2 ln u = -2 ln2 log2 u ; angles 2 pi u in revolutions
  const float ra = sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u24(w.x)));
  const float rb = sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u24(w.z)));
  float s0, c0, s1, c1;
  sincos_rev(u24(w.y), &s0, &c0);
  sincos_rev(u24(w.w), &s1, &c1);
  b0 += sqrtf(fmaxf(b0, 0.0f)) * (ra * c0) + ro * (ra * s0);
  b1 += sqrtf(fmaxf(b1, 0.0f)) * (rb * c1) + ro * (rb * s1);
}

// The same noise for one pixel from its half of a Philox block (wr: radius word, wa: angle
// word), with the hardware square root (about 1 ulp; the noise needs no more).
__device__ __forceinline__ void add_noise_one(float& b, uint32_t wr, uint32_t wa, float ro) {
  const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u24(wr)));
  float s, c;
  sincos_rev(u24(wa), &s, &c);
  b += __builtin_amdgcn_sqrtf(fmaxf(b, 0.0f)) * (r * c) + ro * (r * s);
}

// One axis of a bilinear stencil: element indices (row offsets for the y axis) and weights.
// Periodic layers wrap modulo n; zero-boundary grids give weight 0 to taps off the grid.
struct Tap {
  int32_t i0, i1;
  float w0, w1;
};

__device__ __forceinline__ Tap make_tap(double c, int32_t n, double inv_n, int32_t boundary,
                                        int32_t scale) {
  Tap t;
  if (boundary == 0) {
    double cw = c - (double)n * floor(c * inv_n);  // in [0, n] up to rounding
    const double f0 = floor(cw);
    int32_t i0 = (int32_t)f0;
    const float f = (float)(cw - f0);
    if (i0 >= n) i0 -= n;
    if (i0 < 0) i0 += n;
    int32_t i1 = i0 + 1;
    if (i1 >= n) i1 -= n;
    t.i0 = i0 * scale;
    t.i1 = i1 * scale;
    t.w0 = 1.0f - f;
    t.w1 = f;
  } else {
    const double cc = fmin(fmax(c, -4.0), (double)n + 4.0);
    const double f0 = floor(cc);
    const int32_t i0 = (int32_t)f0;
    const float f = (float)(cc - f0);
    const bool ok0 = i0 >= 0 && i0 < n;
    const bool ok1 = i0 + 1 >= 0 && i0 + 1 < n;
    // a tap off the grid has weight 0 and reads the nearest grid element (any finite value
    // would do; the nearest one is what a footprint staged with clamped indices holds)
    t.i0 = min(max(i0, 0), n - 1) * scale;
    t.i1 = min(max(i0 + 1, 0), n - 1) * scale;
    t.w0 = ok0 ? 1.0f - f : 0.0f;
    t.w1 = ok1 ? f : 0.0f;
  }
  return t;
}

__device__ __forceinline__ Tap col_tap(const FwdParams& p, int s, int l, int ic, double step) {
  const DevLayer L = p.lay[l];
  const DevAffine A = p.aff[s * p.n_layers + l];
  const double u = fma(A.ax, (double)ic, A.bx0) + step * A.dbx;
  return make_tap(u, L.nx, L.inv_nx, L.boundary, 1);
}

__device__ __forceinline__ Tap row_tap(const FwdParams& p, int s, int l, int ir, double step) {
  const DevLayer L = p.lay[l];
  const DevAffine A = p.aff[s * p.n_layers + l];
  const double v = fma(A.ay, (double)ir, A.by0) + step * A.dby;
  return make_tap(v, L.ny, L.inv_ny, L.boundary, L.nx);
}

// Load base[idx] with a wave-uniform base and a 32-bit element index: lets the compiler use
// the scalar-base + 32-bit-offset addressing mode instead of per-lane 64-bit addresses.
__device__ __forceinline__ float ld_idx(const float* base, uint32_t idx) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + (idx << 2));
}

__device__ __forceinline__ float bilinear(const float* __restrict__ g, const Tap& cx,
                                          const Tap& ry) {
  const float v00 = g[ry.i0 + cx.i0], v01 = g[ry.i0 + cx.i1];
  const float v10 = g[ry.i1 + cx.i0], v11 = g[ry.i1 + cx.i1];
  return ry.w0 * fmaf(cx.w0, v00, cx.w1 * v01) + ry.w1 * fmaf(cx.w0, v10, cx.w1 * v11);
}

// Task t of a task table -> (realisation, sensor id, valid-subaperture index).
__device__ __forceinline__ void task_of(const TaskTable& tt, int t, int& b, int& sid, int& v) {
  b = t / tt.per_real;
  int r = t - b * tt.per_real;
  if (tt.order) {
    const int2 e = cload(tt.order, r);
    sid = e.x;
    v = e.y;
    return;
  }
  int k = 0;
  while (k + 1 < tt.n && r >= tt.start[k + 1]) ++k;
  sid = tt.ids[k];
  v = r - tt.start[k];
}

// Time step of a launch: p.step, or the device counter plus p.step (graph replays).
__device__ __forceinline__ int64_t current_step(const FwdParams& p) {
  return p.use_dev_step ? *p.step_dev + p.step : p.step;
}

}  // namespace wfs
