// recon_apply: reconstructor (control matrix) times slopes, C = alpha R S^T + beta C
// (Sec. 2.6-2.7 of the paper: slopes multiplied by the control matrix give the differential
// coefficients added to the mirror).  R is [M][N] row-major FP32 and is streamed from HBM once
// per call; that stream bounds the operation (4 flop per byte of R at B = 8).
//
//   B == 1, or unaligned operands : split-K streaming GEMV on the vector ALUs
//   2 <= B <= 8, 16-byte aligned   : the same streaming order with every realisation at once
//   (N % 4 == 0)                     (vector ALUs; R read once in 1 KB bursts per row, the
//                                    slopes staged in LDS per workgroup)
//   B > 8, aligned                 : split-K GEMM on the FP32 matrix cores
//                                    (v_mfma_f32_16x16x4f32, one 16-row x 16-realisation tile
//                                    per MFMA, 2 row tiles per wavefront)
// Both write per-split partial sums to a workspace; a second kernel adds the splits in a fixed
// order and applies alpha/beta, so results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/wfs.h"

namespace wfs {

constexpr int kRB = 256;
constexpr int kBatchRW = 8;  // rows per wave of the small-batch kernel
constexpr int kBatchMax = 8;  // realisations of the small-batch kernel
constexpr bool kBatchPF = true;  // small-batch kernel: next slice's rows of R in flight

typedef float v4f __attribute__((ext_vector_type(4)));

// 16-byte streaming load of R (read once per call: non-temporal)
__device__ __forceinline__ float4 ldnt4(const float* p) {
  const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

// ---------------------------------------------------------------------------------------
// GEMV / generic: wave per (RW rows, split); lanes stride over k.
// ---------------------------------------------------------------------------------------
template <int RW, bool VEC>
__global__ __launch_bounds__(kRB) void recon_valu_kernel(const float* __restrict__ R, int M,
                                                         int N, const float* __restrict__ S,
                                                         int b, int chunk, int splits,
                                                         int row_groups, float* __restrict__ ws) {
  const int wave = (blockIdx.x * kRB + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= row_groups * splits) return;
  const int g = wave / splits, sp = wave - g * splits;
  const int row0 = g * RW;
  const int k0 = sp * chunk, k1 = min(N, k0 + chunk);
  const float* s = S + (int64_t)b * N;
  float acc[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) acc[r] = 0.0f;
  if (VEC) {
    // k0 and N are multiples of 4; rows 16-byte aligned; two steps of loads in flight
    int k = k0 + 4 * lane;
    for (; k + 4 * 64 < k1; k += 2 * 4 * 64) {
      const float4 s0 = *reinterpret_cast<const float4*>(s + k);
      const float4 s1 = *reinterpret_cast<const float4*>(s + k + 256);
      float4 r0[RW], r1[RW];
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const int row = min(row0 + r, M - 1);
        r0[r] = ldnt4(R + (int64_t)row * N + k);
        r1[r] = ldnt4(R + (int64_t)row * N + k + 256);
      }
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        acc[r] = fmaf(r0[r].x, s0.x, fmaf(r0[r].y, s0.y, fmaf(r0[r].z, s0.z, fmaf(r0[r].w, s0.w, acc[r]))));
        acc[r] = fmaf(r1[r].x, s1.x, fmaf(r1[r].y, s1.y, fmaf(r1[r].z, s1.z, fmaf(r1[r].w, s1.w, acc[r]))));
      }
    }
    for (; k < k1; k += 4 * 64) {
      const float4 sv = *reinterpret_cast<const float4*>(s + k);
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const int row = min(row0 + r, M - 1);
        const float4 rv = ldnt4(R + (int64_t)row * N + k);
        acc[r] = fmaf(rv.x, sv.x, fmaf(rv.y, sv.y, fmaf(rv.z, sv.z, fmaf(rv.w, sv.w, acc[r]))));
      }
    }
  } else {
    for (int k = k0 + lane; k < k1; k += 64) {
      const float sv = s[k];
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        const int row = min(row0 + r, M - 1);
        acc[r] = fmaf(R[(int64_t)row * N + k], sv, acc[r]);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RW; ++r) {
    float v = acc[r];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    acc[r] = v;
  }
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < RW; ++r)
      if (row0 + r < M) ws[((int64_t)sp * 1 + 0) * M + row0 + r] = acc[r];
  }
}

// ---------------------------------------------------------------------------------------
// Small batch (2 <= B <= 8, aligned), slopes staged in LDS: workgroup = one split (columns
// [k0, k1)) x 4 row groups of 8 rows, one per wave.  The split's columns go by in slices of
// 256: the workgroup stages the slice of every realisation's slopes in LDS (double-buffered,
// the next slice's global loads in flight while this one is used; one barrier a slice), and
// each lane streams the float4 at column k + 4 lane of its wave's 8 rows (1 KB contiguous per
// row and instruction) and forms 8 x B dot products, reduced across the wave at the end.
// Holding the slopes in LDS instead of registers halves the vector-memory instructions and
// frees the registers for a second set of R loads (PF: the next slice's rows are in flight
// while this slice is summed).
// ---------------------------------------------------------------------------------------
template <int BB, bool PF>
__global__ __launch_bounds__(kRB) void recon_batch_lds_kernel(const float* __restrict__ R,
                                                              int M, int N,
                                                              const float* __restrict__ S,
                                                              int B, int chunk, int quads,
                                                              float* __restrict__ ws) {
  constexpr int RW = kBatchRW;
  __shared__ float4 slab[2][BB][64];
  const int wg = blockIdx.x;
  const int sp = wg / quads, q = wg - sp * quads;  // consecutive workgroups: one split
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row0 = (q * 4 + wave) * RW;
  const int k0 = sp * chunk, k1 = min(N, k0 + chunk);
  const int ns = (k1 - k0 + 255) / 256;
  const float* rrow[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) rrow[r] = R + (int64_t)min(row0 + r, M - 1) * N;
  // slope slice loads: thread t stages float4 j = t & 63 of realisations t / 64 and 4 + t / 64
  auto load_s = [&](int s, float4 (&v)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int b = (threadIdx.x >> 6) + 4 * h, k = k0 + 256 * s + 4 * (threadIdx.x & 63);
      v[h] = (b < B && b < BB && k < k1)
                 ? *reinterpret_cast<const float4*>(S + (int64_t)b * N + k)
                 : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto store_s = [&](int buf, const float4 (&v)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int b = (threadIdx.x >> 6) + 4 * h;
      if (b < BB) slab[buf][b][threadIdx.x & 63] = v[h];
    }
  };
  auto load_r = [&](int s, float4 (&v)[RW]) {
    const int k = k0 + 256 * s + 4 * lane;
#pragma unroll
    for (int r = 0; r < RW; ++r) v[r] = k < k1 ? ldnt4(rrow[r] + k) : make_float4(0.f, 0.f, 0.f, 0.f);
  };
  float acc[RW][BB];
#pragma unroll
  for (int r = 0; r < RW; ++r)
#pragma unroll
    for (int b = 0; b < BB; ++b) acc[r][b] = 0.0f;
  float4 sv[2], rv[RW], rn[RW];
  load_s(0, sv);
  if constexpr (PF) load_r(0, rv);
  store_s(0, sv);
  __syncthreads();
  for (int s = 0; s < ns; ++s) {
    const int cur = s & 1;
    if (s + 1 < ns) load_s(s + 1, sv);
    if constexpr (PF) {
      if (s + 1 < ns) load_r(s + 1, rn);
    } else {
      load_r(s, rv);
    }
#pragma unroll
    for (int b = 0; b < BB; ++b) {
      const float4 x = slab[cur][b][lane];
#pragma unroll
      for (int r = 0; r < RW; ++r)
        acc[r][b] = fmaf(rv[r].x, x.x, fmaf(rv[r].y, x.y,
                    fmaf(rv[r].z, x.z, fmaf(rv[r].w, x.w, acc[r][b]))));
    }
    if (s + 1 < ns) store_s(cur ^ 1, sv);
    __syncthreads();
    if constexpr (PF) {
#pragma unroll
      for (int r = 0; r < RW; ++r) rv[r] = rn[r];
    }
  }
#pragma unroll
  for (int r = 0; r < RW; ++r)
#pragma unroll
    for (int b = 0; b < BB; ++b) {
      float v = acc[r][b];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
      acc[r][b] = v;
    }
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
      for (int b = 0; b < BB; ++b)
        if (row0 + r < M && b < B) ws[((int64_t)sp * B + b) * M + row0 + r] = acc[r][b];
  }
}

// ---------------------------------------------------------------------------------------
// MFMA GEMM.  v_mfma_f32_16x16x4f32 operand layout (wave64): lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; the four accumulator registers of lane l hold D[4*(l/16)+i][l%16].
// The K index of one MFMA is only a label shared by A and B, so lane (i, kq) feeds the eight
// consecutive columns k + 8 kq + t (t = 0..7) of two adjacent float4 loads to eight MFMAs:
// the two loads of a row's four lanes cover whole 128-byte lines.  Plain (cached) loads: a
// non-temporal hint let lines leave L2 between the two halves and doubled the HBM traffic.
// Tile: D rows = 16 rows of R, D columns = 16 realisations (b0 .. b0+15, masked to B).
// ---------------------------------------------------------------------------------------

template <int TR>
__global__ __launch_bounds__(kRB) void recon_mfma_kernel(const float* __restrict__ R, int M,
                                                         int N, const float* __restrict__ S,
                                                         int B, int b0, int chunk, int splits,
                                                         int row_groups, float* __restrict__ ws) {
  const int wave = (blockIdx.x * kRB + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= row_groups * splits) return;
  const int g = wave / splits, sp = wave - g * splits;
  const int k0 = sp * chunk, k1 = min(N, k0 + chunk);
  const int i16 = lane & 15, kq = lane >> 4;
  const int nb = b0 + i16;  // realisation fed by this lane (B operand column)
  const bool bok = nb < B;
  const float* srow = S + (int64_t)(bok ? nb : 0) * N;
  const float* rrow[TR];
#pragma unroll
  for (int t = 0; t < TR; ++t) {
    const int row = min(g * 16 * TR + t * 16 + i16, M - 1);
    rrow[t] = R + (int64_t)row * N;
  }
  v4f acc[TR];
#pragma unroll
  for (int t = 0; t < TR; ++t) acc[t] = (v4f){0.0f, 0.0f, 0.0f, 0.0f};
  int k = k0;
  // main loop: 32 columns per iteration (two float4 per lane per operand row), the next
  // iteration's loads issued before this iteration's MFMAs (double-buffered registers)
  float4 ra[TR], rb[TR], sa = make_float4(0.f, 0.f, 0.f, 0.f), sb = sa;
  if (k + 32 <= k1) {
    const int ka = k + 8 * kq, kb = ka + 4;
    if (bok) {
      sa = *reinterpret_cast<const float4*>(srow + ka);
      sb = *reinterpret_cast<const float4*>(srow + kb);
    }
#pragma unroll
    for (int t = 0; t < TR; ++t) {
      ra[t] = *reinterpret_cast<const float4*>(rrow[t] + ka);
      rb[t] = *reinterpret_cast<const float4*>(rrow[t] + kb);
    }
  }
  for (; k + 32 <= k1; k += 32) {
    float4 na[TR], nb[TR], nsa = make_float4(0.f, 0.f, 0.f, 0.f), nsb = nsa;
    const bool more = k + 64 <= k1;
    if (more) {
      const int ka = k + 32 + 8 * kq, kb = ka + 4;
      if (bok) {
        nsa = *reinterpret_cast<const float4*>(srow + ka);
        nsb = *reinterpret_cast<const float4*>(srow + kb);
      }
#pragma unroll
      for (int t = 0; t < TR; ++t) {
        na[t] = *reinterpret_cast<const float4*>(rrow[t] + ka);
        nb[t] = *reinterpret_cast<const float4*>(rrow[t] + kb);
      }
    }
#pragma unroll
    for (int t = 0; t < TR; ++t) {
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra[t].x, sa.x, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra[t].y, sa.y, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra[t].z, sa.z, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra[t].w, sa.w, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(rb[t].x, sb.x, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(rb[t].y, sb.y, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(rb[t].z, sb.z, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(rb[t].w, sb.w, acc[t], 0, 0, 0);
    }
    if (more) {
#pragma unroll
      for (int t = 0; t < TR; ++t) {
        ra[t] = na[t];
        rb[t] = nb[t];
      }
      sa = nsa;
      sb = nsb;
    }
  }
  // tail: 16 columns per step, float4 granularity, guarded
  for (; k < k1; k += 16) {
    const int ka = k + 4 * kq;
    const bool in = ka < k1;
    float4 sa = make_float4(0.f, 0.f, 0.f, 0.f);
    if (bok && in) sa = *reinterpret_cast<const float4*>(srow + ka);
#pragma unroll
    for (int t = 0; t < TR; ++t) {
      float4 ra = make_float4(0.f, 0.f, 0.f, 0.f);
      if (in) ra = *reinterpret_cast<const float4*>(rrow[t] + ka);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra.x, sa.x, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra.y, sa.y, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra.z, sa.z, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra.w, sa.w, acc[t], 0, 0, 0);
    }
  }
  // D[4*kq + i][i16]: row = tile base + 4 kq + i, realisation = b0 + i16
  if (bok) {
#pragma unroll
    for (int t = 0; t < TR; ++t) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = g * 16 * TR + t * 16 + 4 * kq + i;
        if (row < M) ws[((int64_t)sp * B + nb) * M + row] = acc[t][i];
      }
    }
  }
}

// C[b][i] = alpha * sum_sp ws[sp][b][i] + beta * C[b][i]   (splits added in order)
__global__ __launch_bounds__(kRB) void recon_reduce_kernel(const float* __restrict__ ws, int M,
                                                           int B, int splits, float* C,
                                                           int64_t ldc, float alpha, float beta,
                                                           int b_first, int b_count) {
  const int64_t gid = (int64_t)blockIdx.x * kRB + threadIdx.x;
  if (gid >= (int64_t)M * b_count) return;
  const int bl = (int)(gid / M), i = (int)(gid - (int64_t)bl * M);
  float s = 0.0f;
  for (int sp = 0; sp < splits; ++sp) s += ws[((int64_t)sp * b_count + bl) * M + i];
  float* c = C + (int64_t)(b_first + bl) * ldc + i;
  *c = beta == 0.0f ? alpha * s : fmaf(alpha, s, beta * *c);
}

// ---------------------------------------------------------------------------------------
// launch shape: every (row group, split) wave of a call runs in ONE round of the device's
// resident wave slots, so no wave of a second round streams its chunk after the others end
// ---------------------------------------------------------------------------------------
static std::mutex g_occ_mu;
static int g_slots[64][4];  // per device: resident waves of the MFMA, GEMV, unaligned and
                            // small-batch kernels

static hipError_t resident_waves(int which, int* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_occ_mu);
  if (g_slots[dev][which] == 0) {
    int cus = 0, blocks = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const void* k = which == 0   ? reinterpret_cast<const void*>(recon_mfma_kernel<2>)
                    : which == 1 ? reinterpret_cast<const void*>(recon_valu_kernel<2, true>)
                    : which == 2 ? reinterpret_cast<const void*>(recon_valu_kernel<2, false>)
                                 : reinterpret_cast<const void*>(
                                       recon_batch_lds_kernel<kBatchMax, kBatchPF>);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k, kRB, 0);
    if (e != hipSuccess) return e;
    g_slots[dev][which] = std::max(1, cus * std::max(1, blocks) * (kRB / 64));
  }
  *out = g_slots[dev][which];
  return hipSuccess;
}

// Splits of the N columns (chunks of a multiple of `align`) for `row_groups` waves per split:
// as many as one round of `slots` resident waves holds, at most N/256, and at most
// `max_splits` (the workspace a caller can offer).
static int choose_splits(int row_groups, int N, int align, int slots, int64_t max_splits,
                         int* chunk) {
  int64_t want = std::max<int64_t>(1, slots / row_groups);
  want = std::min<int64_t>(want, std::max(1, N / 256));
  want = std::max<int64_t>(1, std::min<int64_t>(want, max_splits));
  int c = (int)((N + want - 1) / want);
  c = (c + align - 1) / align * align;
  *chunk = c;
  return (N + c - 1) / c;  // <= want
}

struct ReconShape {
  int batch;       // 1: every realisation at once on the vector ALUs (2 <= B <= 8, aligned)
  int mfma;        // 1: matrix-core GEMM in tiles of 16 realisations; 0: one GEMV per realisation
  int aligned;     // 16-byte aligned R and S, N % 4 == 0
  int row_groups;
  int slots;
  int tile_b;      // realisations per partial-sum tile (16, or 1 for the GEMV)
};

static hipError_t recon_shape(const float* R, int M, int N, const float* S, int B,
                              ReconShape* sh) {
  sh->aligned = (N % 4 == 0) && ((uintptr_t)R % 16 == 0) && ((uintptr_t)S % 16 == 0);
  sh->batch = B >= 2 && B <= kBatchMax && sh->aligned;
  sh->mfma = B > kBatchMax && sh->aligned;
  sh->row_groups = sh->batch ? (M + kBatchRW - 1) / kBatchRW
                             : (sh->mfma ? (M + 31) / 32 : (M + 1) / 2);
  sh->tile_b = sh->batch ? B : (sh->mfma ? std::min(16, B) : 1);
  return resident_waves(sh->batch ? 3 : (sh->mfma ? 0 : (sh->aligned ? 1 : 2)), &sh->slots);
}

// Floats of partial sums a call wants (its split count unconstrained by the workspace).
hipError_t recon_work_floats(const float* R, int M, int N, const float* S, int B,
                             int64_t* floats) {
  ReconShape sh;
  hipError_t e = recon_shape(R, M, N, S, B, &sh);
  if (e != hipSuccess) return e;
  int chunk;
  const int splits = choose_splits(sh.row_groups, N,
                                   (sh.mfma ? 32 : (sh.aligned ? 256 : 64)), sh.slots,
                                   INT32_MAX, &chunk);
  *floats = (int64_t)splits * sh.tile_b * M;
  return hipSuccess;
}

// C = alpha R S^T + beta C with the split partial sums in ws (ws_floats >= M * min(B, 16));
// the split count shrinks to what ws holds.
hipError_t recon_launch(const float* R, int M, int N, const float* S, int B, float* C,
                        int64_t ldc, float alpha, float beta, float* ws, int64_t ws_floats,
                        hipStream_t st, int* used_mfma) {
  ReconShape sh;
  hipError_t e = recon_shape(R, M, N, S, B, &sh);
  if (e != hipSuccess) return e;
  *used_mfma = sh.mfma;
  const int64_t max_splits = ws_floats / ((int64_t)sh.tile_b * M);
  if (max_splits < 1) return hipErrorInvalidValue;
  if (sh.batch) {
    int chunk;
    const int quads = (sh.row_groups + 3) / 4;  // workgroups of 4 row groups per split
    const int splits = choose_splits(quads * 4, N, 256, sh.slots, max_splits, &chunk);
    const int grid = quads * splits;
    if (B <= 2)
      hipLaunchKernelGGL((recon_batch_lds_kernel<2, kBatchPF>), dim3(grid), dim3(kRB), 0, st, R,
                         M, N, S, B, chunk, quads, ws);
    else if (B <= 4)
      hipLaunchKernelGGL((recon_batch_lds_kernel<4, kBatchPF>), dim3(grid), dim3(kRB), 0, st, R,
                         M, N, S, B, chunk, quads, ws);
    else
      hipLaunchKernelGGL((recon_batch_lds_kernel<kBatchMax, kBatchPF>), dim3(grid), dim3(kRB), 0,
                         st, R, M, N, S, B, chunk, quads, ws);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)M * B;
    hipLaunchKernelGGL(recon_reduce_kernel, dim3((unsigned)((n + kRB - 1) / kRB)), dim3(kRB), 0,
                       st, ws, M, B, splits, C, ldc, alpha, beta, 0, B);
    return hipGetLastError();
  }
  if (sh.mfma) {
    constexpr int TR = 2;
    int chunk;
    const int splits = choose_splits(sh.row_groups, N, 32, sh.slots, max_splits, &chunk);
    for (int b0 = 0; b0 < B; b0 += 16) {
      const int bc = std::min(16, B - b0);
      const int waves = sh.row_groups * splits;
      hipLaunchKernelGGL(recon_mfma_kernel<TR>, dim3((waves + 3) / 4), dim3(kRB), 0, st, R, M,
                         N, S + (int64_t)b0 * N, bc, 0, chunk, splits, sh.row_groups, ws);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      const int64_t n = (int64_t)M * bc;
      hipLaunchKernelGGL(recon_reduce_kernel, dim3((unsigned)((n + kRB - 1) / kRB)), dim3(kRB), 0,
                         st, ws, M, bc, splits, C, ldc, alpha, beta, b0, bc);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  constexpr int RW = 2;
  int chunk;
  const int splits =
      choose_splits(sh.row_groups, N, sh.aligned ? 256 : 64, sh.slots, max_splits, &chunk);
  for (int b = 0; b < B; ++b) {
    const int waves = sh.row_groups * splits;
    if (sh.aligned)
      hipLaunchKernelGGL((recon_valu_kernel<RW, true>), dim3((waves + 3) / 4), dim3(kRB), 0, st,
                         R, M, N, S, b, chunk, splits, sh.row_groups, ws);
    else
      hipLaunchKernelGGL((recon_valu_kernel<RW, false>), dim3((waves + 3) / 4), dim3(kRB), 0,
                         st, R, M, N, S, b, chunk, splits, sh.row_groups, ws);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(recon_reduce_kernel, dim3((M + kRB - 1) / kRB), dim3(kRB), 0, st, ws, M,
                       1, splits, C, ldc, alpha, beta, b, 1);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------------------
// recon_apply's workspace: one buffer per (device, stream), so calls on different streams
// never share partial sums.  A buffer is never freed while the process lives (a captured
// graph may still hold it): a larger problem allocates a larger buffer and keeps the old one.
// No buffer is allocated while the stream is capturing.
// ---------------------------------------------------------------------------------------
struct StreamWork {
  int dev;
  hipStream_t stream;
  float* ptr;
  int64_t floats;
};
static std::mutex g_ws_mu;
static std::vector<StreamWork> g_ws;       // current buffer of each (device, stream)
static std::vector<float*> g_ws_retired;   // outgrown buffers, kept for captured graphs

hipError_t recon_stream_work(hipStream_t st, int64_t floats, float** out, bool* capturing) {
  *capturing = false;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_ws_mu);
  StreamWork* w = nullptr;
  for (auto& x : g_ws)
    if (x.dev == dev && x.stream == st) w = &x;
  if (w && w->floats >= floats) {
    *out = w->ptr;
    return hipSuccess;
  }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  e = hipStreamIsCapturing(st, &cs);
  if (e != hipSuccess) return e;
  if (cs != hipStreamCaptureStatusNone) {
    *capturing = true;
    return hipErrorStreamCaptureUnsupported;
  }
  float* p = nullptr;
  e = hipMalloc((void**)&p, sizeof(float) * (size_t)floats);
  if (e != hipSuccess) return e;
  if (w) {
    g_ws_retired.push_back(w->ptr);
    w->ptr = p;
    w->floats = floats;
  } else {
    g_ws.push_back(StreamWork{dev, st, p, floats});
  }
  *out = p;
  return hipSuccess;
}

// ---------------------------------------------------------------------------------------
// Fixed workspace of recon_apply_noalloc: a file-scope device array (each GPU the library runs
// on holds its own copy until the process ends).  In host code `scratch` names a host-side
// stand-in, not device memory: kernels get its device address, fetched once per device with
// hipGetSymbolAddress on the first call there.  Every call on one GPU shares it.
// ---------------------------------------------------------------------------------------
constexpr int64_t kStaticWorkFloats = int64_t(1) << 22;  // 16 MiB of partial sums
static __device__ __align__(256) float scratch[kStaticWorkFloats];
static std::mutex g_static_mu;
static float* g_static_ptr[64];

int64_t recon_static_work_floats() { return kStaticWorkFloats; }

// Floats of partial sums one split of a call needs (M rows x the realisations of one tile).
hipError_t recon_min_work_floats(const float* R, int M, int N, const float* S, int B,
                                 int64_t* floats) {
  ReconShape sh;
  hipError_t e = recon_shape(R, M, N, S, B, &sh);
  if (e != hipSuccess) return e;
  *floats = (int64_t)sh.tile_b * M;
  return hipSuccess;
}

hipError_t recon_static_work(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_static_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_static_ptr[dev];
  return hipSuccess;
}

}  // namespace wfs
