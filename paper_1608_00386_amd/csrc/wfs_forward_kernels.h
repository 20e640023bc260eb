// The spot launch of the forward model, one kernel per (subaperture size, mode): every sensor
// of a plan for every realisation at one time step.
//   blocks [0, fft_blocks)   : FFT path, one subaperture per 256-thread workgroup (large fields)
//   remaining blocks         : lag-domain path, one subaperture per 64-lane wavefront at a time,
//                              with (pipelined frames) the next step's projection blocks spread
//                              evenly among them
// The mode is a template parameter so that each kernel only holds the registers of its own
// paths: FUSED gathers the layers in the lag-domain waves, FFT adds the FFT-path blocks, PROJ
// the projection blocks.
#pragma once

#include "wfs_fft.h"
#include "wfs_otf.h"
#include "wfs_project.h"

namespace wfs {

// Split-schedule lag-domain kernels are held to 5 waves per SIMD for n_sub <= 10 (<= 96
// VGPRs; their LDS, < 7 KB per wave, lets 5 four-wave blocks share a CU), fewer above.
// Measured on config 1: splitting the lag row in 3 or 4 passes to fit 7 or 8 waves per SIMD
// made the kernel slower (the spot stage is bound by VALU issue, not by latency).
template <int NS, bool PROJ>
constexpr int otf_waves_per_simd() {
  return NS <= 10 ? 5 : (NS == 11 ? 4 : 3);
}

template <int NS, bool FUSED, bool FFT, bool PROJ>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu((FUSED || FFT) ? 1 : otf_waves_per_simd<NS, PROJ>())))
void wfs_forward_kernel(
    FwdParams p) {
  extern __shared__ __align__(16) char smem[];
  const int64_t step = current_step(p);
  const int i = blockIdx.x;
  if constexpr (FFT) {
    if (i < p.fft_blocks) {
      fft_subap(p, i, step, smem);
      return;
    }
  }
  const int n = gridDim.x - p.fft_blocks;
  const int ib = i - p.fft_blocks;
  int L = p.xcd_remap ? xcd_logical_block(ib, n) : ib;
  if constexpr (PROJ) {
    // pipelined frames: projection blocks of the next step spread evenly among the spot
    // blocks, so memory-latency-bound gathers share the CUs with VALU-bound spot waves.
    // Block L is a projection block when floor((L+1)P/n) > floor(LP/n).
    const int c0 = (int)((int64_t)L * p.proj_blocks / n);
    const int c1 = (int)((int64_t)(L + 1) * p.proj_blocks / n);
    if (c1 > c0) {
      project_block(p, c0, p.phase_out, (double)(step + 1), smem);
      return;
    }
    L -= c1;
  }
  const int wave = threadIdx.x >> 6;
  char* wsm = smem + wave * p.lds_per_wave;
  const int total = p.otf.per_real * p.batch;
  // one subaperture per wave and no task loop: a loop would let the compiler hoist per-lane
  // index arithmetic out of it and hold those registers across every stage
  const int t = L * kWavesPerBlock + wave;
  if (t < total) otf_subap<NS, FUSED>(p, t, step, wsm);
}

template <int NS, bool FUSED, bool FFT, bool PROJ>
static hipError_t launch_fwd_mode(const FwdParams& p, int grid, int lds, hipStream_t st) {
  hipLaunchKernelGGL((wfs_forward_kernel<NS, FUSED, FFT, PROJ>), dim3(grid), dim3(kBlock), lds,
                     st, p);
  return hipGetLastError();
}

// Launch of the spot kernel for subaperture size NS (lag-domain path), mode from the params.
template <int NS>
hipError_t launch_fwd_ns(const FwdParams& p, hipStream_t st) {
  const int grid = p.fft_blocks + p.otf_blocks + p.proj_blocks;
  if (grid == 0) return hipSuccess;
  int lds = p.lds_per_wave * kWavesPerBlock;
  if (p.proj_blocks > 0 && p.proj_lds > lds) lds = p.proj_lds;
  const bool fused = !p.otf_from_phase, fft = p.fft_blocks > 0, proj = p.proj_blocks > 0;
  if (fused) {  // the pipelined projection only exists in the split schedule
    if (proj) return hipErrorInvalidValue;
    return fft ? launch_fwd_mode<NS, true, true, false>(p, grid, lds, st)
               : launch_fwd_mode<NS, true, false, false>(p, grid, lds, st);
  }
  if (fft)
    return proj ? launch_fwd_mode<NS, false, true, true>(p, grid, lds, st)
                : launch_fwd_mode<NS, false, true, false>(p, grid, lds, st);
  return proj ? launch_fwd_mode<NS, false, false, true>(p, grid, lds, st)
              : launch_fwd_mode<NS, false, false, false>(p, grid, lds, st);
}

}  // namespace wfs
