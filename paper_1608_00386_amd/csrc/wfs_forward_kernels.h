// The spot launch of the forward model, one kernel per (subaperture size, mode): every sensor
// of a plan for every realisation at one time step.
//   blocks [0, fft_blocks)   : FFT path, one spectrum chunk of a large field per wave
//   remaining blocks         : lag-domain path, one subaperture per 64-lane wavefront at a time,
//                              with (pipelined frames) the next step's projection blocks spread
//                              evenly among them
// The mode is a template parameter so that each kernel only holds the registers of its own
// paths: FIELD says where the lag-domain waves get the phase (kField*), FFT adds the FFT-path
// blocks, PROJ the projection blocks.  With the staged footprint (kFieldFoot) one launch can
// cover several frames: the lag-domain blocks repeat once per frame, frame k at step + k.
#pragma once

#include "wfs_fft.h"
#include "wfs_otf.h"
#include "wfs_project.h"

namespace wfs {

// Split-schedule lag-domain kernels are held to 5 waves per SIMD for n_sub <= 10 (<= 96
// VGPRs; their LDS, < 7.5 KB per wave with the lag row in 2 passes, lets 5 four-wave blocks
// share a CU), fewer above.  LP = 3 passes shrink the partial rows so that 7 blocks share a
// CU (n_sub = 10): slower where a launch does not fill the chip (one 80 x 80 LGS: the extra
// pass is pure VALU), faster where it takes several rounds of blocks (8 realisations of six
// LGS: 0.61 -> 0.58 ms per step); the plan picks per launch size and the tuner times both.
template <int NS, bool PROJ>
constexpr int otf_waves_per_simd() {
  return NS <= 10 ? 5 : (NS == 11 ? 4 : 3);
}

template <int NS, int FIELD, bool FFT, bool PROJ, int LP = kOtfLagParts>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu((FIELD == kFieldGather || FFT) ? 1
                                                                  : otf_waves_per_simd<NS, PROJ>())))
void wfs_forward_kernel(
    FwdParams p) {
  extern __shared__ __align__(16) char smem[];
  const int64_t step = current_step(p);
  const int i = blockIdx.x;
  if constexpr (FFT) {
    if (i < p.fft_blocks) {  // FFT path: one spectrum chunk per wave
      const int w = threadIdx.x >> 6;
      fft_wave(p, i * kWavesPerBlock + w, step, smem + w * p.lds_per_wave);
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
  int frame = 0;
  if constexpr (FIELD == kFieldFoot) {  // blocks of frame k follow those of frame k - 1
    frame = L / p.otf_blocks;
    L -= frame * p.otf_blocks;
  }
  const int wave = threadIdx.x >> 6;
  char* wsm = smem + wave * p.lds_per_wave;
  const int total = p.otf.per_real * p.batch;
  // one subaperture per wave and no task loop: a loop would let the compiler hoist per-lane
  // index arithmetic out of it and hold those registers across every stage
  const int t = L * kWavesPerBlock + wave;
  if (t < total) otf_subap<NS, FIELD, LP>(p, t, step + frame, wsm, frame);
}

template <int NS, int FIELD, bool FFT, bool PROJ, int LP = kOtfLagParts>
static hipError_t launch_fwd_mode(const FwdParams& p, int grid, int lds, hipStream_t st) {
  hipLaunchKernelGGL((wfs_forward_kernel<NS, FIELD, FFT, PROJ, LP>), dim3(grid), dim3(kBlock),
                     lds, st, p);
  return hipGetLastError();
}

// split field: the lag row in p.lag_parts passes (2 or 3)
template <int NS, bool FFT, bool PROJ>
static hipError_t launch_fwd_phase(const FwdParams& p, int grid, int lds, hipStream_t st) {
  if (p.lag_parts == 3) return launch_fwd_mode<NS, kFieldPhase, FFT, PROJ, 3>(p, grid, lds, st);
  return launch_fwd_mode<NS, kFieldPhase, FFT, PROJ>(p, grid, lds, st);
}

// Launch of the spot kernel for subaperture size NS (lag-domain path), mode from the params.
template <int NS>
hipError_t launch_fwd_ns(const FwdParams& p, hipStream_t st) {
  const bool foot = p.otf_from_phase == kFieldFoot;
  const int64_t grid64 = (int64_t)p.fft_blocks + p.proj_blocks +
                         (int64_t)p.otf_blocks * (foot ? p.n_frames : 1);
  if (grid64 == 0) return hipSuccess;
  if (grid64 > 0x7FFFFFFF) return hipErrorInvalidValue;
  const int grid = (int)grid64;
  int lds = p.lds_per_wave * kWavesPerBlock;
  if (p.proj_blocks > 0 && p.proj_lds > lds) lds = p.proj_lds;
  const bool fused = p.otf_from_phase == kFieldGather, fft = p.fft_blocks > 0,
             proj = p.proj_blocks > 0;
  if (foot) {  // one launch for every frame; no FFT-path or projection blocks
    if (fft || proj || p.n_frames < 1) return hipErrorInvalidValue;
    return launch_fwd_mode<NS, kFieldFoot, false, false>(p, grid, lds, st);
  }
  if (fused) {  // the pipelined projection only exists in the split schedule
    if (proj) return hipErrorInvalidValue;
    return fft ? launch_fwd_mode<NS, kFieldGather, true, false>(p, grid, lds, st)
               : launch_fwd_mode<NS, kFieldGather, false, false>(p, grid, lds, st);
  }
  if (fft)
    return proj ? launch_fwd_phase<NS, true, true>(p, grid, lds, st)
                : launch_fwd_phase<NS, true, false>(p, grid, lds, st);
  return proj ? launch_fwd_phase<NS, false, true>(p, grid, lds, st)
              : launch_fwd_phase<NS, false, false>(p, grid, lds, st);
}

}  // namespace wfs
