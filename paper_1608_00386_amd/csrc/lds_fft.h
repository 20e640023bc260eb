// In-LDS FFTs shared by the PSF module and the phase-screen generator: power-of-two lengths,
// Stockham autosort, radix-4 stages and one radix-2 stage when log2 N is odd.
#pragma once

#include <hip/hip_runtime.h>

namespace wfs {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-place forward DFT, X[k] = sum_j x[j] exp(-2 pi i j k / N), of `cnt` sequences of N = 2^log2N
// points held in LDS at buf + c * ld.  Each Stockham stage reads its inputs into registers,
// waits for the whole workgroup, writes its outputs and waits again, so one buffer suffices.
template <int POINTS, int THREADS>
__device__ void lds_fft(float2* buf, int cnt, int ld, int N, int log2N,
                        const float2* __restrict__ tw) {
  constexpr int kB4 = POINTS / 4 / THREADS;  // radix-4 butterflies per thread
  constexpr int kB2 = POINTS / 2 / THREADS;  // radix-2 butterflies per thread
  const int tid = threadIdx.x;
  const int q = N >> 2, lq = log2N - 2;
  int Ns = 1;
  for (int st = 0; st + 2 <= log2N; st += 2) {
    const int nb = cnt << lq;
    const int tstep = N / (4 * Ns);
    float2 y[kB4][4];
    int ob[kB4];
#pragma unroll
    for (int it = 0; it < kB4; ++it) {
      const int b = tid + it * THREADS;
      if (b < nb) {
        const int c = b >> lq, j = b & (q - 1);
        const int k = j & (Ns - 1);
        const float2* x = buf + c * ld + j;
        const float2 a0 = x[0];
        float2 a1 = x[q], a2 = x[2 * q], a3 = x[3 * q];
        if (Ns > 1) {
          a1 = cmul(a1, tw[k * tstep]);
          a2 = cmul(a2, tw[2 * k * tstep]);
          a3 = cmul(a3, tw[3 * k * tstep]);
        }
        const float2 s02 = make_float2(a0.x + a2.x, a0.y + a2.y);
        const float2 d02 = make_float2(a0.x - a2.x, a0.y - a2.y);
        const float2 s13 = make_float2(a1.x + a3.x, a1.y + a3.y);
        const float2 d13 = make_float2(a1.x - a3.x, a1.y - a3.y);
        y[it][0] = make_float2(s02.x + s13.x, s02.y + s13.y);
        y[it][1] = make_float2(d02.x + d13.y, d02.y - d13.x);  // d02 - i d13
        y[it][2] = make_float2(s02.x - s13.x, s02.y - s13.y);
        y[it][3] = make_float2(d02.x - d13.y, d02.y + d13.x);  // d02 + i d13
        ob[it] = c * ld + ((j - k) << 2) + k;
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kB4; ++it) {
      const int b = tid + it * THREADS;
      if (b < nb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) buf[ob[it] + r * Ns] = y[it][r];
      }
    }
    __syncthreads();
    Ns <<= 2;
  }
  if (log2N & 1) {  // last stage, radix 2 at Ns = N / 2: outputs land where the inputs were
    const int h = N >> 1, lh = log2N - 1;
    const int nb = cnt << lh;
#pragma unroll
    for (int it = 0; it < kB2; ++it) {
      const int b = tid + it * THREADS;
      if (b < nb) {
        const int c = b >> lh, j = b & (h - 1);
        float2* x = buf + c * ld + j;
        const float2 a0 = x[0];
        const float2 a1 = cmul(x[h], tw[j]);
        x[0] = make_float2(a0.x + a1.x, a0.y + a1.y);
        x[h] = make_float2(a0.x - a1.x, a0.y - a1.y);
      }
    }
    __syncthreads();
  }
}

}  // namespace wfs
