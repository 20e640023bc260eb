// In-LDS FFTs shared by the PSF module and the phase-screen generator: power-of-two lengths
// N = 2^LOG2N, 16 <= N <= 4096, Stockham autosort.  Stages of radix 16 while 16 Ns <= N (Ns =
// the product of the radices before the stage), then one stage of radix 2, 4 or 8 when log2 N
// is not a multiple of 4; each butterfly is a 16- (4 x 4) or 8-point (2 x 4) DFT in registers.
//
// LDS layout: point i of a sequence sits at fft_pad(i) = i + i / 16 (one float2 of padding
// after every 16 points).  With it every stage's reads (16 consecutive butterflies read 16
// consecutive points) and writes (the first stage writes 16 consecutive points per butterfly,
// the later ones 16 consecutive points per 16 butterflies) fall on 16 different float2 bank
// pairs of the 32 four-byte banks, so a 64-bit access of 16 lanes meets no conflict.
//
// Twiddles: one table of N - 1 values, stage after stage; the stage of Ns (radix R) holds
// exp(-2 pi i m k / (R Ns)) at Ns - 1 + (m - 1) Ns + k (m = 1..R-1, k < Ns), so the lanes of a
// stage read consecutive entries.  fft_tw_angle gives each entry's angle in units of 2 pi / N.
#pragma once

#include <hip/hip_runtime.h>

namespace wfs {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__host__ __device__ constexpr int fft_pad(int i) { return i + (i >> 4); }

// LDS float2 of one padded sequence of N points
__host__ __device__ constexpr int fft_span(int N) { return N + (N >> 4); }

// Pitch of C padded sequences side by side: at least the span and congruent to 16 / C modulo
// 16, so that a load or store of the C sequences' point y, y + 1, ... by consecutive lanes
// (lane -> sequence lane % C) spreads over the bank pairs.
__host__ __device__ constexpr int fft_pitch(int N, int C) {
  const int s = fft_span(N);
  const int want = C >= 16 ? 1 : 16 / (C < 1 ? 1 : C);
  return s + (((want - s) % 16) + 16) % 16;
}

// Radix (log2) of the stage that starts at log2 Ns = lns.
__host__ __device__ constexpr int fft_stage_lr(int log2N, int lns) {
  return log2N - lns >= 4 ? 4 : log2N - lns;
}

// Angle of twiddle table entry pos (0 <= pos < N - 1) in units of 2 pi / N: the entry is
// exp(-2 pi i angle / N).
__host__ __device__ inline int fft_tw_angle(int log2N, int pos) {
  int lns = 0;
  while (lns < log2N) {
    const int lr = fft_stage_lr(log2N, lns), ns = 1 << lns;
    const int rel = pos - (ns - 1);
    if (rel < ((1 << lr) - 1) * ns) {
      const int m = rel / ns + 1, k = rel - (m - 1) * ns;
      return (m * k) << (log2N - lns - lr);
    }
    lns += lr;
  }
  return 0;
}

// a * exp(-2 pi i T / 16)
template <int T>
__device__ __forceinline__ float2 rot16(float2 a) {
  constexpr int t = ((T % 16) + 16) % 16;
  if constexpr (t == 0) return a;
  else if constexpr (t == 4) return make_float2(a.y, -a.x);
  else if constexpr (t == 8) return make_float2(-a.x, -a.y);
  else if constexpr (t == 12) return make_float2(-a.y, a.x);
  else {
    // cos and sin of 2 pi t / 16
    constexpr float kCos[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f,
                                0.38268343236508977f, 0.0f, -0.38268343236508977f,
                                -0.70710678118654752f, -0.92387953251128674f, -1.0f,
                                -0.92387953251128674f, -0.70710678118654752f,
                                -0.38268343236508977f, 0.0f, 0.38268343236508977f,
                                0.70710678118654752f, 0.92387953251128674f};
    constexpr float c = kCos[t], s = kCos[(t + 12) % 16];
    return make_float2(fmaf(a.x, c, a.y * s), fmaf(a.y, c, -(a.x * s)));
  }
}

__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  const float2 s02 = make_float2(a0.x + a2.x, a0.y + a2.y);
  const float2 d02 = make_float2(a0.x - a2.x, a0.y - a2.y);
  const float2 s13 = make_float2(a1.x + a3.x, a1.y + a3.y);
  const float2 d13 = make_float2(a1.x - a3.x, a1.y - a3.y);
  a0 = make_float2(s02.x + s13.x, s02.y + s13.y);
  a1 = make_float2(d02.x + d13.y, d02.y - d13.x);  // d02 - i d13
  a2 = make_float2(s02.x - s13.x, s02.y - s13.y);
  a3 = make_float2(d02.x - d13.y, d02.y + d13.x);  // d02 + i d13
}

// In-register R-point DFT, X[r] = sum_m a[m] exp(-2 pi i m r / R), natural order in and out.
template <int R>
__device__ __forceinline__ void dft(float2* a) {
  if constexpr (R == 2) {
    const float2 u = a[0], v = a[1];
    a[0] = make_float2(u.x + v.x, u.y + v.y);
    a[1] = make_float2(u.x - v.x, u.y - v.y);
  } else if constexpr (R == 4) {
    dft4(a[0], a[1], a[2], a[3]);
  } else if constexpr (R == 8) {
    // m = m1 + 2 m2, r = r1 + 4 r2: 4-point DFTs over m2, twiddle exp(-2 pi i m1 r1 / 8),
    // 2-point DFTs over m1
    float2 y0[4] = {a[0], a[2], a[4], a[6]}, y1[4] = {a[1], a[3], a[5], a[7]};
    dft4(y0[0], y0[1], y0[2], y0[3]);
    dft4(y1[0], y1[1], y1[2], y1[3]);
    y1[1] = rot16<2>(y1[1]);
    y1[2] = rot16<4>(y1[2]);
    y1[3] = rot16<6>(y1[3]);
#pragma unroll
    for (int r1 = 0; r1 < 4; ++r1) {
      a[r1] = make_float2(y0[r1].x + y1[r1].x, y0[r1].y + y1[r1].y);
      a[r1 + 4] = make_float2(y0[r1].x - y1[r1].x, y0[r1].y - y1[r1].y);
    }
  } else {
    static_assert(R == 16, "radix 2, 4, 8 or 16");
    // m = m1 + 4 m2, r = r1 + 4 r2: 4-point DFTs over m2, twiddle exp(-2 pi i m1 r1 / 16),
    // 4-point DFTs over m1
    float2 y[4][4];
#pragma unroll
    for (int m1 = 0; m1 < 4; ++m1) {
      y[m1][0] = a[m1];
      y[m1][1] = a[m1 + 4];
      y[m1][2] = a[m1 + 8];
      y[m1][3] = a[m1 + 12];
      dft4(y[m1][0], y[m1][1], y[m1][2], y[m1][3]);
    }
    y[1][1] = rot16<1>(y[1][1]);
    y[1][2] = rot16<2>(y[1][2]);
    y[1][3] = rot16<3>(y[1][3]);
    y[2][1] = rot16<2>(y[2][1]);
    y[2][2] = rot16<4>(y[2][2]);
    y[2][3] = rot16<6>(y[2][3]);
    y[3][1] = rot16<3>(y[3][1]);
    y[3][2] = rot16<6>(y[3][2]);
    y[3][3] = rot16<9>(y[3][3]);
#pragma unroll
    for (int r1 = 0; r1 < 4; ++r1) {
      dft4(y[0][r1], y[1][r1], y[2][r1], y[3][r1]);
      a[r1] = y[0][r1];
      a[r1 + 4] = y[1][r1];
      a[r1 + 8] = y[2][r1];
      a[r1 + 12] = y[3][r1];
    }
  }
}

// One Stockham stage (radix 2^LR at Ns = 2^LNS) over `cnt` sequences at buf + c * ld:
// butterfly j of a sequence takes points j + m N / R, twiddles them by exp(-2 pi i m k /
// (R Ns)), k = j mod Ns, and writes its DFT to (j - k) R + k + r Ns.  Every input is read
// into registers, the workgroup waits, then the outputs are written (one buffer suffices).
template <int LOG2N, int LNS, int LR, int POINTS, int THREADS>
__device__ __forceinline__ void fft_stage(float2* buf, int cnt, int ld,
                                          const float2* __restrict__ tw) {
  constexpr int R = 1 << LR, NS = 1 << LNS, LB = LOG2N - LR, NB = 1 << LB;
  constexpr int MAXB = (POINTS / R + THREADS - 1) / THREADS;
  const int tid = threadIdx.x;
  const int nb = cnt << LB;
  float2 y[MAXB][R];
  int ob[MAXB];
#pragma unroll
  for (int it = 0; it < MAXB; ++it) {
    const int b = tid + it * THREADS;
    if (b < nb) {
      const int c = b >> LB, j = b & (NB - 1), k = j & (NS - 1);
      const float2* x = buf + c * ld;
      if constexpr (NB % 16 == 0) {  // the inputs sit at fixed distances from pad(j)
        const float2* xj = x + fft_pad(j);
#pragma unroll
        for (int m = 0; m < R; ++m) y[it][m] = xj[m * fft_span(NB)];
      } else {
#pragma unroll
        for (int m = 0; m < R; ++m) y[it][m] = x[fft_pad(j + m * NB)];
      }
      if constexpr (NS > 1) {
        const float2* t = tw + (NS - 1) + k;
#pragma unroll
        for (int m = 1; m < R; ++m) y[it][m] = cmul(y[it][m], t[(m - 1) * NS]);
      }
      dft<R>(y[it]);
      ob[it] = ((j - k) << LR) + k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < MAXB; ++it) {
    const int b = tid + it * THREADS;
    if (b < nb) {
      const int o = ob[it];  // (j - k) R + k within the sequence
      float2* s = buf + (b >> LB) * ld;
      if constexpr (NS % 16 == 0) {  // outputs at fixed distances from pad(o)
        float2* so = s + fft_pad(o);
#pragma unroll
        for (int r = 0; r < R; ++r) so[r * fft_span(NS)] = y[it][r];
      } else if constexpr (NS == 1 && R == 16) {  // pad(16 j + r) = 17 j + r
        float2* so = s + fft_pad(o);
#pragma unroll
        for (int r = 0; r < R; ++r) so[r] = y[it][r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) s[fft_pad(o + r * NS)] = y[it][r];
      }
    }
  }
  __syncthreads();
}

template <int LOG2N, int LNS, int POINTS, int THREADS>
__device__ __forceinline__ void fft_stages(float2* buf, int cnt, int ld,
                                           const float2* __restrict__ tw) {
  if constexpr (LNS < LOG2N) {
    constexpr int LR = fft_stage_lr(LOG2N, LNS);
    fft_stage<LOG2N, LNS, LR, POINTS, THREADS>(buf, cnt, ld, tw);
    fft_stages<LOG2N, LNS + LR, POINTS, THREADS>(buf, cnt, ld, tw);
  }
}

// In-place forward DFT, X[k] = sum_j x[j] exp(-2 pi i j k / N), of `cnt` sequences of N =
// 2^LOG2N points, point i of sequence c at buf[c * ld + fft_pad(i)] (cnt N <= POINTS), with
// the twiddle table tw (LDS or global).  The caller waits for its own writes to buf first.
template <int LOG2N, int POINTS, int THREADS>
__device__ __forceinline__ void lds_fft(float2* buf, int cnt, int ld,
                                        const float2* __restrict__ tw) {
  static_assert(LOG2N >= 4 && LOG2N <= 12, "16 <= N <= 4096");
  fft_stages<LOG2N, 0, POINTS, THREADS>(buf, cnt, ld, tw);
}

}  // namespace wfs
