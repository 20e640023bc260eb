// FFT path of the Shack-Hartmann spot model: large subaperture fields without elongation
// (the NGS sensors), one 256-thread workgroup per subaperture.
//
// Spot (our reading of the sensor of Sec. 2.7):  I = c |F|^2,  F = DFT_N(E) of the n x n field
// zero-padded to N x N (kernel e^{-2 pi i k m / N}), then fftshift and b x b binning.
// With N = Q M (M = 16 or 32 points per register FFT, Q residue chunks) every output index
// is f = Q k2 + k1 and every input index x = x2 + M x1, so
//     DFT_N(e)[Q k2 + k1] = DFT_M( W_N^{x2 k1} sum_{x1} e[x2 + M x1] W_Q^{x1 k1} )[k2],
// i.e. chunk k1 of the outputs is one M-point FFT of a twiddled, folded input.  The 2-D
// transform runs chunk by chunk along x (row FFTs of the n field rows into LDS), then for
// every chunk along y (column FFTs, one thread per (k2x, k1y)).
// Binning: with Q = b (or Q = 1) the fftshifted bin of output (Q k2y + k1y, Q k2x + k1x) is
// ((k2y + M/2) mod M, (k2x + M/2) mod M) when Q = b, so each thread accumulates its bins in
// registers over the x chunks and the b partial rows are added in a fixed order at the end;
// with Q = 1 the spot goes to LDS and bins are summed directly.  Deterministic.
// The field phase comes from the projection kernel's buffer (kappa * psi per pixel).
#pragma once

#include "wfs_otf.h"

namespace wfs {

// ---------------------------------------------------------------------------------------
// compile-time twiddles W_M^k = e^{-2 pi i k / M}
// ---------------------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846;

constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 20; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}

constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 20; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

template <int M>
struct Twiddles {
  float c[M / 2 > 0 ? M / 2 : 1];
  float s[M / 2 > 0 ? M / 2 : 1];
  constexpr Twiddles() : c(), s() {
    for (int k = 0; k < M / 2; ++k) {
      const double a = -2.0 * kPi * k / M;  // |a| <= pi: the series converges to 1e-16
      c[k] = (float)taylor_cos(a);
      s[k] = (float)taylor_sin(a);
    }
  }
};

template <int M>
constexpr int bit_reverse(int i) {
  int r = 0;
  for (int m = M >> 1, b = 1; m > 0; m >>= 1, b <<= 1)
    if (i & b) r |= m;
  return r;
}

// In-register forward M-point FFT (radix 2, decimation in time), fully unrolled.
template <int M>
__device__ __forceinline__ void fft_reg(float2 (&x)[M]) {
  constexpr Twiddles<M> tw{};
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const int j = bit_reverse<M>(i);
    if (j > i) {
      const float2 t = x[i];
      x[i] = x[j];
      x[j] = t;
    }
  }
#pragma unroll
  for (int len = 2; len <= M; len <<= 1) {
#pragma unroll
    for (int i = 0; i < M; i += len) {
#pragma unroll
      for (int k = 0; k < len / 2; ++k) {
        const int t = k * (M / len);
        const float2 a = x[i + k];
        const float2 b = x[i + k + len / 2];
        float2 w;
        if (t == 0) {
          w = b;
        } else if (4 * t == M) {  // W = -i
          w = make_float2(b.y, -b.x);
        } else {
          w = make_float2(b.x * tw.c[t] - b.y * tw.s[t], b.x * tw.s[t] + b.y * tw.c[t]);
        }
        x[i + k] = make_float2(a.x + w.x, a.y + w.y);
        x[i + k + len / 2] = make_float2(a.x - w.x, a.y - w.y);
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// sizes
// ---------------------------------------------------------------------------------------
inline int fft_register_size(int n_fft) { return n_fft >= 32 ? 32 : n_fft; }

inline bool fft_supported_impl(int n_sub, int n_fft, int bin) {
  if (n_fft != 16 && n_fft != 32 && n_fft != 64 && n_fft != 128) return false;
  if (n_sub > kFftMaxNsub || 2 * n_sub > n_fft) return false;
  const int M = fft_register_size(n_fft), Q = n_fft / M;
  return Q == 1 || Q == bin;
}

// LDS of one FFT workgroup (bytes):
//   G [n][M] float2 | fin: spot [N][N] (Q = 1) or b row partials [Q][n_pix][n_pix] |
//   binned image [n_pix][n_pix] (Q = 1) | block reduction [16]
// (32 KB for a 64-pixel field in a 128-point transform: a workgroup's share per wave stays
// near a lag-domain wave's, so both kinds of block can share a launch)
struct FftLds {
  int g_off, fin_off, bq_off, red_off, total;
};

__host__ __device__ inline FftLds fft_lds_layout(int n_sub, int n_fft, int n_pix) {
  const int M = n_fft >= 32 ? 32 : n_fft, Q = n_fft / M;
  FftLds o;
  o.g_off = 0;
  o.fin_off = o.g_off + ((n_sub * M * 8 + 15) & ~15);
  o.bq_off = o.fin_off + (((Q == 1) ? n_fft * n_fft * 4 : Q * n_pix * n_pix * 4) + 15) / 16 * 16;
  o.red_off = o.bq_off + (((Q == 1) ? n_pix * n_pix * 4 : 0) + 15) / 16 * 16;
  o.total = o.red_off + 64;
  return o;
}

inline int fft_lds_bytes_impl(int n_sub, int n_fft, int n_pix) {
  return fft_lds_layout(n_sub, n_fft, n_pix).total;
}

// ---------------------------------------------------------------------------------------
// one subaperture per workgroup
// ---------------------------------------------------------------------------------------
template <int M>
__device__ void fft_subap_m(const FwdParams& p, const DevSensor& S, const DevSubap& sb,
                            int sid, int b, int v, int64_t step, char* smem) {
  const int tid = threadIdx.x;
  const int n = S.n_sub, N = S.n_fft, Q = N / M, np = S.n_pix;
  const int nx1 = (n + M - 1) / M;  // input chunks per axis (1 or 2)
  const FftLds lo = fft_lds_layout(n, N, np);
  float2* G = reinterpret_cast<float2*>(smem + lo.g_off);
  float* fin = reinterpret_cast<float*>(smem + lo.fin_off);
  float* red = reinterpret_cast<float*>(smem + lo.red_off);  // 3 x 4 floats

  // field phase in turns (kappa psi / 2 pi - the centring ramp and tip-tilt), read by each row
  // thread straight from the phase buffer; dark pixels contribute nothing
  const float* ph = p.phase_in + (int64_t)b * p.phase_per_real + S.phase_off + (int64_t)v * n * n;
  const uint8_t* mrow0 = p.mask + S.mask_off + (sb.a * n) * S.n_pup + sb.b * n;

  // Q = b: thread (k2x, k1y) owns the partial bins fin[k1y][(k2y + M/2) % M][(k2x + M/2) % M]
  // for every k2y and accumulates them over the x chunks (no other thread touches them)
  if (Q > 1)
    for (int q = tid; q < Q * np * np; q += kBlock) fin[q] = 0.0f;

  for (int k1x = 0; k1x < Q; ++k1x) {
    // rows: G[y][k2x] = DFT_M(W_N^{x2 k1x} sum_x1 e[y][x2 + M x1] W_Q^{x1 k1x})[k2x]
    for (int y = tid; y < n; y += kBlock) {
      float2 xr[M];
#pragma unroll
      for (int x2 = 0; x2 < M; ++x2) {
        float2 s = make_float2(0.0f, 0.0f);
        for (int x1 = 0; x1 < nx1; ++x1) {
          const int x = x2 + M * x1;
          if (x < n) {
            float t = fmaf(ph[y * n + x], 0.15915494309189535f,
                           -fmaf((float)x, S.ramp_x, (float)y * S.ramp_y));
            t -= rintf(t);
            if (mrow0[y * S.n_pup + x]) {
              // e^{2 pi i t} W_Q^{x1 k1x} W_N^{x2 k1x}: one rotation in turns
              const float rot = t - (float)(x1 * k1x) / (float)Q - (float)(x2 * k1x) / (float)N;
              float sn, cs;
              sincos_rev(rot - rintf(rot), &sn, &cs);
              s.x += cs;
              s.y += sn;
            }
          }
        }
        xr[x2] = s;
      }
      fft_reg<M>(xr);
#pragma unroll
      for (int k = 0; k < M; ++k) G[y * M + k] = xr[k];
    }
    __syncthreads();
    // columns: thread (k2x, k1y); F[Q k2y + k1y][Q k2x + k1x]
    for (int w = tid; w < M * Q; w += kBlock) {
      const int k2x = w % M, k1y = w / M;
      float2 xc[M];
#pragma unroll
      for (int y2 = 0; y2 < M; ++y2) {
        float2 s = make_float2(0.0f, 0.0f);
        for (int y1 = 0; y1 < nx1; ++y1) {
          const int y = y2 + M * y1;
          if (y < n) {
            const float2 g = G[y * M + k2x];
            const float rot = -(float)(y1 * k1y) / (float)Q - (float)(y2 * k1y) / (float)N;
            float sn, cs;
            sincos_rev(rot - rintf(rot), &sn, &cs);
            s.x = fmaf(g.x, cs, fmaf(-g.y, sn, s.x));
            s.y = fmaf(g.x, sn, fmaf(g.y, cs, s.y));
          }
        }
        xc[y2] = s;
      }
      fft_reg<M>(xc);
      if (Q == 1) {  // spot column k2x -> LDS (fftshift and binning below)
#pragma unroll
        for (int k = 0; k < M; ++k) fin[k * N + k2x] = S.flux_c * (xc[k].x * xc[k].x + xc[k].y * xc[k].y);
      } else {
        const int qx = (k2x + M / 2) % M;
#pragma unroll
        for (int k = 0; k < M; ++k)
          fin[(k1y * np + (k + M / 2) % M) * np + qx] += xc[k].x * xc[k].x + xc[k].y * xc[k].y;
      }
    }
    __syncthreads();
  }

  float* Bimg = fin;  // binned image [np][np]
  if (Q == 1) {
    // bins of the fftshifted spot: B[qy][qx] = sum_{dy,dx<b} I[(b qy + dy + N/2) % N][...]
    float* Bq = reinterpret_cast<float*>(smem + lo.bq_off);
    const int bb = S.bin;
    for (int q = tid; q < np * np; q += kBlock) {
      const int qy = q / np, qx = q - qy * np;
      float s = 0.0f;
      for (int dy = 0; dy < bb; ++dy) {
        const int fy = (bb * qy + dy + N / 2) % N;
        for (int dx = 0; dx < bb; ++dx) s += fin[fy * N + (bb * qx + dx + N / 2) % N];
      }
      Bq[q] = s;
    }
    Bimg = Bq;
  } else {
    // the b = Q partial rows of every bin, summed in k1y order
    for (int q = tid; q < np * np; q += kBlock) {
      float s = 0.0f;
      for (int k1y = 0; k1y < Q; ++k1y) s += fin[k1y * np * np + q];
      fin[q] = S.flux_c * s;  // rows >= 1 of the partials are not read again
    }
  }
  __syncthreads();

  // noise + centre of gravity over the block (pairs of pixels, fixed reduction order)
  const int np2 = np * np, npairs = (np2 + 1) >> 1;
  const float half = 0.5f * (float)(np - 1);
  float s0 = 0.0f, sx = 0.0f, sy = 0.0f;
  const bool noisy = S.noisy && p.noise_on;
  for (int pr = tid; pr < npairs; pr += kBlock) {
    const int q0 = 2 * pr, q1 = 2 * pr + 1;
    float b0 = Bimg[q0];
    float b1 = q1 < np2 ? Bimg[q1] : 0.0f;
    if (noisy) {
      const uint4 ctr = make_uint4((uint32_t)pr, (uint32_t)v, ((uint32_t)b << 8) | (uint32_t)sid,
                                   (uint32_t)(step + p.noise_dstep));
      add_noise_pair(b0, b1, philox4x32_10(ctr, p.seed_lo, p.seed_hi), S.read_noise);
      if (q1 >= np2) b1 = 0.0f;
    }
    const int y0 = q0 / np, x0 = q0 - y0 * np;
    const int y1 = q1 / np, x1 = q1 - y1 * np;
    s0 += b0 + b1;
    sx = fmaf((float)x0 - half, b0, fmaf((float)x1 - half, b1, sx));
    sy = fmaf((float)y0 - half, b0, fmaf((float)y1 - half, b1, sy));
  }
  s0 = wave_sum(s0);
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  const int wave = tid >> 6;
  __syncthreads();
  if (lane_id() == 0) {
    red[wave] = s0;
    red[4 + wave] = sx;
    red[8 + wave] = sy;
  }
  __syncthreads();
  if (tid == 0) {
    Cog c;
    c.s0 = (red[0] + red[1]) + (red[2] + red[3]);
    c.sx = (red[4] + red[5]) + (red[6] + red[7]);
    c.sy = (red[8] + red[9]) + (red[10] + red[11]);
    write_slopes(p, S, b, v, c);
  }
}

__device__ __forceinline__ void fft_subap(const FwdParams& p, int task, int64_t step,
                                          char* smem) {
  const int total = p.fft.per_real * p.batch;
  if (task >= total) return;  // padding blocks
  int b, sid, v;
  task_of(p.fft, task, b, sid, v);
  const DevSensor S = cload(p.sen, sid);
  const DevSubap sb = cload(p.sub, S.valid_off + v);
  if (S.n_fft >= 32)
    fft_subap_m<32>(p, S, sb, sid, b, v, step, smem);
  else
    fft_subap_m<16>(p, S, sb, sid, b, v, step, smem);
}

}  // namespace wfs
