// FFT path of the Shack-Hartmann spot model: large subaperture fields without elongation
// (the NGS sensors), one 64-lane wave per chunk of the spectrum.
//
// Spot (our reading of the sensor of Sec. 2.7):  I = c |F|^2,  F = DFT_N(E) of the n x n field
// zero-padded to N x N (kernel e^{-2 pi i k m / N}), then fftshift and b x b binning.  With
// N = Q M (M = 16 or 32 points per register FFT) the spectrum splits into Q^2 chunks, each an
// M x M FFT of a folded, twiddled field (fft_chunk_m below), so a subaperture spreads over Q^2
// waves.  Deterministic.  The field phase comes from the projection kernel's buffer.
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

// LDS of one FFT wave (bytes): the chunk X [M][M + 1] float2 (rows padded against bank
// conflicts; later the spot |F|^2 of one chunk in the .x slots, and the binned image) and,
// with one chunk (Q = 1), the binned image [n_pix][n_pix].
__host__ __device__ inline int fft_wave_lds_bytes_impl(int n_fft, int n_pix) {
  const int M = n_fft >= 32 ? 32 : n_fft, Q = n_fft / M;
  return M * (M + 1) * 8 + (Q == 1 ? ((n_pix * n_pix * 4 + 15) & ~15) : 0);
}

// ---------------------------------------------------------------------------------------
// One wave per spectrum chunk.  With N = Q M every output index is f = Q k2 + k1 and every
// input index x = x2 + M x1, so chunk (k1y, k1x) of the 2-D spectrum is an M x M 2-D FFT of
// the folded, twiddled field
//     X[y2][x2] = sum_{y1, x1} e[y2 + M y1][x2 + M x1] W_Q^{y1 k1y + x1 k1x} W_N^{y2 k1y + x2 k1x}
// (one rotation in turns per input pixel).  With Q = b the fftshifted bin of output
// (Q k2y + k1y, Q k2x + k1x) is ((k2y + M/2) mod M, (k2x + M/2) mod M): each chunk adds one
// value to every bin.  The chunk writes its partial image to global memory and bumps the
// subaperture's counter; the wave that completes the count adds the Q^2 partial images in
// chunk order (deterministic), applies the noise and the centre of gravity, and resets the
// counter for the next launch.  With Q = 1 the wave holds the whole spectrum and bins it
// itself.
// ---------------------------------------------------------------------------------------
template <int M>
__device__ void fft_chunk_m(const FwdParams& p, const DevSensor& S, int sid, int b, int u,
                            int64_t step, char* wsm) {
  constexpr int G = kWave / M;  // lanes per column in the fold
  const int lane = lane_id();
  const int n = S.n_sub, N = S.n_fft, Q = N / M, Q2 = Q * Q, np = S.n_pix;
  const int v = u / Q2, c = u - v * Q2;
  const int k1y = c / Q, k1x = c - k1y * Q;
  const DevSubap sb = cload(p.sub, S.valid_off + v);
  const int nx1 = (n + M - 1) / M;
  float2* X = reinterpret_cast<float2*>(wsm);  // [M][M + 1]
  const float* ph = p.phase_in + (int64_t)b * p.phase_per_real + S.phase_off + (int64_t)v * n * n;
  const uint8_t* mrow0 = p.mask + S.mask_off + (sb.a * n) * S.n_pup + sb.b * n;
  // 1. fold: lane (column x2, group g) forms rows y2 = g, g + G, ...
  {
    const int x2 = lane & (M - 1), g = lane / M;
    for (int y2 = g; y2 < M; y2 += G) {
      float2 acc = make_float2(0.0f, 0.0f);
      for (int y1 = 0; y1 < nx1; ++y1) {
        const int y = y2 + M * y1;
        if (y >= n) break;
        for (int x1 = 0; x1 < nx1; ++x1) {
          const int x = x2 + M * x1;
          if (x < n && mrow0[y * S.n_pup + x]) {
            float t = fmaf(ph[y * n + x], 0.15915494309189535f,
                           -fmaf((float)x, S.ramp_x, (float)y * S.ramp_y));
            t -= rintf(t);
            // e^{2 pi i t} W_Q^{y1 k1y + x1 k1x} W_N^{y2 k1y + x2 k1x}
            float rot = t - (float)(y1 * k1y + x1 * k1x) / (float)Q -
                        (float)(y2 * k1y + x2 * k1x) / (float)N;
            rot -= rintf(rot);
            float sn, cs;
            sincos_rev(rot, &sn, &cs);
            acc.x += cs;
            acc.y += sn;
          }
        }
      }
      X[y2 * (M + 1) + x2] = acc;
    }
  }
  wave_sync();
  // 2. row FFTs (lane = row)
  if (lane < M) {
    float2 xr[M];
#pragma unroll
    for (int k = 0; k < M; ++k) xr[k] = X[lane * (M + 1) + k];
    fft_reg<M>(xr);
#pragma unroll
    for (int k = 0; k < M; ++k) X[lane * (M + 1) + k] = xr[k];
  }
  wave_sync();
  // 3. column FFTs (lane = column k2x): |F|^2 of frequency (Q k2y + k1y, Q k2x + k1x)
  float* spot = reinterpret_cast<float*>(X);  // the .x slot of X[k2y][k2x]
  if (lane < M) {
    float2 xc[M];
#pragma unroll
    for (int k = 0; k < M; ++k) xc[k] = X[k * (M + 1) + lane];
    fft_reg<M>(xc);
    if (Q == 1) {
#pragma unroll
      for (int k = 0; k < M; ++k)
        spot[2 * (k * (M + 1) + lane)] = S.flux_c * (xc[k].x * xc[k].x + xc[k].y * xc[k].y);
    } else {
      // partial image of this chunk, binned layout [qy][qx], qx = (k2x + M/2) mod M
      float* part = p.fft_part + (int64_t)b * p.fft_part_per_real + S.fft_part_off +
                    ((int64_t)v * Q2 + c) * (M * M);
      const int qx = (lane + M / 2) & (M - 1);
#pragma unroll
      for (int k = 0; k < M; ++k)
        part[((k + M / 2) & (M - 1)) * M + qx] = xc[k].x * xc[k].x + xc[k].y * xc[k].y;
    }
  }
  float* Bimg;
  if (Q == 1) {
    wave_sync();
    // bins of the fftshifted spot: B[qy][qx] = sum_{dy,dx<b} I[(b qy + dy + N/2) % N][...]
    Bimg = reinterpret_cast<float*>(wsm + M * (M + 1) * 8);
    const int bb = S.bin;
    for (int q = lane; q < np * np; q += kWave) {
      const int qy = q / np, qx = q - qy * np;
      float sum = 0.0f;
      for (int dy = 0; dy < bb; ++dy) {
        const int fy = (bb * qy + dy + N / 2) % N;
        for (int dx = 0; dx < bb; ++dx)
          sum += spot[2 * (fy * (M + 1) + (bb * qx + dx + N / 2) % N)];
      }
      Bimg[q] = sum;
    }
    wave_sync();
  } else {
    // the wave that completes the subaperture's count adds the partial images
    __threadfence();
    int32_t* cnt = p.fft_cnt + (int64_t)b * p.fft_cnt_per_real + S.fft_cnt_off + v;
    int old = 0;
    if (lane == 0) old = atomicAdd(cnt, 1);
    old = __shfl(old, 0, kWave);
    if (old != Q2 - 1) return;  // wave-uniform
    __threadfence();
    if (lane == 0) *cnt = 0;  // ready for the next launch
    const float* part0 = p.fft_part + (int64_t)b * p.fft_part_per_real + S.fft_part_off +
                         (int64_t)v * Q2 * (M * M);
    Bimg = reinterpret_cast<float*>(wsm);  // X is free now
    for (int q = lane; q < M * M; q += kWave) {
      float sum = 0.0f;
      for (int cc = 0; cc < Q2; ++cc) sum += __builtin_nontemporal_load(part0 + cc * (M * M) + q);
      Bimg[q] = S.flux_c * sum;
    }
    wave_sync();
  }
  // 4. noise + centre of gravity (pairs of pixels share a Philox block)
  const int np2 = np * np, npairs = (np2 + 1) >> 1;
  const float half = 0.5f * (float)(np - 1);
  float s0 = 0.0f, sx = 0.0f, sy = 0.0f;
  const bool noisy = S.noisy && p.noise_on;
  for (int pr = lane; pr < npairs; pr += kWave) {
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
  Cog cg;
  cg.s0 = wave_sum(s0);
  cg.sx = wave_sum(sx);
  cg.sy = wave_sum(sy);
  write_slopes(p, S, b, v, cg);
}

// ---------------------------------------------------------------------------------------
// Adjoint of the FFT path (noise off), one wave per spectrum chunk.  With the forward
// slopes (c_x, c_y) and pixel sum S of the subaperture and its slope gradients (g_x, g_y):
//   g_B[q] = (g_x (x_q - c_x) + g_y (y_q - c_y)) / S           (nothing when S <= 0)
//   H_c[k2] = g_B[bin of the chunk's frequency k2] F_c[k2]      (the adjoint of the binning
//                                                               and the fftshift)
//   G[m] = sum_c tw_c(m) IDFT_M(H_c)[m2],  tw_c(m) = e^{+2 pi i (k1 . m2 / N + k1 . m1 / Q)}
//          (G = D^H (g_I F), the unnormalised inverse transform, split by chunks: m = m2 + M m1)
//   g_psi[m] = 2 c Im(conj(E_m) G_m) kappa.
// Every chunk forms its share of g_psi on the n x n field pixels; with one chunk it goes
// straight to the pupil-frame image, otherwise to a partial buffer, and the wave that
// completes the subaperture's count adds the shares in chunk order (deterministic).
// ---------------------------------------------------------------------------------------
__host__ __device__ inline int fft_adj_wave_lds_bytes_impl(int n_fft, int n_pix) {
  const int M = n_fft >= 32 ? 32 : n_fft;
  return M * (M + 1) * 8 + ((n_pix * n_pix * 4 + 15) & ~15);
}

template <int M>
__device__ void fft_adjoint_chunk_m(const AdjParams& ap, const DevSensor& S, int sid, int b,
                                    int u, char* wsm) {
  const FwdParams& p = ap.f;
  constexpr int G = kWave / M;
  const int lane = lane_id();
  const int n = S.n_sub, N = S.n_fft, Q = N / M, Q2 = Q * Q, np = S.n_pix;
  const int v = u / Q2, c = u - v * Q2;
  const int k1y = c / Q, k1x = c - k1y * Q;
  // forward outputs and slope gradients of the subaperture (wave-uniform; all its chunks
  // take the same decision, so a subaperture without gradient writes nothing)
  const int64_t so = (int64_t)b * p.n_slopes + S.slope_off + v;
  const float gx = ap.grad_slopes[so], gy = ap.grad_slopes[so + S.n_valid];
  const float cx = ap.fwd_slopes[so], cy = ap.fwd_slopes[so + S.n_valid];
  const float s0 = ap.fwd_aux[(int64_t)b * p.n_valid_total + S.aux_off + v];
  if (!(s0 > 0.0f) || (gx == 0.0f && gy == 0.0f)) return;
  const DevSubap sb = cload(p.sub, S.valid_off + v);
  const int nx1 = (n + M - 1) / M;
  float2* X = reinterpret_cast<float2*>(wsm);              // [M][M + 1]
  float* gB = reinterpret_cast<float*>(wsm + M * (M + 1) * 8);  // [np][np]
  const float* ph = p.phase_in + (int64_t)b * p.phase_per_real + S.phase_off + (int64_t)v * n * n;
  const uint8_t* mrow0 = p.mask + S.mask_off + (sb.a * n) * S.n_pup + sb.b * n;
  {
    const float half = 0.5f * (float)(np - 1), inv = 1.0f / s0;
    for (int q = lane; q < np * np; q += kWave) {
      const int qy = q / np, qx = q - qy * np;
      gB[q] = (gx * ((float)qx - half - cx) + gy * ((float)qy - half - cy)) * inv;
    }
  }
  // the field's phase in turns at (y, x), or a dark pixel
  auto turns_at = [&](int y, int x, bool& lit) {
    lit = mrow0[y * S.n_pup + x] != 0;
    float t = fmaf(ph[y * n + x], 0.15915494309189535f,
                   -fmaf((float)x, S.ramp_x, (float)y * S.ramp_y));
    return t - rintf(t);
  };
  // 1. the forward chunk: fold, row and column FFTs (as fft_chunk_m)
  {
    const int x2 = lane & (M - 1), g = lane / M;
    for (int y2 = g; y2 < M; y2 += G) {
      float2 acc = make_float2(0.0f, 0.0f);
      for (int y1 = 0; y1 < nx1; ++y1) {
        const int y = y2 + M * y1;
        if (y >= n) break;
        for (int x1 = 0; x1 < nx1; ++x1) {
          const int x = x2 + M * x1;
          if (x >= n) continue;
          bool lit;
          const float t = turns_at(y, x, lit);
          if (lit) {
            float rot = t - (float)(y1 * k1y + x1 * k1x) / (float)Q -
                        (float)(y2 * k1y + x2 * k1x) / (float)N;
            rot -= rintf(rot);
            float sn, cs;
            sincos_rev(rot, &sn, &cs);
            acc.x += cs;
            acc.y += sn;
          }
        }
      }
      X[y2 * (M + 1) + x2] = acc;
    }
  }
  wave_sync();
  if (lane < M) {
    float2 xr[M];
#pragma unroll
    for (int k = 0; k < M; ++k) xr[k] = X[lane * (M + 1) + k];
    fft_reg<M>(xr);
#pragma unroll
    for (int k = 0; k < M; ++k) X[lane * (M + 1) + k] = xr[k];
  }
  wave_sync();
  // 2. column lane k2x: H = g_I F, then the inverse transform along y (conjugate, forward
  //    FFT, conjugate: the unnormalised inverse)
  if (lane < M) {
    float2 xc[M];
#pragma unroll
    for (int k = 0; k < M; ++k) xc[k] = X[k * (M + 1) + lane];
    fft_reg<M>(xc);
#pragma unroll
    for (int k = 0; k < M; ++k) {
      float gi;
      if (Q == 1) {  // frequency (k, lane) of the whole spectrum: bin of its fftshifted pixel
        const int fy = (k + N / 2) % N, fx = (lane + N / 2) % N;
        gi = gB[(fy / S.bin) * np + fx / S.bin];
      } else {
        gi = gB[((k + M / 2) & (M - 1)) * M + ((lane + M / 2) & (M - 1))];
      }
      xc[k] = make_float2(gi * xc[k].x, -gi * xc[k].y);  // conj(g_I F)
    }
    fft_reg<M>(xc);
#pragma unroll
    for (int k = 0; k < M; ++k) X[k * (M + 1) + lane] = make_float2(xc[k].x, -xc[k].y);
  }
  wave_sync();
  // 3. row lane y2: the inverse transform along x
  if (lane < M) {
    float2 xr[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const float2 z = X[lane * (M + 1) + k];
      xr[k] = make_float2(z.x, -z.y);
    }
    fft_reg<M>(xr);
#pragma unroll
    for (int k = 0; k < M; ++k) X[lane * (M + 1) + k] = make_float2(xr[k].x, -xr[k].y);
  }
  wave_sync();
  // 4. this chunk's share of g_psi on the field pixels m = (y2 + M y1, x2 + M x1)
  const float c2k = 2.0f * S.flux_c * S.kappa;
  float* gout = ap.gpsi + (int64_t)b * p.pupil_per_real + S.pupil_off +
                (int64_t)sb.a * n * S.n_pup + sb.b * n;
  float* part = Q == 1 ? nullptr
                       : ap.fft_adj_part + (int64_t)b * ap.fft_adj_per_real + S.fft_adj_off +
                             ((int64_t)v * Q2 + c) * (n * n);
  {
    const int x2 = lane & (M - 1), g = lane / M;
    for (int y2 = g; y2 < M; y2 += G) {
      const float2 yv = X[y2 * (M + 1) + x2];
      for (int y1 = 0; y1 < nx1; ++y1) {
        const int y = y2 + M * y1;
        if (y >= n) break;
        for (int x1 = 0; x1 < nx1; ++x1) {
          const int x = x2 + M * x1;
          if (x >= n) continue;
          bool lit;
          const float t = turns_at(y, x, lit);
          float r = 0.0f;
          if (lit) {
            float rot = (float)(y2 * k1y + x2 * k1x) / (float)N +
                        (float)(y1 * k1y + x1 * k1x) / (float)Q;
            rot -= rintf(rot);
            float sn, cs;
            sincos_rev(rot, &sn, &cs);
            const float gr = yv.x * cs - yv.y * sn, gim = yv.x * sn + yv.y * cs;  // G share
            float es, ec;
            sincos_rev(t, &es, &ec);
            r = c2k * (ec * gim - es * gr);  // 2 c kappa Im(conj(E) G)
          }
          if (Q == 1) gout[y * S.n_pup + x] = r;
          else part[y * n + x] = r;
        }
      }
    }
  }
  if (Q == 1) return;
  // 5. the wave completing the subaperture's count adds the shares in chunk order
  __threadfence();
  int32_t* cnt = p.fft_cnt + (int64_t)b * p.fft_cnt_per_real + S.fft_cnt_off + v;
  int old = 0;
  if (lane == 0) old = atomicAdd(cnt, 1);
  old = __shfl(old, 0, kWave);
  if (old != Q2 - 1) return;  // wave-uniform
  __threadfence();
  if (lane == 0) *cnt = 0;
  const float* part0 = ap.fft_adj_part + (int64_t)b * ap.fft_adj_per_real + S.fft_adj_off +
                       (int64_t)v * Q2 * (n * n);
  for (int q = lane; q < n * n; q += kWave) {
    float sum = 0.0f;
    for (int cc = 0; cc < Q2; ++cc) sum += __builtin_nontemporal_load(part0 + cc * (n * n) + q);
    const int y = q / n, x = q - y * n;
    gout[y * S.n_pup + x] = sum;
  }
}

__device__ __forceinline__ void fft_adjoint_wave(const AdjParams& ap, int task, char* wsm) {
  const FwdParams& p = ap.f;
  const int total = p.fft.per_real * p.batch;
  if (task >= total) return;
  int b, sid, u;
  task = __builtin_amdgcn_readfirstlane(task);
  task_of(p.fft, task, b, sid, u);
  const DevSensor S = cload(p.sen, sid);
  if (S.n_fft >= 32)
    fft_adjoint_chunk_m<32>(ap, S, sid, b, u, wsm);
  else
    fft_adjoint_chunk_m<16>(ap, S, sid, b, u, wsm);
}

// FFT-path task t (one wave): spectrum chunk (t - start) mod Q^2 of subaperture
// (t - start) / Q^2 of its sensor.
__device__ __forceinline__ void fft_wave(const FwdParams& p, int task, int64_t step,
                                         char* wsm) {
  const int total = p.fft.per_real * p.batch;
  if (task >= total) return;  // padding waves
  int b, sid, u;
  task = __builtin_amdgcn_readfirstlane(task);
  task_of(p.fft, task, b, sid, u);
  const DevSensor S = cload(p.sen, sid);
  if (S.n_fft >= 32)
    fft_chunk_m<32>(p, S, sid, b, u, step, wsm);
  else
    fft_chunk_m<16>(p, S, sid, b, u, step, wsm);
}

}  // namespace wfs
