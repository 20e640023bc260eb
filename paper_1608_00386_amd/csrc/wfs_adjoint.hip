// Adjoint of the noise-free forward sensor model (slopes -> layer screens), lag-domain path.
//
// Forward, per subaperture (see wfs_otf.h):  B[q] = c sum_k A[k] T[k] e^{2 pi i k.q / n_pix}
// over all lags k, with A[k] = sum_m E[m] conj(E[m+k]), T[k] = Kel[k] s(kx) s(ky), and the
// slopes c_x = sum (x_q) B / sum B, c_y likewise.  Given g = dL/d(c_x, c_y):
//   g_B[q] = (g_x (x_q - c_x) + g_y (y_q - c_y)) / sum B          (0 when sum B <= 0)
//   U[k]   = c T[k] ghat[k],  ghat[k] = sum_q g_B[q] e^{2 pi i k.q / n_pix}   (Hermitian in k)
//   dL     = Re sum_k U[k] dA[k],  dE[m] = i E[m] dpsi[m]
//   =>  g_psi[p] = -2 Im(E[p] V[p]),   V[p] = sum_{m'} U[m' - p] conj(E[m'])
// and the layer gradient is the transpose of the bilinear projection, kappa w_l times the
// stencil weights, accumulated with floating-point atomics (subaperture fields recomputed).
#include "wfs_otf.h"

namespace wfs {

struct AdjLds {
  int u_off, gz_off, gh_off, gb_off, total;
};

__host__ __device__ inline AdjLds adj_lds_layout(int ns, int n_layers, int n_pix) {
  const OtfLds f = otf_lds_layout(ns, n_layers, n_pix);
  const int nl = 2 * ns - 1, np2 = n_pix * n_pix;
  AdjLds a;
  int o = f.total;
  a.u_off = o;
  o += nl * nl * 8;
  a.gz_off = o;
  o += np2 * 8;
  a.gh_off = o;
  o += np2 * 8;
  a.gb_off = o;
  o += np2 * 4;
  a.total = (o + 15) & ~15;
  return a;
}

template <int NS, bool FUSED>
__device__ void otf_adjoint_subap(const AdjParams& ap, int t, int64_t step, char* wsm) {
  const FwdParams& p = ap.f;
  const int lane = lane_id();
  int b, sid, v;
  t = __builtin_amdgcn_readfirstlane(t);
  task_of(p.otf, t, b, sid, v);
  const DevSensor S = cload(p.sen, sid);
  const DevSubap sb = cload(p.sub, S.valid_off + v);
  const int np = S.n_pix, np2 = np * np;
  const OtfLds lo = otf_lds_layout(NS, p.n_layers, np);
  const AdjLds la = adj_lds_layout(NS, p.n_layers, np);
  const float gx = ap.grad_slopes[(int64_t)b * p.n_slopes + S.slope_off + v];
  const float gy = ap.grad_slopes[(int64_t)b * p.n_slopes + S.slope_off + S.n_valid + v];
  float s0, cx, cy;
  if (ap.fwd_slopes) {
    otf_field<NS, FUSED>(p, S, sb, sid, b, (double)step, wsm, lo);
    s0 = ap.fwd_aux[(int64_t)b * p.n_valid_total + S.aux_off + v];
    cx = ap.fwd_slopes[(int64_t)b * p.n_slopes + S.slope_off + v];
    cy = ap.fwd_slopes[(int64_t)b * p.n_slopes + S.slope_off + S.n_valid + v];
  } else {
    otf_spot<NS, FUSED>(p, S, sb, sid, b, step, wsm, lo);
    const Cog c = cog_sums(p, S, sid, b, v, step, reinterpret_cast<const float*>(wsm + lo.b_off));
    s0 = c.s0;
    cx = s0 > 0.0f ? c.sx / s0 : 0.0f;
    cy = s0 > 0.0f ? c.sy / s0 : 0.0f;
  }
  wave_sync();
  if (!(s0 > 0.0f) || (gx == 0.0f && gy == 0.0f)) return;  // wave-uniform

  const float half = 0.5f * (float)(np - 1);
  const float inv = 1.0f / s0;
  float* gB = reinterpret_cast<float*>(wsm + la.gb_off);
  for (int q = lane; q < np2; q += kWave) {
    const int qy = fdiv(q, np, S.inv_npix), qx = q - qy * np;
    gB[q] = (gx * ((float)qx - half - cx) + gy * ((float)qy - half - cy)) * inv;
  }
  wave_sync();
  // ghat[Ky][Kx] = sum_q gB[q] W^{Kx qx + Ky qy}, separable (W = e^{2 pi i / n_pix})
  const float2* wt = reinterpret_cast<const float2*>(wsm + lo.wtab_off);
  float2* GZ = reinterpret_cast<float2*>(wsm + la.gz_off);  // [qy][Kx]
  for (int t2 = lane; t2 < np2; t2 += kWave) {
    const int qy = fdiv(t2, np, S.inv_npix), Kx = t2 - qy * np;
    float2 z = make_float2(0.0f, 0.0f);
    int idx = 0;
    for (int qx = 0; qx < np; ++qx) {
      const float g = gB[qy * np + qx];
      const float2 w = wt[idx];
      z.x = fmaf(g, w.x, z.x);
      z.y = fmaf(g, w.y, z.y);
      idx += Kx;
      if (idx >= np) idx -= np;
    }
    GZ[t2] = z;
  }
  wave_sync();
  float2* GH = reinterpret_cast<float2*>(wsm + la.gh_off);  // [Ky][Kx]
  for (int t2 = lane; t2 < np2; t2 += kWave) {
    const int Ky = fdiv(t2, np, S.inv_npix), Kx = t2 - Ky * np;
    float2 h = make_float2(0.0f, 0.0f);
    int idx = 0;
    for (int qy = 0; qy < np; ++qy) {
      const float2 z = GZ[qy * np + Kx];
      const float2 w = wt[idx];
      h.x = fmaf(z.x, w.x, fmaf(-z.y, w.y, h.x));
      h.y = fmaf(z.x, w.y, fmaf(z.y, w.x, h.y));
      idx += Ky;
      if (idx >= np) idx -= np;
    }
    GH[t2] = h;
  }
  wave_sync();
  // U[k] = c Kel(k) s(kx) s(ky) ghat[k mod n_pix] on all (2 NS - 1)^2 lags
  constexpr int NL = 2 * NS - 1;
  float2* U = reinterpret_cast<float2*>(wsm + la.u_off);
  const float2* stab = reinterpret_cast<const float2*>(wsm + lo.stab_off);
  for (int t2 = lane; t2 < NL * NL; t2 += kWave) {
    const int iy = t2 / NL, ix = t2 - iy * NL;
    const int dy = iy - (NS - 1), dx = ix - (NS - 1);
    // lags -> bins modulo n_pix (|lag| < NS, so one shift by a multiple of n_pix is enough)
    const int dyp = dy + np * NS, dxp = dx + np * NS;
    const int Ky = dyp - np * fdiv(dyp, np, S.inv_npix);
    const int Kx = dxp - np * fdiv(dxp, np, S.inv_npix);
    const float2 g = GH[Ky * np + Kx];
    const float2 sx = stab[ix], sy = stab[iy];
    const float proj = fmaf((float)dx, sb.ex, (float)dy * sb.ey);
    const float kel = __expf(-sb.alpha * proj * proj) * S.flux_c;
    const float tr = (sx.x * sy.x - sx.y * sy.y) * kel;
    const float ti = (sx.x * sy.y + sx.y * sy.x) * kel;
    U[t2] = make_float2(tr * g.x - ti * g.y, tr * g.y + ti * g.x);
  }
  // taps again (the forward scratch region is free now)
  const int nlay = p.n_layers;
  Tap* taps = reinterpret_cast<Tap*>(wsm + lo.taps_off);
  const double stepd = (double)step;
  for (int t2 = lane; t2 < 2 * NS * nlay; t2 += kWave) {
    const int l = t2 / (2 * NS), k = t2 - l * (2 * NS);
    taps[t2] = (k < NS) ? col_tap(p, sid, l, sb.b * NS + k, stepd)
                        : row_tap(p, sid, l, sb.a * NS + (k - NS), stepd);
  }
  wave_sync();
  const float2* E = reinterpret_cast<const float2*>(wsm + lo.e_off);
  float* gl = ap.grad_layers + (int64_t)b * p.layer_stride;
  for (int q = lane; q < NS * NS; q += kWave) {
    const int r = q / NS, c = q - r * NS;
    const float2 e = E[q];
    if (e.x == 0.0f && e.y == 0.0f) continue;  // dark pixel
    float2 V = make_float2(0.0f, 0.0f);
#pragma unroll 2
    for (int r2 = 0; r2 < NS; ++r2) {
      const float2* urow = U + (r2 - r + NS - 1) * NL + (NS - 1 - c);
#pragma unroll
      for (int c2 = 0; c2 < NS; ++c2) {
        const float2 u = urow[c2];
        const float2 f = E[r2 * NS + c2];
        // u * conj(f)
        V.x = fmaf(u.x, f.x, fmaf(u.y, f.y, V.x));
        V.y = fmaf(u.y, f.x, fmaf(-u.x, f.y, V.y));
      }
    }
    const float gpsi = -2.0f * (e.x * V.y + e.y * V.x) * S.kappa;
    for (int l = 0; l < nlay; ++l) {
      const DevLayer& L = p.lay[l];
      const Tap cxt = taps[l * 2 * NS + c];
      const Tap ryt = taps[l * 2 * NS + NS + r];
      const float gw = gpsi * L.weight;
      float* g = gl + L.offset;
      const float w00 = ryt.w0 * cxt.w0 * gw, w01 = ryt.w0 * cxt.w1 * gw;
      const float w10 = ryt.w1 * cxt.w0 * gw, w11 = ryt.w1 * cxt.w1 * gw;
      if (w00 != 0.0f) atomicAdd(g + ryt.i0 + cxt.i0, w00);
      if (w01 != 0.0f) atomicAdd(g + ryt.i0 + cxt.i1, w01);
      if (w10 != 0.0f) atomicAdd(g + ryt.i1 + cxt.i0, w10);
      if (w11 != 0.0f) atomicAdd(g + ryt.i1 + cxt.i1, w11);
    }
  }
  wave_sync();
}

template <int NS, bool FUSED>
__global__ __launch_bounds__(kBlock) void wfs_adjoint_kernel(AdjParams ap) {
  extern __shared__ __align__(16) char smem[];
  const FwdParams& p = ap.f;
  const int64_t step = current_step(p);
  const int wave = threadIdx.x >> 6;
  char* wsm = smem + wave * p.lds_per_wave;
  const int total = p.otf.per_real * p.batch;
  const int L = p.xcd_remap ? xcd_logical_block(blockIdx.x, gridDim.x) : blockIdx.x;
  const int t = L * kWavesPerBlock + wave;  // one subaperture per wave
  if (t < total) otf_adjoint_subap<NS, FUSED>(ap, t, step, wsm);
}

__global__ __launch_bounds__(kBlock) void zero_kernel(float* x, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) x[i] = 0.0f;
}

template <int NS>
static hipError_t launch_adj(AdjParams a, hipStream_t st) {
  const int64_t n = a.f.layer_stride * a.f.batch;
  const int zb = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 8192);
  hipLaunchKernelGGL(zero_kernel, dim3(zb > 0 ? zb : 1), dim3(kBlock), 0, st, a.grad_layers, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t tasks = (int64_t)a.f.otf.per_real * a.f.batch;
  if (tasks == 0) return hipSuccess;
  const int64_t waves = tasks;
  const int grid = (int)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
  if (a.f.otf_from_phase)
    hipLaunchKernelGGL((wfs_adjoint_kernel<NS, false>), dim3(grid), dim3(kBlock),
                       a.f.lds_per_wave * kWavesPerBlock, st, a);
  else
    hipLaunchKernelGGL((wfs_adjoint_kernel<NS, true>), dim3(grid), dim3(kBlock),
                       a.f.lds_per_wave * kWavesPerBlock, st, a);
  return hipGetLastError();
}

int adj_lds_bytes(int ns, int n_layers, int n_pix) {
  return adj_lds_layout(ns, n_layers, n_pix).total;
}

hipError_t launch_adjoint(const AdjParams& a, int ns, hipStream_t st) {
  switch (ns) {
    case 2: return launch_adj<2>(a, st);
    case 3: return launch_adj<3>(a, st);
    case 4: return launch_adj<4>(a, st);
    case 5: return launch_adj<5>(a, st);
    case 6: return launch_adj<6>(a, st);
    case 7: return launch_adj<7>(a, st);
    case 8: return launch_adj<8>(a, st);
    case 9: return launch_adj<9>(a, st);
    case 10: return launch_adj<10>(a, st);
    case 11: return launch_adj<11>(a, st);
    case 12: return launch_adj<12>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace wfs
