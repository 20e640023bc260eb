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
// stencil weights (subaperture fields recomputed).  Two ways to form it:
//   gather (default): g_psi (kappa applied) goes to a phase-layout buffer, then one thread per
//     layer pixel sums, sensor by sensor, the stencil weights of the pupil pixels whose
//     forward taps touch it (the same FP64 taps as the forward) -- bitwise deterministic.
//     Layers whose pupil and layer pitches are within about a factor of two read those
//     pupil pixels from per-step lists (one small kernel per call builds them, the gather
//     then needs no FP64 and no searches); the others search their candidates per tile;
//   atomic scatter: each pupil pixel adds its four weighted taps with FP32 atomics.
#include "wfs_fft.h"
#include "wfs_otf.h"

namespace wfs {

struct AdjLds {
  int u_off, gz_off, gh_off, gb_off, total;
};

// Row pitch (float2) of the adjoint's lag array U: at least 2 n_sub - 1 and congruent to n_sub
// modulo 16, so that lane q = r n_sub + c of the correlation loop, reading U at offset
// -(pitch r + c), falls on bank pair q mod 16: every half-wave meets each pair twice, the
// fewest a 64-bit read can (a pitch of 2 n_sub - 1 put up to four lanes on one pair).
__host__ __device__ constexpr int adj_u_pitch(int ns) {
  return 2 * ns - 1 + (((1 - ns) % 16) + 16) % 16;
}

// Per-wave LDS of the adjoint: the forward layout, then the backward arrays U, GZ, GH, gB.  Once
// the spot (or only the field) is formed, only E and the sensor tables of the forward layout
// are read again, so in the gather form (no stencil taps) the backward arrays go into the dead
// regions between E and the tables when they fit (n_sub = 10, 8 x 8 pixels: 7.3 KB per wave
// instead of 12.7 KB, 5 four-wave blocks a CU instead of 3); the atomic form keeps its taps in
// the forward union and places the backward arrays after the forward layout.
__host__ __device__ inline AdjLds adj_lds_layout(int ns, int n_layers, int n_pix, bool gather) {
  const OtfLds f = otf_lds_layout(ns, n_layers, n_pix);
  const int nl = 2 * ns - 1, np2 = n_pix * n_pix;
  AdjLds a;
  const int ub = nl * adj_u_pitch(ns) * 8, gbb = (np2 * 4 + 7) & ~7, gzb = np2 * 8;
  const int e_end = (ns * otf_pitch(ns) * 8 + 15) & ~15;
  if (gather && e_end + ub + gbb + 2 * gzb <= f.stab_off) {
    a.u_off = e_end;
    a.gb_off = a.u_off + ub;
    a.gz_off = a.gb_off + gbb;
    a.gh_off = a.gz_off + gzb;
    a.total = f.total;
    return a;
  }
  int o = f.total;
  a.u_off = o;
  o += nl * adj_u_pitch(ns) * 8;
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
  const AdjLds la = adj_lds_layout(NS, p.n_layers, np, ap.gpsi != nullptr);
  const float gx = ap.grad_slopes[(int64_t)b * p.n_slopes + S.slope_off + v];
  const float gy = ap.grad_slopes[(int64_t)b * p.n_slopes + S.slope_off + S.n_valid + v];
  float s0, cx, cy;
  if (ap.fwd_slopes) {
    otf_field<NS, FUSED ? kFieldGather : kFieldPhase>(p, S, sb, sid, b, (double)step, wsm, lo);
    s0 = ap.fwd_aux[(int64_t)b * p.n_valid_total + S.aux_off + v];
    cx = ap.fwd_slopes[(int64_t)b * p.n_slopes + S.slope_off + v];
    cy = ap.fwd_slopes[(int64_t)b * p.n_slopes + S.slope_off + S.n_valid + v];
  } else {
    otf_spot<NS, FUSED ? kFieldGather : kFieldPhase>(p, S, sb, sid, b, step, wsm, lo);
    const Cog c = cog_sums(p, S, sid, b, v, step, reinterpret_cast<const float*>(wsm + lo.b_off));
    s0 = c.s0;
    cx = s0 > 0.0f ? c.sx / s0 : 0.0f;
    cy = s0 > 0.0f ? c.sy / s0 : 0.0f;
  }
  wave_sync();
  // gather mode: this subaperture's block of the sensor's pupil-frame gradient image
  float* gout = ap.gpsi ? ap.gpsi + (int64_t)b * p.pupil_per_real + S.pupil_off +
                              (int64_t)sb.a * NS * S.n_pup + sb.b * NS
                        : nullptr;
  if (!(s0 > 0.0f) || (gx == 0.0f && gy == 0.0f)) {  // wave-uniform: no gradient (the image
    return;                                            // was cleared before the launch)
  }

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
  constexpr int UP = adj_u_pitch(NS);
  const NaEntry el = na_entry(p, step);
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
    const float2 k = elong_tf(sb, el, proj, S.flux_c);
    const float sr = sx.x * sy.x - sx.y * sy.y, si = sx.x * sy.y + sx.y * sy.x;
    const float tr = sr * k.x - si * k.y;
    const float ti = sr * k.y + si * k.x;
    U[iy * UP + ix] = make_float2(tr * g.x - ti * g.y, tr * g.y + ti * g.x);
  }
  // taps again (the forward scratch region is free now); the gather mode needs none
  const int nlay = p.n_layers;
  Tap* taps = reinterpret_cast<Tap*>(wsm + lo.taps_off);
  const double stepd = (double)step;
  if (!gout) {
    for (int t2 = lane; t2 < 2 * NS * nlay; t2 += kWave) {
      const int l = t2 / (2 * NS), k = t2 - l * (2 * NS);
      taps[t2] = (k < NS) ? col_tap(p, sid, l, sb.b * NS + k, stepd)
                          : row_tap(p, sid, l, sb.a * NS + (k - NS), stepd);
    }
  }
  wave_sync();
  const float2* E = reinterpret_cast<const float2*>(wsm + lo.e_off);
  float* gl = ap.grad_layers + (int64_t)b * p.layer_stride;
  for (int q = lane; q < NS * NS; q += kWave) {
    const int r = q / NS, c = q - r * NS;
    const float2 e = E[r * Otf<NS>::kEP + c];
    if (e.x == 0.0f && e.y == 0.0f) continue;  // dark pixel
    float2 V = make_float2(0.0f, 0.0f);
#pragma unroll 2
    for (int r2 = 0; r2 < NS; ++r2) {
      const float2* urow = U + (r2 - r + NS - 1) * UP + (NS - 1 - c);
#pragma unroll
      for (int c2 = 0; c2 < NS; ++c2) {
        const float2 u = urow[c2];
        const float2 f = E[r2 * Otf<NS>::kEP + c2];
        // u * conj(f)
        V.x = fmaf(u.x, f.x, fmaf(u.y, f.y, V.x));
        V.y = fmaf(u.y, f.x, fmaf(-u.x, f.y, V.y));
      }
    }
    const float gpsi = -2.0f * (e.x * V.y + e.y * V.x) * S.kappa;
    if (gout) {
      gout[r * S.n_pup + c] = gpsi;
      continue;
    }
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

// Gather tiles: kGTW layer columns x kGTH layer rows per block; wave w takes the rows
// w, w + 4, ... (kGPix rows per thread).
constexpr int kGTW = 64;
constexpr int kGPix = 4;
constexpr int kGTH = kGPix * kBlock / kGTW;
constexpr int kGCols = 128;  // candidate pupil columns per pass
constexpr int kGRows = 32;   // candidate pupil rows per pass

// Candidate taps of a tile: pupil index k, the tap's lower index relative to the tile start
// (floor(w) - m n - tile start, w the layer coordinate, m the periodic image) and the weight
// of the upper neighbour.  The lower weight is 1 - w1, as in the forward's make_tap.
struct GTap {
  int32_t k, rel;
  float w1;
  int32_t pad;
};

// Exact forward tap of pupil index k against layer image m (see make_tap: for a periodic
// grid the fractional part of the unwrapped coordinate equals that of the wrapped one; for a
// zero boundary, candidates lie within a few pixels of the grid, where no clamping happens).
__device__ __forceinline__ GTap gather_tap(double a, double b0, double db, double stepd,
                                           int k, int64_t shift) {
  const double w = fma(a, (double)k, b0) + stepd * db;
  const double f0 = floor(w);
  GTap t;
  t.k = k;
  t.rel = (int32_t)((int64_t)f0 - shift);
  t.w1 = (float)(w - f0);
  t.pad = 0;
  return t;
}

// Pupil index range [lo, hi] whose coordinate w = a k + b (a > 0) falls in [t0 - 1, t1 + 1),
// with one index of slack on each side, clamped to [0, npup).
__device__ __forceinline__ void cand_range(double inv_a, double b, double t0, double t1,
                                           int npup, int& lo, int& hi) {
  // one index of slack on each side also covers the rounding of the reciprocal
  const double lo_d = floor((t0 - 1.0 - b) * inv_a) - 1.0;
  const double hi_d = ceil((t1 + 1.0 - b) * inv_a) + 1.0;
  lo = lo_d < 0.0 ? 0 : (lo_d > (double)npup ? npup : (int)lo_d);
  hi = hi_d < -1.0 ? -1 : (hi_d > (double)(npup - 1) ? npup - 1 : (int)hi_d);
}

// Periodic images m whose layer window [t0 - 1 + m n, t1 + 1 + m n) can meet the pupil's
// coordinate range [w(0), w(npup - 1)]; a single image for a zero boundary.
__device__ __forceinline__ void image_range(double a, double b, int n, double inv_n, int npup,
                                            int t0, int t1, int boundary, int& m_lo,
                                            int& m_hi) {
  if (boundary != 0) {
    m_lo = m_hi = 0;
    return;
  }
  const double w0 = b, w1 = fma(a, (double)(npup - 1), b);
  // floor / ceil of the bounds already include every image the rounding could move in
  m_lo = (int)floor((w0 - t1 - 1.0) * inv_n);
  m_hi = (int)ceil((w1 - t0 + 1.0) * inv_n);
}

// Layer gradient, gather form: block = (realisation, layer, kGTH x kGTW tile); thread =
// layer pixel.  For every sensor, pass by pass over the tile's candidate pupil rows and
// columns (every periodic image, kGRows x kGCols at a time): their exact forward taps and the
// rectangle of the sensor's phase-gradient image they span go to LDS (one batch of coalesced
// loads); then each wave (one layer row) walks the candidate rows, and each lane the few
// candidate columns whose taps reach its pixel, summing weight x gradient in a fixed order.
__global__ __launch_bounds__(kBlock) void wfs_adjoint_gather_kernel(GatherParams g) {
  __shared__ GTap ct[kGCols];
  __shared__ GTap rt[kGRows];
  __shared__ float gt[kGRows][kGCols];
  __shared__ float tt[kGRows][kGTW];  // column-transposed rows: sum over c of w_c g[r][c]
  __shared__ int rfirst[kGTH];        // first candidate row reaching each tile row
  const FwdParams& p = g.f;
  const int nl = p.n_layers;
  const int per_real = g.blk_start[nl];
  const int b = blockIdx.x / per_real;
  const int rb = blockIdx.x - b * per_real;
  int l = 0;
  while (l + 1 < nl && rb >= g.blk_start[l + 1]) ++l;  // block-uniform
  const DevLayer L = cload(p.lay, l);
  const int tiles_x = (L.nx + kGTW - 1) / kGTW;
  const int tile = rb - g.blk_start[l];
  const int ty0 = (tile / tiles_x) * kGTH, tx0 = (tile - (tile / tiles_x) * tiles_x) * kGTW;
  const int tid = threadIdx.x;
  const int wy = __builtin_amdgcn_readfirstlane(tid / kGTW);  // wave: tile rows wy + 4 k
  const int lx = tid - wy * kGTW;
  const int i = tx0 + lx;
  constexpr int kWavesG = kBlock / kGTW;
  const double stepd = (double)current_step(p);
  const float* gb = g.gpsi + (int64_t)b * p.pupil_per_real;
  float acc[kGPix];
#pragma unroll
  for (int k = 0; k < kGPix; ++k) acc[k] = 0.0f;
  for (int s = 0; s < p.n_sensors; ++s) {
    const DevSensor S = cload(p.sen, s);
    const DevAffine A = cload(p.aff, (int64_t)s * nl + l);
    const double bx = A.bx0 + stepd * A.dbx, by = A.by0 + stepd * A.dby;
    const int npup = S.n_pup;
    const float* gs = gb + S.pupil_off;
    int my_lo, my_hi, mx_lo, mx_hi;
    image_range(A.ay, by, L.ny, L.inv_ny, npup, ty0, ty0 + kGTH - 1, L.boundary, my_lo, my_hi);
    image_range(A.ax, bx, L.nx, L.inv_nx, npup, tx0, tx0 + kGTW - 1, L.boundary, mx_lo, mx_hi);
    for (int my = my_lo; my <= my_hi; ++my) {
      const int64_t yshift = (int64_t)my * L.ny + ty0;
      int r_lo, r_hi;
      cand_range(A.inv_ay, by, (double)yshift, (double)(yshift + kGTH - 1), npup, r_lo, r_hi);
      for (int r0 = r_lo; r0 <= r_hi; r0 += kGRows) {
        const int nr = min(kGRows, r_hi - r0 + 1);
        for (int mx = mx_lo; mx <= mx_hi; ++mx) {
          const int64_t xshift = (int64_t)mx * L.nx + tx0;
          int c_lo, c_hi;
          cand_range(A.inv_ax, bx, (double)xshift, (double)(xshift + kGTW - 1), npup, c_lo,
                     c_hi);
          for (int c0 = c_lo; c0 <= c_hi; c0 += kGCols) {
            const int nc = min(kGCols, c_hi - c0 + 1);
            __syncthreads();  // previous pass done with the tables
            if (tid < nr) rt[tid] = gather_tap(A.ay, A.by0, A.dby, stepd, r0 + tid, yshift);
            if (tid < nc) ct[tid] = gather_tap(A.ax, A.bx0, A.dbx, stepd, c0 + tid, xshift);
            {  // gradient rectangle rows r0.., columns c0.. (kGCols-pitched), loads issued first
              constexpr int kPer = kGRows * kGCols / kBlock, kStep = kBlock / kGCols;
              const int qc = tid & (kGCols - 1), qb = tid / kGCols;
              const uint32_t o0 = (uint32_t)(r0 * npup + c0 + qc);  // < pupil_per_real < 2^31
              float v[kPer];
#pragma unroll
              for (int k = 0; k < kPer; ++k) {
                const int q = qb + k * kStep;
                v[k] = (q < nr && qc < nc) ? ld_idx(gs, o0 + (uint32_t)(q * npup)) : 0.0f;
              }
#pragma unroll
              for (int k = 0; k < kPer; ++k) {
                const int q = qb + k * kStep;
                if (q < nr) gt[q][qc] = v[k];
              }
            }
            __syncthreads();
            // separable transpose, first along columns: T[r][lx] = sum over the candidate
            // columns whose taps reach lx (rel in {lx - 1, lx}, a contiguous run: rel is
            // non-decreasing) of w_c g[r][c]; up to kGC4 of them kept in registers
            int q0 = 0, q1 = nc;
            while (q0 < q1) {
              const int mid = (q0 + q1) >> 1;
              if (ct[mid].rel + 1 < lx) q0 = mid + 1;
              else q1 = mid;
            }
            constexpr int kGC4 = 4;
            int qk[kGC4];
            float wk[kGC4];
            int nk = 0;
            bool more = false;
#pragma unroll
            for (int k = 0; k < kGC4; ++k) {
              qk[k] = 0;
              wk[k] = 0.0f;
              const int qc = q0 + k;
              if (qc < nc && ct[qc].rel <= lx) {
                const GTap tc = ct[qc];
                qk[k] = qc;
                wk[k] = (tc.rel == lx ? 1.0f - tc.w1 : 0.0f) + (tc.rel + 1 == lx ? tc.w1 : 0.0f);
                nk = k + 1;
              }
            }
            if (nk == kGC4 && q0 + kGC4 < nc && ct[q0 + kGC4].rel <= lx) more = true;
            for (int r = wy; r < nr; r += kWavesG) {
              float t = 0.0f;
#pragma unroll
              for (int k = 0; k < kGC4; ++k) t = fmaf(wk[k], gt[r][qk[k]], t);
              if (more) {  // coarse layer: more than kGC4 pupil columns per layer column
                for (int qc = q0 + kGC4; qc < nc; ++qc) {
                  const GTap tc = ct[qc];
                  if (tc.rel > lx) break;
                  const float wc =
                      (tc.rel == lx ? 1.0f - tc.w1 : 0.0f) + (tc.rel + 1 == lx ? tc.w1 : 0.0f);
                  t = fmaf(wc, gt[r][qc], t);
                }
              }
              tt[r][lx] = t;
            }
            if (tid < kGTH) {  // first candidate row whose taps reach tile row tid
              int r = 0, r1 = nr;
              while (r < r1) {
                const int mid = (r + r1) >> 1;
                if (rt[mid].rel + 1 < tid) r = mid + 1;
                else r1 = mid;
              }
              rfirst[tid] = r;
            }
            __syncthreads();
            // then along rows: G[ry][lx] += sum over the candidate rows reaching ry of w_r T
#pragma unroll
            for (int k = 0; k < kGPix; ++k) {
              const int ry = wy + k * kWavesG;  // wave-uniform
              for (int rr = rfirst[ry]; rr < nr; ++rr) {
                const GTap tr = rt[rr];
                if (tr.rel > ry) break;
                const float wr =
                    (tr.rel == ry ? 1.0f - tr.w1 : 0.0f) + (tr.rel + 1 == ry ? tr.w1 : 0.0f);
                acc[k] = fmaf(wr, tt[rr][lx], acc[k]);
              }
            }
          }
        }
      }
    }
  }
  if (i < L.nx) {
#pragma unroll
    for (int k = 0; k < kGPix; ++k) {
      const int j = ty0 + wy + k * kWavesG;
      if (j < L.ny)
        g.grad[(int64_t)b * p.layer_stride + L.offset + (int64_t)j * L.nx + i] =
            acc[k] * L.weight;
    }
  }
}

// ---------------------------------------------------------------------------------------
// Table-driven gather (layers whose inverse stencil lists are short: pupil and layer pitches
// within a factor of about two, one periodic image per layer pixel).
//
// Taps kernel, thread per (segment, layer index i): the pupil indices whose forward taps (the
// same FP64 coordinate and make_tap as the projection, bit for bit) touch i, in increasing
// order, with the weight i has in their stencil.  Candidates: for every periodic image m, the
// indices whose coordinate lies in [i - 1 + m n, i + 1 + m n), with a margin of one index.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void wfs_adjoint_taps_kernel(GatherTabParams g) {
  const FwdParams& p = g.f;
  const AdjSeg sg = g.segs[blockIdx.y];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= sg.n) return;
  const DevLayer L = p.lay[sg.l];
  const DevAffine A = p.aff[(int64_t)sg.s * p.n_layers + sg.l];
  const int npup = p.sen[sg.s].n_pup;
  const double stepd = (double)current_step(p);
  const bool ax = sg.axis == 0;
  const double a = ax ? A.ax : A.ay, b0 = ax ? A.bx0 : A.by0, db = ax ? A.dbx : A.dby;
  const double inv_a = ax ? A.inv_ax : A.inv_ay;
  const int32_t n = ax ? L.nx : L.ny;
  const double inv_n = ax ? L.inv_nx : L.inv_ny;
  const double b = b0 + stepd * db;
  int m_lo, m_hi;
  image_range(a, b, n, inv_n, npup, i, i, L.boundary, m_lo, m_hi);
  int2 out[kAdjKI];
#pragma unroll
  for (int k = 0; k < kAdjKI; ++k) out[k] = make_int2(-1, 0);
  int cnt = 0;
  for (int m = m_lo; m <= m_hi; ++m) {
    int lo, hi;
    const double base = (double)i + (double)m * (double)n;
    cand_range(inv_a, b, base, base, npup, lo, hi);
    for (int c = lo; c <= hi; ++c) {
      const double w = fma(a, (double)c, b0) + stepd * db;
      const Tap t = make_tap(w, n, inv_n, L.boundary, 1);
      const float wt = (t.i0 == i ? t.w0 : 0.0f) + (t.i1 == i ? t.w1 : 0.0f);
      if (wt != 0.0f && cnt < kAdjKI) {
#pragma unroll
        for (int k = 0; k < kAdjKI; ++k)
          if (k == cnt) out[k] = make_int2(c, __float_as_int(wt));
        ++cnt;
      }
    }
  }
  int2* dst = g.tab + sg.off + (int64_t)i * kAdjKI;
#pragma unroll
  for (int k = 0; k < kAdjKI; ++k) dst[k] = out[k];
}

// Gather kernel for tabled layers (one periodic image per layer pixel: for every sensor the
// pupil rows touching a run of layer rows are consecutive, and so are the pupil columns of
// one layer column).  Block = (realisation, tabled layer, 64 x 64 tile); wave = 64 layer
// columns (one per lane) x kG2R rows, accumulated in the wave's own LDS rows (the waves never
// wait for each other).  For every sensor in order, each pupil row r whose taps reach the
// wave's rows is reduced along the lane's column list,
//     T = sum_j wc_j g[r][cf + j],
// and added to the (at most two) layer rows of its forward row tap with that tap's weights
// (the same FP64 coordinate and make_tap as the projection).  Fixed order of every sum:
// bitwise deterministic.
constexpr int kG2R = 16;
constexpr int kG2TH = kG2R * kWavesPerBlock;
constexpr int kG2MaxPR = 64;  // pupil rows per sensor and wave (above: direct per-row lists)
constexpr int kG2Chunk = 8;   // pupil rows whose loads are in flight together

__global__ __launch_bounds__(kBlock) void wfs_adjoint_gather_tab_kernel(GatherTabParams g) {
  __shared__ float acc_s[kWavesPerBlock][kG2R][kWave];
  __shared__ float4 rtap_s[kWavesPerBlock][kG2MaxPR];  // (row - y0 of tap 0, of tap 1, w0, w1)
  const FwdParams& p = g.f;
  const int nl = p.n_layers;
  const int per_real = g.blk_start[nl];
  const int b = blockIdx.x / per_real;
  const int rb = blockIdx.x - b * per_real;
  int l = 0;
  while (l + 1 < nl && rb >= g.blk_start[l + 1]) ++l;  // block-uniform
  const DevLayer L = cload(p.lay, l);
  const int tiles_x = (L.nx + kWave - 1) / kWave;
  const int tile = rb - g.blk_start[l];
  const int tyi = tile / tiles_x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & (kWave - 1);
  const int x = (tile - tyi * tiles_x) * kWave + lane;
  const int y0 = tyi * kG2TH + wave * kG2R;
  const int nrows = min(kG2R, L.ny - y0);  // wave-uniform, may be <= 0
  if (nrows <= 0) return;                  // no block-wide barrier below
  const bool xin = x < L.nx;
  float* acc = &acc_s[wave][0][0];
  float4* rtap = rtap_s[wave];
#pragma unroll
  for (int yy = 0; yy < kG2R; ++yy) acc[yy * kWave + lane] = 0.0f;
  const float* gb = g.gpsi + (int64_t)b * p.pupil_per_real;
  const double stepd = (double)current_step(p);
  const int xl = xin ? x : 0;
  // the lane's column list of a sensor: consecutive pupil columns from its first entry, with
  // their weights (0 past the list's end); the next sensor's list is loaded while this one's
  // rows are summed
  int2 ce[kAdjKI];
  {
    const int2* e0 = g.tab + g.tab_off[l] + (int64_t)xl * kAdjKI;
#pragma unroll
    for (int k = 0; k < kAdjKI; ++k) ce[k] = e0[k];
  }
  for (int s = 0; s < p.n_sensors; ++s) {
    float wc[kAdjKI];
    int cf = 0, ncol = 0;
#pragma unroll
    for (int k = 0; k < kAdjKI; ++k) {
      const bool ok = xin && ce[k].x >= 0;
      if (k == 0) cf = ok ? ce[k].x : 0;
      wc[k] = ok ? __int_as_float(ce[k].y) : 0.0f;
      if (__builtin_amdgcn_ballot_w64(ok) != 0) ncol = k + 1;  // wave-uniform
    }
    if (s + 1 < p.n_sensors) {
      const int2* e1 = g.tab + g.tab_off[(int64_t)(s + 1) * nl + l] + (int64_t)xl * kAdjKI;
#pragma unroll
      for (int k = 0; k < kAdjKI; ++k) ce[k] = e1[k];
    }
    const DevSensor S = cload(p.sen, s);
    const DevAffine A = cload(p.aff, (int64_t)s * nl + l);
    const float* gs = gb + S.pupil_off;
    const int npup = S.n_pup;
    // pupil rows whose taps can reach the wave's rows, every periodic image (FP64, the
    // candidate rule of the taps kernel: one index of slack on each side)
    const double by = A.by0 + stepd * A.dby;
    int m_lo, m_hi;
    image_range(A.ay, by, L.ny, L.inv_ny, npup, y0, y0 + nrows - 1, L.boundary, m_lo, m_hi);
    int r_lo = 0x7FFFFFFF, r_hi = -1;
    for (int m = m_lo; m <= m_hi; ++m) {
      int lo, hi;
      const double base = (double)m * (double)L.ny;
      cand_range(A.inv_ay, by, base + y0, base + y0 + nrows - 1, npup, lo, hi);
      if (lo <= hi) {
        r_lo = min(r_lo, lo);
        r_hi = max(r_hi, hi);
      }
    }
    if (r_hi < r_lo || ncol == 0) continue;  // wave-uniform: no contribution
    const int nr = r_hi - r_lo + 1;
    if (nr <= kG2MaxPR) {
      // forward row taps of those pupil rows, relative to y0
      if (lane < nr) {
        const double v = fma(A.ay, (double)(r_lo + lane), A.by0) + stepd * A.dby;
        const Tap t = make_tap(v, L.ny, L.inv_ny, L.boundary, 1);
        rtap[lane] = make_float4(__int_as_float(t.i0 - y0), __int_as_float(t.i1 - y0), t.w0,
                                 t.w1);
      }
      wave_sync();
      int cq[kAdjKI];
#pragma unroll
      for (int q = 0; q < kAdjKI; ++q) cq[q] = min(cf + q, npup - 1);
      const float* gr0 = gs + (int64_t)r_lo * npup;
      // chunks of kG2Chunk pupil rows: every load of a chunk in flight before its sums (double
      // buffering the chunks measured slower: the registers cost more occupancy than it hid)
      for (int j0 = 0; j0 < nr; j0 += kG2Chunk) {
        float v[kG2Chunk][kAdjKI];
#pragma unroll
        for (int jj = 0; jj < kG2Chunk; ++jj) {
          const float* gr = gr0 + (int64_t)min(j0 + jj, nr - 1) * npup;
#pragma unroll
          for (int q = 0; q < kAdjKI; ++q) v[jj][q] = q < ncol ? gr[cq[q]] : 0.0f;
        }
#pragma unroll
        for (int jj = 0; jj < kG2Chunk; ++jj) {
          if (j0 + jj >= nr) break;
          float t = 0.0f;
#pragma unroll
          for (int q = 0; q < kAdjKI; ++q)
            if (q < ncol) t = fmaf(wc[q], v[jj][q], t);
          const float4 tp = rtap[j0 + jj];  // wave-uniform (broadcast)
          const int r0 = __builtin_amdgcn_readfirstlane(__float_as_int(tp.x));
          const int r1 = __builtin_amdgcn_readfirstlane(__float_as_int(tp.y));
          if (r0 >= 0 && r0 < nrows)
            acc[r0 * kWave + lane] = fmaf(tp.z, t, acc[r0 * kWave + lane]);
          if (r1 >= 0 && r1 < nrows)
            acc[r1 * kWave + lane] = fmaf(tp.w, t, acc[r1 * kWave + lane]);
        }
      }
      wave_sync();  // the next sensor rewrites the taps
    } else {
      // the wave's rows take pupil rows from two periodic images: each layer row walks its
      // own list
      const int2* rows = g.tab + g.tab_off[(int64_t)s * nl + l] + (int64_t)L.nx * kAdjKI;
      for (int yy = 0; yy < nrows; ++yy) {
        float a = 0.0f;
#pragma unroll
        for (int k = 0; k < kAdjKI; ++k) {
          const int2 e = rows[(int64_t)(y0 + yy) * kAdjKI + k];
          if (e.x < 0) break;
          const float* gr = gs + (int64_t)e.x * npup;
          float t = 0.0f;
#pragma unroll
          for (int q = 0; q < kAdjKI; ++q)
            if (q < ncol) t = fmaf(wc[q], gr[min(cf + q, npup - 1)], t);
          a = fmaf(__int_as_float(e.y), t, a);
        }
        acc[yy * kWave + lane] += a;
      }
    }
  }
  if (xin) {
    float* out = g.grad + (int64_t)b * p.layer_stride + L.offset + x;
    for (int yy = 0; yy < nrows; ++yy)
      out[(int64_t)(y0 + yy) * L.nx] = acc[yy * kWave + lane] * L.weight;
  }
}

__global__ __launch_bounds__(kBlock) void zero_kernel(float* x, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) x[i] = 0.0f;
}

template <int NS>
static hipError_t launch_adj(AdjParams a, bool clear_grad, bool clear, hipStream_t st) {
  // atomic mode accumulates into the gradient; gather mode into the phase-gradient images
  // (cleared by the first of the launches that add into them)
  hipError_t e = hipSuccess;
  if (clear) {
    float* z = a.gpsi ? a.gpsi : a.grad_layers;
    const int64_t n = a.gpsi ? a.f.pupil_per_real * a.f.batch : a.f.layer_stride * a.f.batch;
    const int zb = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 8192);
    hipLaunchKernelGGL(zero_kernel, dim3(zb > 0 ? zb : 1), dim3(kBlock), 0, st, z, n);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // the gather writes every grid pixel; the rest of the gradient buffer (gaps between the
  // grids inside the stride) is cleared only when there is such a gap
  if (clear && a.gpsi && clear_grad) {
    const int64_t ng = a.f.layer_stride * a.f.batch;
    const int zg = (int)std::min<int64_t>((ng + kBlock - 1) / kBlock, 8192);
    hipLaunchKernelGGL(zero_kernel, dim3(zg > 0 ? zg : 1), dim3(kBlock), 0, st, a.grad_layers,
                       ng);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
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

int adj_lds_bytes(int ns, int n_layers, int n_pix, bool gather) {
  return adj_lds_layout(ns, n_layers, n_pix, gather).total;
}

hipError_t launch_adjoint_gather(const FwdParams& f, const float* gpsi, float* grad,
                                 const int32_t* blk_start, hipStream_t st) {
  GatherParams g;
  g.f = f;
  g.gpsi = gpsi;
  g.grad = grad;
  for (int l = 0; l <= f.n_layers; ++l) g.blk_start[l] = blk_start[l];
  const int64_t blocks = (int64_t)blk_start[f.n_layers] * f.batch;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(wfs_adjoint_gather_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, g);
  return hipGetLastError();
}

hipError_t launch_adjoint_gather_tab(const FwdParams& f, const float* gpsi, float* grad,
                                     int2* tab, const AdjSeg* segs, int n_segs, int max_n,
                                     const int64_t* tab_off, const int32_t* blk_start,
                                     hipStream_t st) {
  if (n_segs == 0) return hipSuccess;
  GatherTabParams g;
  g.f = f;
  g.gpsi = gpsi;
  g.grad = grad;
  g.tab = tab;
  g.segs = segs;
  g.tab_off = tab_off;
  for (int l = 0; l <= f.n_layers; ++l) g.blk_start[l] = blk_start[l];
  hipLaunchKernelGGL(wfs_adjoint_taps_kernel, dim3((max_n + kBlock - 1) / kBlock, n_segs),
                     dim3(kBlock), 0, st, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t blocks = (int64_t)blk_start[f.n_layers] * f.batch;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(wfs_adjoint_gather_tab_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st,
                     g);
  return hipGetLastError();
}

int adj_tab_rows() { return kG2TH; }

// FFT-path sensors: one wave per spectrum chunk (fft_adjoint_chunk_m), after the clear of the
// phase-gradient images and before the gather
__global__ __launch_bounds__(kBlock) void wfs_adjoint_fft_kernel(AdjParams ap, int lds_per_wave) {
  extern __shared__ __align__(16) char smem[];
  const int w = threadIdx.x >> 6;
  fft_adjoint_wave(ap, blockIdx.x * kWavesPerBlock + w, smem + w * lds_per_wave);
}

int fft_adj_wave_lds_bytes(int n_fft, int n_pix) { return fft_adj_wave_lds_bytes_impl(n_fft, n_pix); }

hipError_t launch_adjoint_fft(const AdjParams& a, int lds_per_wave, hipStream_t st) {
  const int64_t tasks = (int64_t)a.f.fft.per_real * a.f.batch;
  if (tasks == 0) return hipSuccess;
  const int64_t blocks = (tasks + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(wfs_adjoint_fft_kernel, dim3((unsigned)blocks), dim3(kBlock),
                     lds_per_wave * kWavesPerBlock, st, a, lds_per_wave);
  return hipGetLastError();
}

hipError_t launch_adjoint(const AdjParams& a, int ns, bool clear_grad, bool clear,
                          hipStream_t st) {
  switch (ns) {
    case 2: return launch_adj<2>(a, clear_grad, clear, st);
    case 3: return launch_adj<3>(a, clear_grad, clear, st);
    case 4: return launch_adj<4>(a, clear_grad, clear, st);
    case 5: return launch_adj<5>(a, clear_grad, clear, st);
    case 6: return launch_adj<6>(a, clear_grad, clear, st);
    case 7: return launch_adj<7>(a, clear_grad, clear, st);
    case 8: return launch_adj<8>(a, clear_grad, clear, st);
    case 9: return launch_adj<9>(a, clear_grad, clear, st);
    case 10: return launch_adj<10>(a, clear_grad, clear, st);
    case 11: return launch_adj<11>(a, clear_grad, clear, st);
    case 12: return launch_adj<12>(a, clear_grad, clear, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace wfs
