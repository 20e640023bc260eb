// Lag-domain ("OTF") path of the Shack-Hartmann spot model: device functions shared by the
// forward and adjoint kernels.  One 64-lane wavefront handles one subaperture at a time.
//
// The paper's sensor turns the residual phase into X/Y slopes
// (Sec. 2.7); our reading forms the spot as |DFT_N(E)|^2 of the zero-padded subaperture field,
// convolves it with the sodium-profile kernel, shifts, bins and takes the centre of gravity.
// Because the field has n_sub x n_sub support and N >= 2 n_sub, the DFT of the spot is
// exactly c N^2 times the field's autocorrelation A[k] = sum_m E[m] conj(E[m+k]) on the
// (2 n_sub - 1)^2 lags, and binning after the fftshift is, in the Fourier domain, a
// multiplication by s(kx) s(ky) (s(k) = (-1)^k sum_{d<b} e^{2 pi i k d / N}) followed by
// folding the lags modulo n_pix.  So the binned image is
//     B[q] = c Re sum_{K} P[K] e^{2 pi i K.q / n_pix},
//     P[K] = sum_{k = K mod n_pix, half plane} w_k A[k] Kel[k] s(kx) s(ky),
// (w = 1 on the ky = 0 row, 2 above it, using A[-k] = conj A[k]) which needs n_sub^2 complex
// multiply-adds per row pair instead of two N x N transforms, and no N x N array at all.
// The result equals the FFT definition up to rounding; the FP64 oracle checks it.
#pragma once

#include "wfs_common.h"
#include "wfs_project.h"

namespace wfs {

// ------------------------------------------------------------------------------------------
// Lag-domain path
// ------------------------------------------------------------------------------------------

__host__ __device__ constexpr int otf_pitch(int n) { return n | 1; }

template <int NS, int LP = kOtfLagParts>
struct Otf {
  static constexpr int kJobs = NS * (NS + 1) / 2;  // row pairs (dy, r), dy >= 0
  static constexpr int kLags = 2 * NS - 1;         // dx = -(NS-1) .. NS-1
  static constexpr int kParts = LP;                // passes over the lag row
  static constexpr int kChunk = (kLags + kParts - 1) / kParts;  // lag columns per pass
  // odd LDS pitches (float2) of the field rows and of the partial lag rows: lanes reading
  // different rows of E, or writing their own partial row, fall on distinct bank pairs
  static constexpr int kEP = otf_pitch(NS);
  static constexpr int kPS = otf_pitch(kChunk);
  static constexpr int kRounds = (kJobs + kWave - 1) / kWave;
  static constexpr int kJobsPerRound = (kJobs + kRounds - 1) / kRounds;
  // one round (n_sub <= 10): partial-row slots grouped by pairs of lag rows (dy, NS - 1 - dy),
  // NS + 1 slots a pair (the middle row of an odd NS pairs with itself and leaves slots free)
  static constexpr int kPairs = (NS + 1) / 2;
  static constexpr int kSlots = kRounds == 1 ? kPairs * (NS + 1) : kJobsPerRound;
};

// Partial-row slots of one round (the LDS layout's `part` region).
__host__ __device__ constexpr int otf_part_rows(int ns) {
  return (ns * (ns + 1) / 2 + kWave - 1) / kWave == 1
             ? ((ns + 1) / 2) * (ns + 1)
             : (ns * (ns + 1) / 2 + ((ns * (ns + 1) / 2 + kWave - 1) / kWave) - 1) /
                   ((ns * (ns + 1) / 2 + kWave - 1) / kWave);
}

// Per-wave LDS layout (bytes), shared with the host sizing code:
//   E [n_sub][pitch] float2 (pitch = n_sub rounded up to odd) | AW [n_sub][2 n_sub - 1]
//   float2 (weighted lag sums) |
//   union( taps [n_layers][2 n_sub] Tap (fused gather and adjoint only),
//          partial lag rows (one round, one pass over the lag row at a time:
//          [jobs][ceil((2 n_sub - 1) / lag passes) rounded up to odd] float2),
//          P (later B) + Z (after the last round) ) |
//   tables: s(k) [2 n_sub - 1] float2, twiddles [n_pix] float2
// With a staged footprint (foot_floats > 0) the field stage also lays out, from offset 0
// (E, AW, the union and the tables are free until the field is formed): stencil entries
// [n_layers][2 n_sub] FootTap (12 bytes) | the footprint [foot_floats] float (first holding
// the window origins, [n_layers][2] int).  The tables are then copied in after the window
// has been read.
struct OtfLds {
  int e_off, stab_off, wtab_off, aw_off, taps_off, part_off, p_off, z_off, b_off;
  int fw_off, fp_off, total;
};

__host__ __device__ inline OtfLds otf_lds_layout(int ns, int n_layers, int n_pix,
                                                 bool with_taps = true, int foot_floats = 0,
                                                 int lag_parts = kOtfLagParts) {
  OtfLds o;
  const int jobs = otf_part_rows(ns), lags = 2 * ns - 1, np2 = n_pix * n_pix;
  o.e_off = 0;
  o.aw_off = ns * otf_pitch(ns) * 8;
  const int u0 = (o.aw_off + ns * lags * 8 + 15) & ~15;
  const int taps = 2 * ns * n_layers * 16;
  const int part = jobs * otf_pitch((lags + lag_parts - 1) / lag_parts) * 8;
  o.taps_off = u0;
  o.part_off = u0;
  o.p_off = u0;  // the fold writes P after the last round has read its partial rows
  o.z_off = o.p_off + np2 * 8;
  o.b_off = o.p_off;  // B overwrites P: the image's second pass reads only Z
  int end = o.z_off + np2 * 8;
  if (o.p_off + 1024 > end) end = o.p_off + 1024;  // matrix-core image: 16 x 16 floats
  if (u0 + part > end) end = u0 + part;
  if (with_taps && u0 + taps > end) end = u0 + taps;
  o.stab_off = (end + 7) & ~7;
  o.wtab_off = o.stab_off + lags * 8;
  end = o.wtab_off + n_pix * 8;
  o.fw_off = 0;
  o.fp_off = (2 * ns * n_layers * 12 + 15) & ~15;
  const int fpb = 4 * (foot_floats > 2 * n_layers ? foot_floats : 2 * n_layers);
  if (foot_floats > 0 && o.fp_off + fpb > end) end = o.fp_off + fpb;
  o.total = (end + 15) & ~15;
  return o;
}

template <int NS>
__device__ __forceinline__ void job_of(int j, int& dy, int& r) {
  int d = 0;
  while (j >= NS - d) {
    j -= NS - d;
    ++d;
  }
  dy = d;
  r = j;
}

template <int NS>
__device__ __forceinline__ int job_base(int dy) {
  return dy * NS - (dy * (dy - 1)) / 2;
}

// Row-pair job of partial-row slot j in the one-round layout (false: a free slot).
template <int NS>
__device__ __forceinline__ bool slot_job(int j, int& dy, int& r) {
  const int q = j / (NS + 1), t = j - q * (NS + 1), nA = NS - q;
  if (t < nA) {
    dy = q;
    r = t;
    return true;
  }
  dy = NS - 1 - q;
  r = t - nA;
  return dy != q;
}

// Tap of a given layer for the lanes of one half-wave: the layer parameters are wave-uniform
// (scalar loads), two layers per pass (lanes 0-31 and 32-63).
__device__ __forceinline__ Tap tap_of(const DevLayer& L, const DevAffine& A, bool row, int idx,
                                      double stepd) {
  if (!row) {
    const double u = fma(A.ax, (double)idx, A.bx0) + stepd * A.dbx;
    return make_tap(u, L.nx, L.inv_nx, L.boundary, 1);
  }
  const double v = fma(A.ay, (double)idx, A.by0) + stepd * A.dby;
  return make_tap(v, L.ny, L.inv_ny, L.boundary, L.nx);
}

// Sodium-profile entry of the frame at time step `step` (wave-uniform): its first peak and the
// peak count, or no peaks when the plan has no profile table (single Gaussians).
struct NaEntry {
  const float4* pk;
  int n;
};

__device__ __forceinline__ NaEntry na_entry(const FwdParams& p, int64_t step) {
  NaEntry e;
  e.n = 0;
  e.pk = nullptr;
  if (p.na_entries > 0) {
    const int64_t k = step % (int64_t)p.na_entries;
    e.pk = p.na_tab + (k < 0 ? k + p.na_entries : k) * p.na_peaks;
    e.n = p.na_peaks;
  }
  return e;
}

// Sodium transfer function at the lag whose projection on the elongation direction is `proj`
// (lag units), times `scale`: the subaperture's single Gaussian exp(-alpha proj^2), or, with
// a profile entry, sum_j w_j exp(-2 pi^2 sigma_j^2 t^2) e^{-2 pi i dh_j t}, t = gam proj
// (peak j widened by gam sigma_j and shifted by gam dh_j FFT pixels per unit lag, Sec. 2.7).
__device__ __forceinline__ float2 elong_tf(const DevSubap& sb, const NaEntry& el, float proj,
                                           float scale) {
  if (el.n == 0 || sb.gam == 0.0f)
    return make_float2(__expf(-sb.alpha * proj * proj) * scale, 0.0f);
  const float t = sb.gam * proj;
  float kr = 0.0f, ki = 0.0f;
  for (int j = 0; j < el.n; ++j) {
    const float4 q = el.pk[j];  // (2 pi^2 sigma_h^2, dh, w, 0)
    const float m = q.z * __expf(-q.x * t * t);
    float turns = q.y * t;
    turns -= rintf(turns);
    float sn, cs;
    sincos_rev(turns, &sn, &cs);
    kr = fmaf(m, cs, kr);
    ki = fmaf(-m, sn, ki);
  }
  return make_float2(kr * scale, ki * scale);
}

// Phase in turns subtracted at local pixel (row r, column c) of a subaperture: the half-pixel
// centring ramp and the sensor's tip-tilt (both linear in the pixel index).
__device__ __forceinline__ float field_ramp(const DevSensor& S, int r, int c) {
  return fmaf((float)c, S.ramp_x, (float)r * S.ramp_y);
}

// Where the lag-domain field stage gets the phase (a compile-time choice, so that each kernel
// only holds the registers of its own path).
constexpr int kFieldGather = 0;  // bilinear stencils straight from the layers, per pixel
constexpr int kFieldPhase = 1;   // the projection kernel's phase buffer p.phase_in
constexpr int kFieldFoot = 2;    // the subaperture's layer footprint, staged in LDS

// One axis of a bilinear stencil for the staged footprint: the weights of make_tap (same
// arithmetic, bit for bit) and the first tap's grid index, wrapped into [0, n) on a periodic
// grid, the floor of the clamped coordinate on a zero-boundary grid.  The window of a
// subaperture starts at the index of its pupil pixel with the smaller coordinate.
__device__ __forceinline__ float2 foot_axis_tap(double c, int32_t n, double inv_n,
                                                int32_t boundary, int* i0_out) {
  if (boundary == 0) {
    const double cw = c - (double)n * floor(c * inv_n);
    const double f0 = floor(cw);
    int32_t i0 = (int32_t)f0;
    const float f = (float)(cw - f0);
    if (i0 >= n) i0 -= n;
    if (i0 < 0) i0 += n;
    *i0_out = i0;
    return make_float2(1.0f - f, f);
  }
  const double cc = fmin(fmax(c, -4.0), (double)n + 4.0);
  const double f0 = floor(cc);
  const int32_t i0 = (int32_t)f0;
  const float f = (float)(cc - f0);
  const bool ok0 = i0 >= 0 && i0 < n;
  const bool ok1 = i0 + 1 >= 0 && i0 + 1 < n;
  *i0_out = i0;
  return make_float2(ok0 ? 1.0f - f : 0.0f, ok1 ? f : 0.0f);
}

// Stencil entry of one pupil column (w0, w1, byte offset of the window-relative column) or
// row (w0 * layer weight, w1 * layer weight, byte offset of the window row) of one layer.
struct FootTap {
  float w0, w1;
  int32_t k;
};

// Phase of the lane's pixels from a footprint staged in LDS (Sec. 2.2, inside the spot wave):
//   1. the origin of each layer window along each axis (the window holds the layer pixels the
//      subaperture's stencils can touch; bounds fixed per sensor and layer), then every
//      stencil entry (lane per layer, axis and pupil index), both from the launch's table of
//      stencil entries (FP64 coordinates, computed once per frame for every pupil index);
//   2. each lane loads up to two window columns (all rows; the column descriptors are read
//      at the start), then the window goes to LDS over the origins table;
//   3. each pixel sums its stencils from LDS, layer by layer.
// Indices, weights and the order of every floating-point operation are those of the
// projection kernel, so the phase (and everything after it) matches the split schedule bit
// for bit.
template <int NS>
__device__ __forceinline__ void foot_phase(const FwdParams& p, const DevSensor& S,
                                           const DevSubap& sb, int sid, int b, int frame,
                                           char* wsm, const OtfLds& lo, float* ph) {
  constexpr int NPIX = NS * NS;
  constexpr int PPL = (NPIX + kWave - 1) / kWave;
  constexpr int ROWS = NS + 2;                   // window rows loaded per column
  constexpr int SLOT = otf_pitch(ROWS);          // LDS floats per window column
  constexpr int TPL = 2 * NS;       // stencil entries per layer: columns, then rows
  constexpr int LPP = kWave / TPL;  // layers per pass
  const int lane = lane_id();
  const int nl = p.n_layers;
  FootTap* tab = reinterpret_cast<FootTap*>(wsm + lo.fw_off);  // [nl][2 NS]
  int* forg = reinterpret_cast<int*>(wsm + lo.fp_off);         // [nl][2], until step 2
  float* fp = reinterpret_cast<float*>(wsm + lo.fp_off);
  const int64_t fbase = (int64_t)sid * nl;
  FootCol fc[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int pc = lane + k * kWave;
    fc[k] = pc < S.foot_ncols ? p.foot_cols[S.foot_cols_off + pc]
                              : FootCol{0, 1, 1, 0, 0, 0, 0, 0};
  }
  // 1. window origins, lane per (layer, axis): the first tap of the pupil index with the
  //    smaller coordinate; then the stencil entries, lane per (layer, axis, pupil index),
  //    from the launch's entry table of this frame
  const FootEnt* ent =
      p.foot_ent + (int64_t)frame * p.foot_ent_per_frame + S.foot_ent_off;  // [nl][2][n_pup]
  for (int e = lane; e < 2 * nl; e += kWave) {
    const int i0 = (e & 1) ? sb.a * NS : sb.b * NS;
    const double a = p.foot_axis[fbase * 2 + e].a;
    forg[e] = ent[e * S.n_pup + (a >= 0.0 ? i0 : i0 + NS - 1)].i0;
  }
  wave_sync();
  {
    const int lp = lane / TPL, j = lane - lp * TPL;
    const int axis = j >= NS ? 1 : 0;
    const int idx = axis ? sb.a * NS + (j - NS) : sb.b * NS + j;
    for (int l0 = 0; l0 < nl; l0 += LPP) {
      const int l = l0 + lp;
      if (lp < LPP && l < nl) {
        const FootEnt E = ent[(2 * l + axis) * S.n_pup + idx];
        FootTap t;
        t.w0 = E.w0;  // rows: the projection kernel's ry.w0 * wl
        t.w1 = E.w1;
        t.k = E.k;  // byte offset in the window
        tab[l * TPL + j] = t;
      }
    }
  }
  // 2. window columns (32-bit byte offsets: the plan keeps every layer below 2^30 floats),
  // all ROWS rows of a column slot (rows fh.. of a slot are loaded and stored but never
  // read).  Rows leave the grid (wrap, or clamp on a zero-boundary grid) only for windows at
  // a grid edge: when no lane's window does, the rows are plain strides and each column is
  // ROWS unpredicated loads and stores at immediate offsets.
  const char* lay_b = reinterpret_cast<const char*>(p.layers + (int64_t)b * p.layer_stride);
  float val[2][ROWS];
  int cbase[2], oyv[2];
  bool edge = false;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const FootCol& C = fc[k];
    const int l = C.lj >> 8, j = C.lj & 255;
    const int ox = forg[2 * l];
    oyv[k] = forg[2 * l + 1];
    int col = ox + j;
    if (C.boundary == 0) col -= col >= C.nx ? C.nx : 0;
    else col = min(max(col, 0), C.nx - 1);
    cbase[k] = C.offset + col;
    edge = edge || (C.fh > 0 && (oyv[k] < 0 || oyv[k] + ROWS > C.ny));
  }
  if (__builtin_amdgcn_ballot_w64(edge) == 0) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      // a lane without a column reads the realisation's first float ROWS times
      const bool has = fc[k].fh > 0;
      uint32_t off = has ? (uint32_t)(cbase[k] + oyv[k] * fc[k].nx) * 4u : 0u;
      const uint32_t stride = has ? (uint32_t)fc[k].nx * 4u : 0u;
#pragma unroll
      for (int i = 0; i < ROWS; ++i) {
        val[k][i] = *reinterpret_cast<const float*>(lay_b + off);
        off += stride;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const FootCol& C = fc[k];
      const bool periodic = C.boundary == 0;
#pragma unroll
      for (int i = 0; i < ROWS; ++i) {
        int rr = oyv[k] + i;
        if (rr >= C.ny) rr = periodic ? rr - C.ny : C.ny - 1;
        rr = max(rr, 0);
        val[k][i] = i < C.fh ? ld_idx(reinterpret_cast<const float*>(lay_b),
                                       (uint32_t)(cbase[k] + rr * C.nx))
                             : 0.0f;
      }
    }
  }
  wave_sync();  // the window overwrites the origins
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (fc[k].fh > 0) {
      float* dst = fp + fc[k].dst;
#pragma unroll
      for (int i = 0; i < ROWS; ++i) dst[i] = val[k][i];
    }
  }
  wave_sync();
  // 3. stencils, in the projection kernel's chunks of layers (a last partial chunk is padded
  // with zero-weight repeats of the last layer, as there)
  int pr[PPL], pc[PPL];
  float psi[PPL];
#pragma unroll
  for (int i = 0; i < PPL; ++i) {
    const int q = min(lane + i * kWave, NPIX - 1);
    pr[i] = q / NS;
    pc[i] = q - pr[i] * NS;
    psi[i] = 0.0f;
  }
  auto stencil = [&](int l, bool pad) {
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      const FootTap cx = tab[l * TPL + pc[i]];
      const FootTap ry = tab[l * TPL + NS + pr[i]];
      // column-major window: the next row is the next float, the next column a slot later
      const float* w0p =
          reinterpret_cast<const float*>(reinterpret_cast<const char*>(fp) + (ry.k + cx.k));
      const float v00 = w0p[0], v10 = w0p[1];
      const float v01 = w0p[SLOT], v11 = w0p[SLOT + 1];
      const float r0v = fmaf(cx.w0, v00, cx.w1 * v01);
      const float r1v = fmaf(cx.w0, v10, cx.w1 * v11);
      const float wy0 = pad ? 0.0f : ry.w0, wy1 = pad ? 0.0f : ry.w1;
      psi[i] = fmaf(wy0, r0v, fmaf(wy1, r1v, psi[i]));
    }
  };
  int l0 = 0;
  for (; l0 + kProjLC <= nl; l0 += kProjLC) {
#pragma unroll
    for (int jj = 0; jj < kProjLC; ++jj) stencil(l0 + jj, false);
  }
  if (l0 < nl) {
#pragma unroll
    for (int jj = 0; jj < kProjLC; ++jj) stencil(min(l0 + jj, nl - 1), l0 + jj >= nl);
  }
#pragma unroll
  for (int i = 0; i < PPL; ++i) ph[i] = psi[i] * S.kappa;
}

// Fills the wave's E region with the subaperture field E[r][c] = A exp(i(psi - pi (r+c)/N)),
// and the wave's copies of the sensor's lag-phase and twiddle tables.  All per-subaperture
// values (S, sb, sid, b) are wave-uniform.  FIELD says where the phase comes from.
template <int NS, int FIELD>
__device__ __forceinline__ void otf_field(const FwdParams& p, const DevSensor& S,
                                          const DevSubap& sb, int sid, int b, double stepd,
                                          char* wsm, const OtfLds& lo, int frame = 0) {
  constexpr int NPIX = NS * NS;
  constexpr int PPL = (NPIX + kWave - 1) / kWave;  // pixels per lane
  const int lane = lane_id();
  const int nl = p.n_layers;
  // small per-sensor tables -> LDS (consumed by the lag sums and the image stages); with a
  // staged footprint they overlay the window, so they follow it
  auto tables = [&]() {
    float2* st = reinterpret_cast<float2*>(wsm + lo.stab_off);
    float2* wt = reinterpret_cast<float2*>(wsm + lo.wtab_off);
    for (int k = lane; k < 2 * NS - 1 + S.n_pix; k += kWave) {
      if (k < 2 * NS - 1) st[k] = p.stab[S.stab_off + k];
      else wt[k - (2 * NS - 1)] = p.wtab[S.wtab_off + k - (2 * NS - 1)];
    }
  };
  if constexpr (FIELD != kFieldFoot) tables();
  if constexpr (FIELD == kFieldFoot) {
    float ph[PPL];
    foot_phase<NS>(p, S, sb, sid, b, frame, wsm, lo, ph);
    wave_sync();  // E and the tables overlay the stencil entries and the window just read
    tables();
    float2* E = reinterpret_cast<float2*>(wsm + lo.e_off);
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      const int q = lane + i * kWave;
      if (q < NPIX) {
        const int r = q / NS, c = q - r * NS;
        const uint8_t amp = p.mask[S.mask_off + (sb.a * NS + r) * S.n_pup + sb.b * NS + c];
        float turns = fmaf(ph[i], 0.15915494309189535f, -field_ramp(S, r, c));
        turns -= rintf(turns);
        float sn, cs;
        sincos_rev(turns, &sn, &cs);
        E[r * Otf<NS>::kEP + c] = amp ? make_float2(cs, sn) : make_float2(0.0f, 0.0f);
      }
    }
    wave_sync();
  } else if constexpr (FIELD == kFieldPhase) {  // the projection kernel already wrote kappa psi
    const float* ph = p.phase_in + (int64_t)b * p.phase_per_real + S.phase_off +
                      (int64_t)sb.v * NPIX;
    float2* E = reinterpret_cast<float2*>(wsm + lo.e_off);
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      const int q = lane + i * kWave;
      if (q < NPIX) {
        const int r = q / NS, c = q - r * NS;
        const uint8_t amp = p.mask[S.mask_off + (sb.a * NS + r) * S.n_pup + sb.b * NS + c];
        float turns = fmaf(ph[q], 0.15915494309189535f, -field_ramp(S, r, c));
        turns -= rintf(turns);
        float sn, cs;
        sincos_rev(turns, &sn, &cs);
        E[r * Otf<NS>::kEP + c] = amp ? make_float2(cs, sn) : make_float2(0.0f, 0.0f);
      }
    }
    wave_sync();
  } else {
    // amplitude of this lane's pixels (issued early)
    uint8_t amp[PPL];
    int pr[PPL], pc[PPL];
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      const int q = lane + i * kWave;
      const int qq = q < NPIX ? q : 0;
      pr[i] = qq / NS;
      pc[i] = qq - pr[i] * NS;
      amp[i] = q < NPIX ? p.mask[S.mask_off + (sb.a * NS + pr[i]) * S.n_pup + sb.b * NS + pc[i]]
                        : 0;
    }
    // taps: [l][0..NS) columns, [l][NS..2NS) rows
    Tap* taps = reinterpret_cast<Tap*>(wsm + lo.taps_off);
    {
      const int g = lane >> 5, j = lane & 31;
      const bool row = j >= NS;
      const int idx = row ? sb.a * NS + (j - NS) : sb.b * NS + j;
      for (int l0 = 0; l0 < nl; l0 += 2) {
        const int l1 = l0 + 1 < nl ? l0 + 1 : l0;
        const DevLayer L0 = cload(p.lay, l0), L1 = cload(p.lay, l1);
        const DevAffine A0 = cload(p.aff, sid * nl + l0), A1 = cload(p.aff, sid * nl + l1);
        const Tap t = tap_of(g ? L1 : L0, g ? A1 : A0, row, idx, stepd);
        if (j < 2 * NS && (g == 0 || l0 + 1 < nl)) taps[(l0 + g) * 2 * NS + j] = t;
      }
    }
    wave_sync();
    // projection: every load of a 4-layer chunk for all of the lane's pixels in flight at once
    const float* lay_b = p.layers + (int64_t)b * p.layer_stride;
    float psi[PPL];
#pragma unroll
    for (int i = 0; i < PPL; ++i) psi[i] = 0.0f;
    // chunks of LC layers with every load in flight; layers past the end repeat the last one
    // with weight 0 (no predicated register arrays)
    constexpr int LC = 5;
    for (int l0 = 0; l0 < nl; l0 += LC) {
      float v[LC][PPL][4];
      Tap cx[LC][PPL], ry[LC][PPL];
      float wl[LC];
#pragma unroll
      for (int jj = 0; jj < LC; ++jj) {
        const int l = min(l0 + jj, nl - 1);
        const DevLayer L = cload(p.lay, l);
        wl[jj] = l0 + jj < nl ? L.weight : 0.0f;
        const float* g = lay_b + L.offset;
#pragma unroll
        for (int i = 0; i < PPL; ++i) {
          cx[jj][i] = taps[l * 2 * NS + pc[i]];
          ry[jj][i] = taps[l * 2 * NS + NS + pr[i]];
          v[jj][i][0] = ld_idx(g, (uint32_t)(ry[jj][i].i0 + cx[jj][i].i0));
          v[jj][i][1] = ld_idx(g, (uint32_t)(ry[jj][i].i0 + cx[jj][i].i1));
          v[jj][i][2] = ld_idx(g, (uint32_t)(ry[jj][i].i1 + cx[jj][i].i0));
          v[jj][i][3] = ld_idx(g, (uint32_t)(ry[jj][i].i1 + cx[jj][i].i1));
        }
      }
#pragma unroll
      for (int jj = 0; jj < LC; ++jj) {
#pragma unroll
        for (int i = 0; i < PPL; ++i) {
          const Tap& a = cx[jj][i];
          const Tap& r = ry[jj][i];
          const float val = r.w0 * fmaf(a.w0, v[jj][i][0], a.w1 * v[jj][i][1]) +
                            r.w1 * fmaf(a.w0, v[jj][i][2], a.w1 * v[jj][i][3]);
          psi[i] = fmaf(wl[jj], val, psi[i]);
        }
      }
    }
    float2* E = reinterpret_cast<float2*>(wsm + lo.e_off);
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      const int q = lane + i * kWave;
      // phase in turns, reduced to [-1/2, 1/2] before the sincos
      float turns =
          fmaf(psi[i], S.kappa * 0.15915494309189535f, -field_ramp(S, pr[i], pc[i]));
      turns -= rintf(turns);
      float sn, cs;
      sincos_rev(turns, &sn, &cs);
      if (q < NPIX)
        E[pr[i] * Otf<NS>::kEP + pc[i]] = amp[i] ? make_float2(cs, sn) : make_float2(0.0f, 0.0f);
    }
    wave_sync();
  }
}

// Lag sums of one round of row-pair jobs for the lag columns [IX0, IX0 + W) (held in the
// partial-row region, kChunk columns per job), times the elongation and binning factors:
// AW[dy][dx] (+)= w_dy Kel(dx, dy) s(dx) s(dy) sum_r part, lane per lag (dy, dx).
template <int NS, int LP, int IX0, int W>
__device__ __forceinline__ void otf_lagsum(const DevSensor& S, const DevSubap& sb,
                                           const NaEntry& el, char* wsm, const OtfLds& lo,
                                           int j0) {
  constexpr int NL = Otf<NS>::kLags;
  const int lane = lane_id();
  const float2* part = reinterpret_cast<const float2*>(wsm + lo.part_off);
  const float2* stab = reinterpret_cast<const float2*>(wsm + lo.stab_off);
  float2* aw = reinterpret_cast<float2*>(wsm + lo.aw_off);
  // weighted lag value at (dy, column ix) from the row sum a
  auto weigh = [&](int dy, int ix, float2 a) {
    const int dx = ix - (NS - 1);
    const float2 sx = stab[ix], sy = stab[dy + NS - 1];
    const float proj = fmaf((float)dx, sb.ex, (float)dy * sb.ey);
    const float2 k = elong_tf(sb, el, proj, dy == 0 ? 1.0f : 2.0f);
    const float sr = sx.x * sy.x - sx.y * sy.y, si = sx.x * sy.y + sx.y * sy.x;
    const float tr = sr * k.x - si * k.y;
    const float ti = sr * k.y + si * k.x;
    return make_float2(a.x * tr - a.y * ti, a.x * ti + a.y * tr);
  };
  if constexpr (Otf<NS>::kRounds == 1) {
    // every job in one round: lane per (pair of lag rows dy and NS-1-dy, column).  The two
    // rows hold NS - dy and dy + 1 jobs, in NS + 1 consecutive slots, so each lane sums
    // exactly NS + 1 partial rows.
    constexpr int NQ = (NS + 1) / 2;
    static_assert(NQ * W <= kWave, "one pass");
    const int q = lane / W, k = lane - q * W;
    if (q < NQ) {
      const int dyA = q, dyB = NS - 1 - q, nA = NS - q;
      const float2* rows = part + q * (NS + 1) * Otf<NS, LP>::kPS + k;  // the pair's slots
      float2 a = make_float2(0.0f, 0.0f), bsum = make_float2(0.0f, 0.0f);
#pragma unroll
      for (int t = 0; t <= NS; ++t) {
        const bool inA = t < nA;
        const float2 v = rows[t * Otf<NS, LP>::kPS];
        if (inA) {
          a.x += v.x;
          a.y += v.y;
        } else {
          bsum.x += v.x;
          bsum.y += v.y;
        }
      }
      aw[dyA * NL + IX0 + k] = weigh(dyA, IX0 + k, a);
      if (dyB != dyA) aw[dyB * NL + IX0 + k] = weigh(dyB, IX0 + k, bsum);
    }
    wave_sync();
    return;
  }
  const int j1 = j0 + Otf<NS>::kJobsPerRound;
#pragma unroll
  for (int o0 = 0; o0 < NS * W; o0 += kWave) {
    const int o = o0 + lane;
    if (o < NS * W) {
      const int dy = o / W, k = o - dy * W, ix = IX0 + k;
      const int base = job_base<NS>(dy);
      const int r0 = max(0, j0 - base), r1 = min(NS - dy, j1 - base);
      float2 a = make_float2(0.0f, 0.0f);
#pragma unroll
      for (int r = 0; r < NS; ++r) {
        if (r >= r0 && r < r1) {
          const float2 v = part[(base + r - j0) * Otf<NS, LP>::kPS + k];
          a.x += v.x;
          a.y += v.y;
        }
      }
      float2 t = weigh(dy, ix, a);
      const int oa = dy * NL + ix;
      if (j0 > 0) {
        const float2 prev = aw[oa];
        t.x += prev.x;
        t.y += prev.y;
      }
      aw[oa] = t;
    }
  }
  wave_sync();
}

// One round of autocorrelation row-pair jobs [j0, j0 + jobs per round), lag columns
// [IX0, IX0 + W): lane per (dy, r) forms sum_c E[r][c] conj(E[r+dy][c+dx]) for those dx in
// registers and leaves them in the partial-row region, then the lag sums over r.  Taking the
// lag row in kOtfLagParts passes keeps the registers and the LDS region at that fraction of a
// row per job, at the same number of multiply-adds.
template <int NS, int LP, int IX0, int W>
__device__ __forceinline__ void otf_corr_part(const DevSensor& S, const DevSubap& sb,
                                              const NaEntry& el, char* wsm, const OtfLds& lo,
                                              int j0) {
  const int lane = lane_id();
  const float2* E = reinterpret_cast<const float2*>(wsm + lo.e_off);
  float2* part = reinterpret_cast<float2*>(wsm + lo.part_off);
  int dy = 0, r = 0;
  bool ok;
  if constexpr (Otf<NS>::kRounds == 1) {
    ok = lane < Otf<NS>::kSlots && slot_job<NS>(lane, dy, r);
  } else {
    const int j = j0 + lane;
    ok = lane < Otf<NS>::kJobsPerRound && j < Otf<NS>::kJobs;
    if (ok) job_of<NS>(j, dy, r);
  }
  if (ok) {
    // the second row stays in registers; the first streams from LDS one pixel at a time
    float2 e2[NS];
#pragma unroll
    for (int c = 0; c < NS; ++c) e2[c] = E[(r + dy) * Otf<NS>::kEP + c];
    float2 acc[W];
#pragma unroll
    for (int k = 0; k < W; ++k) acc[k] = make_float2(0.0f, 0.0f);
#pragma unroll
    for (int c1 = 0; c1 < NS; ++c1) {
      const float2 e1 = E[r * Otf<NS>::kEP + c1];
#pragma unroll
      for (int c2 = 0; c2 < NS; ++c2) {
        // E[r][c1] conj(E[r+dy][c2]) -> lag dx = c2 - c1, column c2 - c1 + NS - 1
        const int k = c2 - c1 + NS - 1 - IX0;
        if (k >= 0 && k < W) {
          float2& a = acc[k];
          a.x = fmaf(e1.x, e2[c2].x, fmaf(e1.y, e2[c2].y, a.x));
          a.y = fmaf(e1.y, e2[c2].x, fmaf(-e1.x, e2[c2].y, a.y));
        }
      }
    }
#pragma unroll
    for (int k = 0; k < W; ++k) part[lane * Otf<NS, LP>::kPS + k] = acc[k];
  }
  wave_sync();
  otf_lagsum<NS, LP, IX0, W>(S, sb, el, wsm, lo, j0);
}

template <int NS, int LP, int IX0 = 0>
__device__ __forceinline__ void otf_corr_round(const DevSensor& S, const DevSubap& sb,
                                               const NaEntry& el, char* wsm, const OtfLds& lo,
                                               int j0) {
  constexpr int NL = Otf<NS, LP>::kLags, CW = Otf<NS, LP>::kChunk;
  constexpr int W = IX0 + CW <= NL ? CW : NL - IX0;
  otf_corr_part<NS, LP, IX0, W>(S, sb, el, wsm, lo, j0);
  if constexpr (IX0 + W < NL) otf_corr_round<NS, LP, IX0 + W>(S, sb, el, wsm, lo, j0);
}

// Fold modulo n_pix: P[Ky][Kx] = sum over lags (dy, dx) = (Ky, Kx) mod n_pix of AW, lane per K.
template <int NS>
__device__ __forceinline__ void otf_fold(const DevSensor& S, char* wsm, const OtfLds& lo) {
  constexpr int NL = Otf<NS>::kLags;
  const int lane = lane_id();
  const int np = S.n_pix, np2 = np * np;
  const float2* aw = reinterpret_cast<const float2*>(wsm + lo.aw_off);
  float2* P = reinterpret_cast<float2*>(wsm + lo.p_off);
  if (np == 8) {  // the common 8 x 8 image: lane = K, trip counts known (same sums, same order)
    const int Ky = lane >> 3, Kx = lane & 7, dx0 = Kx - 8 * ((Kx + NS - 1) >> 3);
    float2 acc = make_float2(0.0f, 0.0f);
#pragma unroll
    for (int a = 0; a < (NS + 7) / 8; ++a) {
      const int dy = Ky + 8 * a;
#pragma unroll
      for (int c = 0; c < (NL + 7) / 8 + 1; ++c) {
        const int dx = dx0 + 8 * c;
        if (dy < NS && dx < NS) {
          const float2 v = aw[dy * NL + dx + NS - 1];
          acc.x += v.x;
          acc.y += v.y;
        }
      }
    }
    P[lane] = acc;
    wave_sync();
    return;
  }
  for (int K = lane; K < np2; K += kWave) {
    const int Ky = fdiv(K, np, S.inv_npix), Kx = K - Ky * np;
    const int dx0 = Kx - np * fdiv(Kx + NS - 1, np, S.inv_npix);
    float2 acc = make_float2(0.0f, 0.0f);
    for (int dy = Ky; dy < NS; dy += np) {
      for (int dx = dx0; dx < NS; dx += np) {
        const float2 v = aw[dy * NL + dx + NS - 1];
        acc.x += v.x;
        acc.y += v.y;
      }
    }
    P[K] = acc;
  }
  wave_sync();
}

typedef float v4f_t __attribute__((ext_vector_type(4)));

// B[q] = c Re sum_K P[K] W^{K.q} on the matrix cores (n_pix <= 8), as two real 16 x 16 x 16
// products of four v_mfma_f32_16x16x4f32 each:  [Zr | Zi] = [Pr | Pi] F1 with
// F1 = [[C, S], [-S, C]], then B = c F2 [Zr ; Zi] with F2 = [C | -S] (C, S: cosine and sine of
// 2 pi (k n mod n_pix) / n_pix, per-sensor tables).  Operand layout: lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; accumulator i of lane l holds D[4 (l/16) + i][l%16].
// The intermediate [Zr | Zi] goes through LDS over the P and Z regions.
__device__ __forceinline__ void otf_image_mfma(const FwdParams& p, const DevSensor& S,
                                               char* wsm, const OtfLds& lo) {
  const int lane = lane_id();
  const int np = S.n_pix;
  const int r16 = lane & 15, kq = lane >> 4;
  const float* F1 = p.mtab + S.mtab_off;
  const float* F2 = F1 + 256;
  const float2* P = reinterpret_cast<const float2*>(wsm + lo.p_off);
  float* D = reinterpret_cast<float*>(wsm + lo.p_off);  // [16][16]
  float* B = reinterpret_cast<float*>(wsm + lo.b_off);
  float a[4], f[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = kq + 4 * s, kk = k & 7;
    const float2 v = (r16 < np && kk < np) ? P[r16 * np + kk] : make_float2(0.0f, 0.0f);
    a[s] = k < 8 ? v.x : v.y;
    f[s] = F1[k * 16 + r16];
  }
  v4f_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], f[s], acc, 0, 0, 0);
  wave_sync();
#pragma unroll
  for (int i = 0; i < 4; ++i) D[(4 * kq + i) * 16 + r16] = acc[i];
  wave_sync();
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = kq + 4 * s;
    f[s] = F2[r16 * 16 + k];
    a[s] = k < 8 ? D[k * 16 + (r16 & 7)] : D[(k - 8) * 16 + 8 + (r16 & 7)];
  }
  acc = (v4f_t){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(f[s], a[s], acc, 0, 0, 0);
  wave_sync();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int qy = 4 * kq + i;
    if (qy < np && r16 < np) B[qy * np + r16] = S.flux_c * acc[i];
  }
  wave_sync();
}

// B[q] = c Re sum_K P[K] W^{K.q}, separable through Z[Ky][qx] (W = e^{2 pi i / n_pix}).
__device__ __forceinline__ void otf_image(const FwdParams& p, const DevSensor& S, char* wsm,
                                          const OtfLds& lo) {
  if (S.mtab_off >= 0) {
    otf_image_mfma(p, S, wsm, lo);
    return;
  }
  const int lane = lane_id();
  const int np = S.n_pix, np2 = np * np;
  const float2* P = reinterpret_cast<const float2*>(wsm + lo.p_off);
  float2* Z = reinterpret_cast<float2*>(wsm + lo.z_off);
  float* B = reinterpret_cast<float*>(wsm + lo.b_off);
  const float2* wt = reinterpret_cast<const float2*>(wsm + lo.wtab_off);
  for (int t = lane; t < np2; t += kWave) {
    const int Ky = fdiv(t, np, S.inv_npix), qx = t - Ky * np;
    float2 z = make_float2(0.0f, 0.0f);
    int idx = 0;
#pragma unroll 8
    for (int Kx = 0; Kx < np; ++Kx) {
      const float2 a = P[Ky * np + Kx];
      const float2 w = wt[idx];
      z.x = fmaf(a.x, w.x, fmaf(-a.y, w.y, z.x));
      z.y = fmaf(a.x, w.y, fmaf(a.y, w.x, z.y));
      idx += qx;
      if (idx >= np) idx -= np;
    }
    Z[t] = z;
  }
  wave_sync();
  for (int t = lane; t < np2; t += kWave) {
    const int qy = fdiv(t, np, S.inv_npix), qx = t - qy * np;
    float v = 0.0f;
    int idx = 0;
#pragma unroll 8
    for (int Ky = 0; Ky < np; ++Ky) {
      const float2 z = Z[Ky * np + qx];
      const float2 w = wt[idx];
      v = fmaf(z.x, w.x, fmaf(-z.y, w.y, v));
      idx += qy;
      if (idx >= np) idx -= np;
    }
    B[t] = S.flux_c * v;
  }
  wave_sync();
}

// Noise and centre-of-gravity sums over the binned image (sum B', sum x B', sum y B'), one
// pixel per lane: pixels 2j and 2j + 1 share Philox block j (words x, y and z, w); every lane
// returns the wave totals.
struct Cog {
  float s0, sx, sy;
};

__device__ __forceinline__ Cog cog_sums(const FwdParams& p, const DevSensor& S, int sid, int b,
                                        int v, int64_t step, const float* B) {
  const int lane = lane_id();
  const int np = S.n_pix, np2 = np * np;
  const float half = 0.5f * (float)(np - 1);
  float s0 = 0.0f, sx = 0.0f, sy = 0.0f;
  const bool noisy = S.noisy && p.noise_on;
  for (int q = lane; q < np2; q += kWave) {
    float bq = B[q];
    if (noisy) {
      const uint4 ctr = make_uint4((uint32_t)(q >> 1), (uint32_t)v,
                                   ((uint32_t)b << 8) | (uint32_t)sid, (uint32_t)step);
      const uint4 w = philox4x32_10(ctr, p.seed_lo, p.seed_hi);
      const bool odd = (q & 1) != 0;
      add_noise_one(bq, odd ? w.z : w.x, odd ? w.w : w.y, S.read_noise);
    }
    const int y = fdiv(q, np, S.inv_npix), x = q - y * np;
    s0 += bq;
    sx = fmaf((float)x - half, bq, sx);
    sy = fmaf((float)y - half, bq, sy);
  }
  Cog c;
  c.s0 = wave_sum(s0);
  c.sx = wave_sum(sx);
  c.sy = wave_sum(sy);
  return c;
}

// Slopes (0 when the flux is not positive) and the flux of subaperture v, of frame `frame`
// of a multi-frame launch (outputs [frame][B][...]).
__device__ __forceinline__ void write_slopes(const FwdParams& p, const DevSensor& S, int b,
                                             int v, const Cog& c, int frame = 0) {
  if (lane_id() == 0) {
    const bool ok = c.s0 > 0.0f;
    const int64_t fb = (int64_t)frame * p.batch + b;
    float* out = p.slopes + fb * p.n_slopes + S.slope_off;
    out[v] = ok ? c.sx / c.s0 : 0.0f;
    out[S.n_valid + v] = ok ? c.sy / c.s0 : 0.0f;
    if (p.aux) p.aux[fb * p.n_valid_total + S.aux_off + v] = c.s0;
  }
}

// Binned noise-free (or noisy) image of one subaperture into the wave's B region (LP: passes
// over each lag row, which sets the partial-row region of the layout `lo`).
template <int NS, int FIELD, int LP = kOtfLagParts>
__device__ __forceinline__ void otf_spot(const FwdParams& p, const DevSensor& S,
                                         const DevSubap& sb, int sid, int b, int64_t step,
                                         char* wsm, const OtfLds& lo, int frame = 0) {
  otf_field<NS, FIELD>(p, S, sb, sid, b, (double)step, wsm, lo, frame);
  const NaEntry el = na_entry(p, step);
#pragma unroll
  for (int rd = 0; rd < Otf<NS>::kRounds; ++rd)
    otf_corr_round<NS, LP>(S, sb, el, wsm, lo, rd * Otf<NS>::kJobsPerRound);
  otf_fold<NS>(S, wsm, lo);
  otf_image(p, S, wsm, lo);
}

template <int NS, int FIELD, int LP = kOtfLagParts>
__device__ void otf_subap(const FwdParams& p, int t, int64_t step, char* wsm, int frame = 0) {
  int b, sid, v;
  t = __builtin_amdgcn_readfirstlane(t);  // wave-uniform: per-subaperture data in SGPRs
  task_of(p.otf, t, b, sid, v);
  const DevSensor S = cload(p.sen, sid);
  const DevSubap sb = cload(p.sub, S.valid_off + v);
  // the layout the host sized the launch with: the per-pixel gather holds its stencil taps
  // in the union (the sensor tables follow whichever of taps, partial rows and image is last)
  const OtfLds lo = otf_lds_layout(NS, p.n_layers, S.n_pix, FIELD == kFieldGather,
                                   FIELD == kFieldFoot ? S.foot_floats : 0, LP);
  otf_spot<NS, FIELD, LP>(p, S, sb, sid, b, step, wsm, lo, frame);
  const Cog c = cog_sums(p, S, sid, b, v, step + p.noise_dstep,
                         reinterpret_cast<const float*>(wsm + lo.b_off));
  write_slopes(p, S, b, v, c, frame);
  wave_sync();
}

}  // namespace wfs
