// Internal device tables and kernel parameter blocks of libwfs (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wfs {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kBlock = 256;        // threads per workgroup of every sensor kernel
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kMaxLayers = 64;
constexpr int kMaxSensors = 64;
constexpr int kOtfMaxNsub = 12;    // lag-domain path: subapertures up to 12 x 12 pixels
constexpr int kFftMaxNsub = 64;    // FFT path: fields up to 64 x 64 pixels
constexpr int kFftMaxN = 128;      // FFT path: transforms up to 128 points per axis
constexpr int kOtfLagParts = 2;    // lag-domain path: default passes over each lag row

enum Path : int32_t { kPathOtf = 0, kPathFft = 1 };

struct DevLayer {
  int64_t offset;
  int32_t nx, ny;
  float weight;
  int32_t boundary;  // 0 periodic, 1 zero outside
  double inv_nx, inv_ny;
};

// Continuous layer coordinates of pupil pixel (column i, row j) of sensor s seen through
// layer l at time step k:  u = ax*i + bx0 + k*dbx,  v = ay*j + by0 + k*dby.
struct DevAffine {
  double ax, bx0, dbx;
  double ay, by0, dby;
  double inv_ax, inv_ay;  // 1 / ax, 1 / ay (adjoint gather)
};

struct DevSensor {
  int32_t n_sa, n_sub, n_fft, bin;
  int32_t n_pix, n_pup, n_valid, valid_off;  // valid_off: first row of the subap table
  int32_t slope_off, aux_off, mask_off, path;
  int32_t noisy, elong, phase_off, pad5;  // phase_off: offset in the phase buffer
  float kappa;       // lambda_ref / lambda
  float flux_c;      // F_ph / (n_fft^2 n_sub^2)
  float read_noise;  // electrons rms
  float ramp_x;      // turns per pixel column subtracted from the field phase: the half-pixel
                     // centring ramp 1 / (2 n_fft) less the sensor's tip, tilt_x dx / lambda
                     // (its constant part over a subaperture does not change the spot)
  int32_t stab_off;  // first entry of this sensor's lag-phase table s(k), k = -(n_sub-1)..
  int32_t wtab_off;  // first entry of this sensor's n_pix-point twiddle table
  float inv_npix;    // 1 / n_pix
  int32_t subidx_off;  // first entry of this sensor's [n_sa][n_sa] valid-index table (-1 = unused)
  int32_t foot_ncols;  // staged footprint: layer columns of one subaperture, all layers
  float inv_nsub;    // 1 / n_sub
  int32_t mtab_off;  // matrix-core image operands (n_pix <= 8), -1: vector path
  int32_t pupil_off;  // offset of this sensor's [n_pup][n_pup] image in a pupil-frame buffer
  int32_t foot_cols_off;  // first entry of this sensor's footprint-column table
  int32_t foot_floats;    // footprint floats of one subaperture, all layers
  float ramp_y;           // the same per pixel row: 1 / (2 n_fft) - tilt_y dx / lambda
  int32_t fft_part_off;   // FFT path with several spectrum chunks: first float of this sensor's
                          // partial images in one realisation's part of the partial buffer
  int32_t fft_cnt_off;    // first of this sensor's chunk counters in one realisation's part
  int32_t fft_adj_off;    // adjoint: first float of this sensor's chunk partials (n_sub^2 per
                          // chunk) in one realisation's part of the adjoint partial buffer
  int32_t foot_ent_off;   // staged footprint: first of this sensor's stencil entries in a
                          // frame's table, [n_layers][2 axes][n_pup]
};

// Staged-footprint field: the layer pixels one subaperture's bilinear stencils can touch,
// per layer a [rows][cols] window (bounds fixed per sensor and layer) at a running offset.
constexpr int kFootMaxCols = 2 * kWave;  // columns summed over layers: two per lane

// One axis of one (sensor, layer) for the staged footprint: coordinate c = a i + b0 + k db of
// pupil index i at step k on a grid of n points (1/n, boundary), and how a stencil entry is
// stored: weights times `weight`, window index koff + kmul * (tap - window origin).
// ent_off: first entry of this axis (one per pupil index) in a frame's stencil-entry table.
struct FootAxis {
  double a, b0, db, inv_n;
  int32_t n, boundary, kmul, koff;
  float weight;
  int32_t ent_off;
  int32_t pad[2];
};

// Bilinear stencil of one pupil index along one axis at one step, as the staged footprint
// uses it: the two weights times the axis weight (0 for taps off a zero-boundary grid), the
// byte offset of the first tap in the window of the pupil index's subaperture, and the first
// tap's grid index (wrapped into [0, n) on a periodic grid, the floor of the clamped
// coordinate on a zero-boundary one; the window origin when the index is the subaperture's
// one of smallest coordinate).
struct FootEnt {
  float w0, w1;
  int32_t k, i0;
};

// One window column of one sensor's footprint: where it is read and where it goes.
struct FootCol {
  int32_t offset, nx, ny, boundary;  // layer start (floats), grid, 0 periodic / 1 zero
  int32_t fw, fh, dst, lj;           // window columns and rows, first LDS float, layer << 8 | column
};

struct DevSubap {
  int32_t a, b;   // subaperture row and column
  float alpha;    // 2 pi^2 sigma_px^2 / n_fft^2 (0: no elongation)
  float ex, ey;   // unit elongation direction
  int32_t v;      // index among the sensor's valid subapertures
  float gam;      // sodium-profile scale |b| / (H^2 p_fft n_fft): a peak dh metres above the
                  // focus shifts by gam dh per unit lag along e (0: no elongation)
  int32_t pad1;
};

constexpr int kMaxNaPeaks = 8;  // peaks per entry of a sodium-profile table

// Flat list of sensors served by one launch (one lag-domain template instance plus the FFT
// path); task t of realisation b is subaperture (t - start[k]) of sensor ids[k].
struct TaskTable {
  int32_t n;                  // sensors in the list
  int32_t per_real;           // tasks per realisation
  int32_t ids[kMaxSensors];
  int32_t start[kMaxSensors + 1];
  // optional: task r of a realisation is (sensor, subaperture) order[r] (the sensors'
  // subapertures interleaved by pupil position); null: sensor after sensor as above
  const int2* order;
};

struct FwdParams {
  const float* layers;
  int64_t layer_stride;
  const DevLayer* lay;
  const DevAffine* aff;  // [n_sensors][n_layers]
  const DevSensor* sen;
  const DevSubap* sub;
  const uint8_t* mask;
  const float2* stab;
  const float2* wtab;
  const float* mtab;        // per sensor: the 16x16 operands of the two image products
  const int64_t* step_dev;  // read when use_dev_step
  int64_t step;
  int32_t use_dev_step;
  int32_t n_layers;
  int32_t n_sensors;
  int32_t batch;
  uint32_t seed_lo, seed_hi;
  int32_t noise_on;         // 0 in the adjoint's recompute
  int32_t noise_dstep;      // noise counter step = time step + noise_dstep (calibration chunks)
  // sodium profile: [na_entries][na_peaks] peaks (2 pi^2 sigma_h^2, dh, normalised weight, 0);
  // the frame at step k uses entry k mod na_entries; na_entries = 0: single Gaussians
  const float4* na_tab;
  int32_t na_entries, na_peaks;
  float* slopes;
  int32_t n_slopes;
  float* aux;
  int32_t n_valid_total;
  // schedule
  int32_t otf_blocks;       // blocks serving the lag-domain tasks
  int32_t fft_blocks;       // blocks serving FFT tasks (one subaperture each), launched first
  int32_t xcd_remap;
  int32_t lds_per_wave;     // bytes (lag-domain waves, or a quarter of an FFT workgroup)
  int32_t lds_per_wave_otf; // bytes when the launch holds no FFT-path blocks
  int32_t otf_from_phase;   // lag-domain field source: 0 gather, 1 phase_in (split), 2 footprint
  int32_t lag_parts;        // split field: passes over each lag row (2 or 3; sets its LDS)
  int32_t fft_inline;       // host side: FFT-path blocks in the same launch as the others
  // FFT path: partial binned images of the spectrum chunks ([B][fft_part_per_real] floats)
  // and per-subaperture chunk counters ([B][fft_cnt_per_real], zero between launches)
  float* fft_part;
  int32_t* fft_cnt;
  int64_t fft_part_per_real;
  int32_t fft_cnt_per_real;
  TaskTable otf;
  TaskTable fft;
  // projection blocks of one realisation: (first pupil row | column strip << 16, sensor)
  const int2* proj_desc;
  int32_t proj_per_real;
  const int32_t* subidx;     // valid-subaperture index of (sensor, a, b), -1 if not valid
  const float* phase_in;     // split mode: phase of every valid pixel (kappa applied), or null
  int64_t phase_per_real;    // floats per realisation in the phase buffer
  int64_t pupil_per_real;    // floats per realisation in a pupil-frame buffer (sum n_pup^2)
  // pipelined frames: the spot launch of step k also projects step k + 1 into phase_out
  int32_t proj_blocks;       // projection blocks interleaved with the spot blocks (0: none)
  int32_t proj_lds;          // bytes of LDS a projection block needs
  float* phase_out;
  // staged footprint: per (sensor, layer) {cols, rows, first float, 0}, the per-axis
  // coordinate tables and the window columns; frames of one launch
  const int4* foot;
  const FootAxis* foot_axis;   // [n_sensors][n_layers][2] (x, y)
  const FootCol* foot_cols;    // per sensor: its window columns, layer by layer
  int32_t n_frames;
  // stencil entries of every frame of a footprint launch, [frame][entries of one frame]
  const FootEnt* foot_ent;
  int32_t foot_ent_per_frame;
};

// A plan-owned second stream with fork/join events: a launch that holds FFT-path blocks runs
// them there, concurrently with the lag-domain blocks on the caller's stream.
struct SideStream {
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

struct AdjParams {
  FwdParams f;              // forward tables (noise off)
  const float* grad_slopes; // [B][n_slopes]
  const float* fwd_slopes;  // or null
  const float* fwd_aux;     // or null
  float* grad_layers;       // [B][layer_stride]
  float* gpsi;              // gather mode: [B][pupil_per_real] phase-gradient images, or null
  float* fft_adj_part;      // FFT path: [B][fft_adj_per_real] per-chunk phase-gradient partials
  int64_t fft_adj_per_real;
};

// Table-driven gather of the layer gradient.  For a (sensor, layer, axis) whose inverse
// stencil lists fit kAdjKI entries, entry k of layer index i is (pupil index, weight) of the
// k-th pupil index whose forward taps touch i (increasing pupil index; pupil index -1 ends a
// shorter list).  One segment per (sensor, layer, axis) of such layers: its first entry, its
// layer size and who it is.
constexpr int kAdjKI = 4;
struct AdjSeg {
  int64_t off;
  int32_t n, s, l, axis;
};

struct GatherTabParams {
  FwdParams f;
  const float* gpsi;         // [B][pupil_per_real] pupil-frame images, kappa applied
  float* grad;               // [B][layer_stride]
  int2* tab;                 // the lists (written by the taps kernel for the call's step)
  const AdjSeg* segs;
  const int64_t* tab_off;    // [n_sensors][n_layers]: first entry of the column lists of
                             // (s, l), the row lists follow nx * kAdjKI later; -1: not tabled
  int32_t blk_start[kMaxLayers + 1];  // first block of each layer within a realisation
};

// Gather of the layer gradient from the phase gradients: thread per layer pixel.
struct GatherParams {
  FwdParams f;
  const float* gpsi;         // [B][pupil_per_real] pupil-frame images, kappa applied
  float* grad;               // [B][layer_stride]
  int32_t blk_start[kMaxLayers + 1];  // first block of each layer within a realisation
};

}  // namespace wfs
