/*
 * wfs.h -- C ABI of the MI355X Shack-Hartmann wavefront-sensor library (libwfs.so).
 *
 * The operations follow the closed-loop description of Arcidiacono et al., "The numerical
 * simulation tool for the MAORY multiconjugate adaptive optics system":
 *   - Sec. 2.1: turbulence is a set of static phase screens at given altitudes (frozen flow);
 *   - Sec. 2.2: the wavefront of each guide star is the geometric projection of the screens
 *     along its direction, the laser guide star being at a finite distance (cone effect);
 *   - Sec. 2.7: the wavefront-sensor module turns the residual phase (open loop minus DM) into
 *     X/Y slopes; the slopes times the control matrix give differential coefficients added to
 *     the mirror (pure integrator); the sodium layer enters at this level;
 *   - Sec. 1: the sensors are Shack-Hartmann (six LGS, three NGS in MAORY).
 *
 * Conventions shared by every call
 *   - All data buffers are DEVICE pointers owned by the caller (float32, row-major).
 *   - Every call that takes a `stream` (a hipStream_t; NULL = the default stream) is
 *     asynchronous on it and never synchronises the device, except wfs_plan, wfs_plan_destroy,
 *     wfs_plan_na_profile and wfs_plan_tune (and wfs_tlse, include/wfs_tlse.h).  No call allocates device memory
 *     except wfs_plan, wfs_plan_na_profile, recon_apply (first use on a stream, or a larger
 *     problem than that stream has seen; never while the stream is capturing a graph) and
 *     wfs_adjoint (first use of a plan).
 *   - Arguments are validated on the host before anything is launched: a bad argument returns
 *     WFS_EINVAL and launches nothing.  A failed HIP call returns WFS_EDEVICE.  The message of
 *     the last failure on the calling thread is returned by wfs_last_error().
 *   - Layer buffer: one realisation occupies `layer_stride` floats; layer l of realisation b
 *     starts at layers + b*layer_stride + desc[l].offset and is a [ny][nx] row-major grid.
 *   - Slopes: per realisation, sensors in plan order; per sensor the x slopes of its valid
 *     subapertures (row-major subaperture order) followed by their y slopes.  Units: binned
 *     detector pixels (wfs_plan_info gives radians per pixel).  Layout [B][n_slopes].
 *   - Concurrent calls on one plan must use one stream (they share the plan's device state).
 */
#ifndef WFS_H
#define WFS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  WFS_OK = 0,
  WFS_EINVAL = -1,       /* bad argument or shape; nothing launched                   */
  WFS_ENOMEM = -2,       /* device allocation failed                                  */
  WFS_EDEVICE = -3,      /* a HIP runtime call or a launch failed                     */
  WFS_EUNSUPPORTED = -4  /* valid request outside what the kernels implement          */
};

/* Plan flags (wfs_plan `flags`). */
#define WFS_FLAG_FORCE_OTF (1u << 0)    /* every sensor on the lag-domain (autocorrelation) path */
#define WFS_FLAG_FORCE_FFT (1u << 1)    /* every sensor on the FFT path (needs no elongation)     */
#define WFS_FLAG_NO_XCD_REMAP (1u << 2) /* keep the hardware block order (no per-XCD grouping)    */
#define WFS_FLAG_FUSED (1u << 3)        /* spot waves gather the layers per pixel (no projection
                                           pass; frames one after the other); default: a
                                           projection kernel first, and wfs_forward_steps as
                                           one staged-footprint launch where every lag-domain
                                           sensor allows it                               */
#define WFS_FLAG_ADJOINT_ATOMIC (1u << 4) /* wfs_adjoint scatters with FP32 atomics instead of
                                           the deterministic gather                        */
#define WFS_FLAG_SPLIT (1u << 5)        /* projection kernel first, never the staged footprint
                                           (same bits as the footprint field)             */
#define WFS_FLAG_FOOTPRINT (1u << 6)    /* staged footprint for single frames too (one launch
                                           per wfs_forward); ignored where a sensor cannot
                                           stage its footprint; with FFT-path sensors only
                                           frames in a row take it (wfs_forward_steps)    */

/* `step` value meaning "read the step from the plan's device-resident counter". */
#define WFS_STEP_DEVICE (-1)

typedef struct wfs_plan_s* wfs_plan_t; /* opaque; owns device tables until wfs_plan_destroy */

/* One turbulence layer or deformable-mirror grid (Sec. 2.1 screens; Sec. 2.7 DM). */
typedef struct {
  int64_t offset;  /* element offset of the [ny][nx] grid inside one realisation         */
  int32_t nx, ny;  /* grid size in pixels                                                */
  double pitch_m;  /* pixel pitch (m)                                                    */
  double alt_m;    /* altitude above the telescope (m)                                   */
  double vx_mps;   /* frozen-flow wind (m/s); the screen is sampled at X - v t           */
  double vy_mps;
  float weight;    /* +1 turbulence, -1 DM (residual = open loop - DM)                   */
  int32_t boundary;/* 0 = periodic screen, 1 = zero outside the grid (DM)                */
} wfs_layer_desc;

/* One Shack-Hartmann sensor and its guide star (Sec. 1, Sec. 2.2, Sec. 2.7). */
typedef struct {
  double theta_x_rad, theta_y_rad; /* guide-star direction                                 */
  double src_alt_m;                /* LGS altitude H (cone factor 1 - h/H); INFINITY = NGS */
  double lambda_m;                 /* sensing wavelength                                   */
  double pupil_d_m, obs_d_m;       /* pupil and central-obstruction diameters              */
  int32_t n_sa;                    /* subapertures across the pupil                        */
  int32_t n_sub;                   /* pupil pixels across a subaperture                    */
  int32_t n_fft;                   /* FFT size (zero padding); n_fft >= 2*n_sub            */
  int32_t bin;                     /* detector binning; n_fft % bin == 0                   */
  double valid_frac;               /* subaperture used when lit fraction >= valid_frac     */
  double na_fwhm_m;                /* Gaussian sodium profile FWHM; 0 = no elongation      */
  double launch_x_m, launch_y_m;   /* laser launch position in the pupil                   */
  double photons;                  /* photons per fully lit subaperture per frame;
                                      0 = unit flux and no noise                           */
  double read_noise_e;             /* read noise (electrons rms), used when photons > 0    */
  double tilt_x_rad, tilt_y_rad;   /* extra tip-tilt of this sensor (Sec. 2.3: an NGS WFS
                                      mispositioned by these sky angles): the phase
                                      2 pi (tilt_x x + tilt_y y) / lambda_m at the pupil
                                      pixel centres (x, y) is added to the projected phase;
                                      0 = none                                            */
} wfs_sensor_desc;

/*
 * wfs_plan -- build the geometry tables of a set of sensors looking through a set of layers.
 *   layers[n_layers], sensors[n_sensors]: descriptors (copied).  layer_stride: floats per
 *   realisation in the layer buffer.  batch: realisations per call (B).  lambda_ref_m: the
 *   wavelength at which the layer values are radians of phase.  dt_s: time per step (the
 *   screens are sampled at t = step*dt).  flags: WFS_FLAG_*.  *out receives the plan.
 *   Validation: n_fft % bin == 0, n_fft >= 2*n_sub, grids inside the stride, positive sizes.
 *   Lag-domain sensors (n_sub <= 12) may have different n_sub: each size gets its own spot
 *   launch.  Allocates the device tables, the phase buffers and, where every lag-domain
 *   sensor can stage its footprint, a table of stencil entries for up to 256 frames of one
 *   footprint launch (64 MiB at most).  Synchronises the device (uploads the tables).
 */
int wfs_plan(const wfs_layer_desc* layers, int32_t n_layers, int64_t layer_stride,
             const wfs_sensor_desc* sensors, int32_t n_sensors, int32_t batch,
             double lambda_ref_m, double dt_s, uint32_t flags, wfs_plan_t* out);

/*
 * wfs_plan_info -- sizes of a plan (any output pointer may be NULL).
 *   n_slopes: slopes per realisation; n_valid_total: valid subapertures over all sensors
 *   (length of one realisation's aux row); n_valid_per_sensor[n_sensors];
 *   pix_scale_rad[n_sensors]: radians per binned pixel, bin*lambda/(n_fft*dx).
 */
int wfs_plan_info(wfs_plan_t plan, int32_t* n_slopes, int32_t* n_valid_total,
                  int32_t* n_valid_per_sensor, double* pix_scale_rad);

/*
 * wfs_plan_na_profile -- time-varying, multi-peak sodium profile of the plan's elongated LGS
 *   sensors (Sec. 2.7: the temporal evolution of the sodium layer).  table: host
 *   [n_entries][n_peaks][3] doubles (dh_m, fwhm_m, weight) per peak; the frame at time step k
 *   uses entry k mod n_entries.  A peak dh metres above the LGS altitude H with Gaussian width
 *   fwhm (0 allowed: a thin peak) carries the fraction weight / (sum of the entry's weights)
 *   of the return; a subaperture at baseline b from the launch sees it shifted by
 *   |b| dh / H^2 and widened by |b| sigma / H^2 (radians) along b / |b|, so its transfer
 *   function is sum_j w_j exp(-2 pi^2 sigma_j^2 u^2) exp(-2 pi i mu_j u) in FFT pixels.  The
 *   profile replaces the single Gaussian of na_fwhm_m on every sensor with na_fwhm_m > 0 and
 *   a finite source altitude; other sensors are unaffected.  n_entries = 0 (table NULL)
 *   restores the single Gaussians.  Limits: 1 <= n_peaks <= 8, n_entries <= 2^20; weights
 *   >= 0 with a positive sum per entry, fwhm >= 0, all finite (WFS_EINVAL otherwise).
 *   Synchronises the device; allocates the device copy (a table that fits the plan's current
 *   buffer reuses it; a captured graph reads whatever table is current when it replays).
 */
int wfs_plan_na_profile(wfs_plan_t plan, int32_t n_entries, int32_t n_peaks,
                        const double* table);

/* wfs_plan_path -- which path each sensor runs: 0 = lag-domain (OTF), 1 = FFT. */
int wfs_plan_path(wfs_plan_t plan, int32_t* path_per_sensor);

/* wfs_plan_destroy -- free the plan and its device tables (synchronises the device). */
int wfs_plan_destroy(wfs_plan_t plan);

/*
 * wfs_forward -- slopes of every sensor for every realisation (Sec. 2.2 + Sec. 2.7):
 *   projection of the layers along each guide-star direction (cone factor for the LGS,
 *   frozen-flow shift v*t, periodic/zero boundary), the sensor's tip-tilt offset added,
 *   field A exp(i phase) with a half-pixel centring ramp on each valid n_sub x n_sub
 *   subaperture zero-padded to n_fft, spot |DFT|^2 scaled to `photons`, sodium elongation
 *   along the launch baseline (the sensor's Gaussian, or the plan's sodium-profile entry for
 *   this step, wfs_plan_na_profile),
 *   fftshift and bin x bin binning, Gaussian photon + read noise (Philox4x32-10 keyed by
 *   seed, counters from realisation, sensor, subaperture, pixel pair and step) when the
 *   sensor has photons > 0, and centre of gravity in binned pixels (0 when the flux <= 0).
 *   layers: device [B][layer_stride].  step >= 0, or WFS_STEP_DEVICE.  slopes: device
 *   [B][n_slopes] (written).  aux: device [B][n_valid_total] sum of the binned pixels of
 *   each subaperture, or NULL.  Deterministic (bitwise) for fixed inputs.
 */
int wfs_forward(wfs_plan_t plan, const float* layers, int64_t step, uint64_t seed,
                float* slopes, float* aux, void* stream);

/*
 * wfs_forward_steps -- n_steps consecutive frames, steps step0 .. step0 + n_steps - 1 (or,
 *   with step0 = WFS_STEP_DEVICE, the device counter + 0 .. n_steps - 1; the counter is not
 *   advanced): the same results, bit for bit, as n_steps calls of wfs_forward.  slopes:
 *   device [n_steps][B][n_slopes]; aux: device [n_steps][B][n_valid_total] or NULL.  The
 *   frames run as wfs_plan_schedule's `frames` says (overlapped: projections on a second
 *   stream, forked from and joined to `stream`): with the staged footprint, one launch
 *   covers up to 256 frames (frame k's blocks follow frame k - 1's: no launch gap, no phase
 *   buffer; a small launch before it fills the frames' stencil entries); pipelined, each launch forms the spots of step k and projects the layers for
 *   step k + 1 into the plan's second phase buffer.  Frozen flow (Sec. 2.1) makes every
 *   frame's input known in advance.  Layers must not change during the call.
 */
int wfs_forward_steps(wfs_plan_t plan, const float* layers, int64_t step0, int32_t n_steps,
                      uint64_t seed, float* slopes, float* aux, void* stream);

/*
 * wfs_spots -- the spot stage alone (Sec. 2.7): slopes from a given phase buffer laid out as
 *   wfs_project writes it ([B][sum over sensors of n_valid*n_sub^2], phase in radians at
 *   the sensor wavelength, device memory).  Same noise, outputs and determinism as wfs_forward, which is
 *   wfs_project into a plan-owned buffer followed by this call (or the fused gather).
 */
int wfs_spots(wfs_plan_t plan, const float* phase, int64_t step, uint64_t seed, float* slopes,
              float* aux, void* stream);

/*
 * wfs_plan_schedule -- the launch schedule the plan currently uses (set at creation, changed
 *   by wfs_plan_tune).  field: where wfs_forward's lag-domain waves get the phase, 0 = they
 *   gather the layers per pixel (WFS_FLAG_FUSED), 1 = a projection kernel writes it first
 *   (split), 2 = each wave stages its subaperture's layer footprint in LDS and projects it
 *   itself (one launch, no phase buffer).  frames: how wfs_forward_steps runs, 0 = one
 *   wfs_forward per frame, 1 = pipelined split frames, 2 = one footprint launch for all
 *   frames (FFT-path sensors, which read the projected phase, then run frame by frame on
 *   the plan's second stream beside it), 3 = overlapped split frames (frame k + 1 projected
 *   on a plan-owned stream while frame k's spots run on `stream`; the call forks from and
 *   joins `stream`).  Fields 1 and 2 and frames 0-3 give the same bits;
 *   field 0 its own.  Field 2 for single frames needs a plan without FFT-path sensors.
 *   xcd_remap = 1 when blocks are renumbered so neighbouring tasks share an XCD.
 *   fft_launch (plans with both paths, fields 0 and 1): 0 = the FFT-path blocks run as a
 *   launch of their own on the plan's second stream, concurrently; 1 = they are blocks of
 *   the same launch as the lag-domain blocks (and, pipelined, the next step's projection:
 *   one launch per step).  proj_rows: the projection kernel's tile height, pupil rows per
 *   block (8, 16 or 32 where a block's layer taps fit 32 KiB of LDS; taller blocks share each
 *   column tap among more pixels, shorter ones give more blocks).  lag_passes: the split
 *   field's spot waves form each lag row of the autocorrelation in 2 or 3 passes (3: less LDS
 *   per wave, more waves per CU, a little more arithmetic).  All choices give the same bits.
 *   Any output pointer may be NULL.
 */
int wfs_plan_schedule(wfs_plan_t plan, int32_t* field, int32_t* frames, int32_t* xcd_remap,
                      int32_t* fft_launch, int32_t* proj_rows, int32_t* lag_passes);

/*
 * wfs_plan_set_schedule -- pin a launch schedule (values as wfs_plan_schedule reports them;
 *   -1 keeps a choice).  WFS_EUNSUPPORTED when the plan cannot run it: field 1 or frames 1
 *   or 3 without a phase buffer, field 2 or frames 2 where a lag-domain sensor cannot stage its
 *   footprint, field 2 for single frames with FFT-path sensors, frames 1 or 2 with field 0,
 *   a proj_rows the plan does not offer; WFS_EINVAL for lag_passes other than -1, 2, 3.
 *   Host only; no device work.
 */
int wfs_plan_set_schedule(wfs_plan_t plan, int32_t field, int32_t frames, int32_t xcd_remap,
                          int32_t fft_launch, int32_t proj_rows, int32_t lag_passes);

/*
 * wfs_plan_footprint -- algorithmic read footprint of the projection at time step `step`:
 *   the number of distinct layer pixels (per realisation, all layers and sensors) that the
 *   bilinear stencils of the pixels of valid subapertures touch, and the number of projected
 *   pixels.  Host computation; no device work.
 */
int wfs_plan_footprint(wfs_plan_t plan, int64_t step, int64_t* distinct_layer_pixels,
                       int64_t* phase_pixels);

/*
 * wfs_project -- the projection step alone (Sec. 2.2): phase at the sensor wavelength of
 *   every pixel of every valid subaperture, [B][sum over sensors of n_valid*n_sub^2], per
 *   sensor subaperture-major then row-major pixels; dark pixels hold their projected phase.
 */
int wfs_project(wfs_plan_t plan, const float* layers, int64_t step, float* phase,
                void* stream);

/*
 * wfs_adjoint -- gradient with respect to the layer buffer of a scalar loss, given the
 *   gradient with respect to the noise-free slopes (the adjoint of wfs_forward with noise
 *   off).  Subaperture fields are recomputed from the layers.  fwd_slopes/fwd_aux: the
 *   noise-free forward outputs for the same layers and step (both given, or both NULL: then
 *   they are recomputed).  grad_layers: device [B][layer_stride], overwritten (zero outside
 *   the grids).  By default the phase gradients go through the plan's second phase buffer and
 *   each layer pixel gathers its contributions in a fixed order: bitwise deterministic.  With
 *   WFS_FLAG_ADJOINT_ATOMIC the taps are scattered with FP32 atomics (reproducible to
 *   rounding, not bitwise).  Sensors on the FFT path (large fields) take the gather form
 *   only: with them, WFS_FLAG_ADJOINT_ATOMIC returns WFS_EUNSUPPORTED.  When fwd_slopes and
 *   fwd_aux are NULL and the plan has FFT-path sensors, the noise-free forward runs first
 *   into a plan-owned buffer (allocated on the first call, with the FFT path's chunk shares).
 */
int wfs_adjoint(wfs_plan_t plan, const float* layers, const float* grad_slopes,
                const float* fwd_slopes, const float* fwd_aux, int64_t step,
                float* grad_layers, void* stream);

/* wfs_set_step / wfs_advance_step -- write / add to the plan's device step counter
 * (captured-graph replays read it with step = WFS_STEP_DEVICE). */
int wfs_set_step(wfs_plan_t plan, int64_t step, void* stream);
int wfs_advance_step(wfs_plan_t plan, int64_t delta, void* stream);

/*
 * wfs_plan_tune -- time every launch schedule the plan can run (field, frame schedule incl.
 *   overlapped frames, block
 *   order, projection tile height where the projection kernel runs, lag passes of the split
 *   field's spot waves and, with both paths,
 *   where the FFT-path blocks run) on max(2, iters) frames in a
 *   row from `layers` and keep the fastest (the four fastest of a first pass are timed three more times each); only schedules whose single frames and frames in
 *   a row give the same bits are candidates.  Then, where the split and footprint fields both
 *   fit the kept frame schedule (they share their bits), single frames take the faster.
 *   Honours WFS_FLAG_FUSED / SPLIT / FOOTPRINT.  Synchronises; writes scratch slopes
 *   internally.  On return *best_us holds the time per wfs_forward call of the kept schedule
 *   (may be NULL).
 */
int wfs_plan_tune(wfs_plan_t plan, const float* layers, int32_t iters, double* best_us,
                  void* stream);

/*
 * recon_apply -- reconstructor (control matrix) times slopes, Sec. 2.6-2.7:
 *   C[b][i] = alpha * sum_j R[i][j] S[b][j] + beta * C[b][i],  i < M, j < N, b < B.
 *   R: device [M][N] row-major.  S: device [B][N].  C: device, row b at C + b*ldc
 *   (ldc >= M).  beta = 0 ignores the old C.  A pure integrator a += g R s is
 *   alpha = g, beta = 1 on the DM actuator rows.  B = 1 runs a streaming GEMV, 2 <= B <= 8
 *   the same stream with every realisation at once (16-byte aligned R and S, N % 4 == 0),
 *   larger batches a split-K matrix-core (MFMA) GEMM.  Deterministic.  The split partial sums go to a
 *   library-owned buffer of the calling stream (kept for the life of the process, so graphs
 *   captured with it stay valid); a call that would have to grow that buffer while the stream
 *   is capturing returns WFS_EINVAL (run it once outside the capture first).  Calls on one
 *   stream are ordered; calls on different streams never share a buffer.
 */
int recon_apply(const float* R, int32_t M, int32_t N, const float* S, int32_t B, float* C,
                int64_t ldc, float alpha, float beta, void* stream);

/*
 * recon_apply_noalloc -- recon_apply for callers that cannot allocate device memory (code
 *   under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 *   arguments, operation, layouts and error codes as recon_apply, same kernels; it never
 *   allocates, frees or synchronises.  The split partial sums go to a fixed library array of
 *   2^22 floats (16 MiB) on each GPU, held until the process ends; the split count shrinks to
 *   what it holds, so results may differ from recon_apply's by rounding order only.  Returns
 *   WFS_EINVAL when one split does not fit: M * B > 2^22 for 2 <= B <= 8 and
 *   M * min(B, 16) > 2^22 for larger B (aligned operands), M > 2^22 otherwise.  Every call on one GPU shares the array: calls that overlap
 *   in time on one GPU (different streams, or threads) race and give wrong results; order
 *   them on one stream.  The caller owns R, S and C as for recon_apply.
 */
int recon_apply_noalloc(const float* R, int32_t M, int32_t N, const float* S, int32_t B,
                        float* C, int64_t ldc, float alpha, float beta, void* stream);

/*
 * wfs_calibrate -- interaction-matrix calibration (Sec. 2.5: the chosen modes are pushed
 *   through the sensor model and their slopes recorded, optionally with noise or with a
 *   turbulence screen present, together with the reference slopes).  The modes are single
 *   actuator pokes: actuator j (0 <= j < n_act) is element act_offset + j of a realisation's
 *   layer buffer (a DM grid declared as a layer, so its bilinear interpolation is the influence
 *   function).  With h = plan batch / 2 (the batch must be even), each chunk of h actuators is
 *   one wfs_forward of a batch whose realisation r < h holds actuator j0 + r at +amplitude and
 *   realisation h + r the same actuator at -amplitude, on top of `base` (device
 *   [layer_stride], one realisation: e.g. an on-sky screen; NULL = flat); then row j of `im`
 *   is (s+ - s-) / (2 amplitude).  Every chunk samples the layers at time step `step`, so
 *   all rows share one operating point even when the base screen moves with the wind; chunk c
 *   draws its noise (sensors with photons > 0) with step counter `step` + c, so noise differs
 *   between chunks.  im: device
 *   [n_act][ld_im] (ld_im >= n_slopes): row j = d slopes / d actuator j, i.e. the
 *   interaction matrix transposed.  ref_slopes: device [n_slopes], realisation 0 of an
 *   unpoked batch at `step` (NULL = not wanted).  work: device, at least the number of floats
 *   wfs_calibrate_work returns.  Asynchronous on `stream`; deterministic for fixed inputs.
 */
int wfs_calibrate_work(wfs_plan_t plan, int64_t* work_floats);
int wfs_calibrate(wfs_plan_t plan, const float* base, int64_t act_offset, int32_t n_act,
                  float amplitude, int64_t step, uint64_t seed, float* im, int64_t ld_im,
                  float* ref_slopes, float* work, int64_t work_floats, void* stream);

/*
 * Point-spread functions and Strehl ratios (Sec. 2.8: PSFs at user wavelengths and pixel
 * scales for a constellation of test stars; Strehl ratio from the PSF or, with the Marechal
 * approximation, from the history of the residual wavefront).
 *
 * psf_plan -- test stars at infinity in directions star_theta_xy[2*s], [2*s+1] (rad), seeing
 *   the layers (turbulence +1, DM grids -1: the residual phase) on a full n_pup x n_pup pupil
 *   grid of pitch pupil_d_m / n_pup (pixel centres (i + 1/2 - n_pup/2) dx, amplitude 1 where
 *   obs_d_m/2 <= r <= pupil_d_m/2).  Per wavelength lambda_m[l] the field
 *   A exp(i (lambda_ref/lambda) phi) is zero-padded to n_fft[l] x n_fft[l] (a power of two in
 *   [max(16, n_pup), 4096]; PSF pixel = lambda / (n_fft dx) rad).  Layers as in wfs_plan
 *   (offsets inside layer_stride, periodic or zero boundary, frozen flow at t = step dt_s).
 *   Allocates the plan's device tables and a [n_stars][n_pup][max n_fft] complex work buffer.
 * psf_plan_info -- floats of the PSF buffer (sum over l of n_stars n_fft[l]^2), the first float
 *   of each wavelength's images (psf_offsets[n_lambda]), and the lit pupil pixels.  Any output
 *   may be NULL.
 * psf_accumulate -- adds one frame: psf (device, psf_floats) gets, per wavelength l and star s,
 *   the image [n_fft][n_fft] at psf + psf_offsets[l] + s n_fft^2 of |DFT(field)|^2 / (n_fft^2
 *   n_lit) (unit sum per frame; zero frequency at pixel (n_fft/2, n_fft/2); row = y frequency).
 *   layers: device [layer_stride], one realisation.  phase_var: device double [n_lambda]
 *   [n_stars] or NULL; gets the piston-removed variance over the lit pupil of the phase at
 *   each wavelength (rad^2).  Asynchronous; deterministic.
 * psf_strehl -- after n_frames accumulations: sr_psf[l][s] = the long-exposure image at zero
 *   frequency over the diffraction-limited peak (n_frames n_lit / n_fft^2); sr_marechal[l][s] =
 *   exp(-phase_var[l][s] / n_frames).  Device outputs (float), either may be NULL.
 */
typedef struct psf_plan_s* psf_plan_t;
int psf_plan(const wfs_layer_desc* layers, int32_t n_layers, int64_t layer_stride,
             const double* star_theta_xy, int32_t n_stars, double pupil_d_m, double obs_d_m,
             int32_t n_pup, const double* lambda_m, const int32_t* n_fft, int32_t n_lambda,
             double lambda_ref_m, double dt_s, psf_plan_t* out);
int psf_plan_info(psf_plan_t plan, int64_t* psf_floats, int64_t* psf_offsets, int64_t* n_lit);
int psf_plan_destroy(psf_plan_t plan);
int psf_accumulate(psf_plan_t plan, const float* layers, int64_t step, float* psf,
                   double* phase_var, void* stream);
int psf_strehl(psf_plan_t plan, const float* psf, const double* phase_var, int64_t n_frames,
               float* sr_psf, float* sr_marechal, void* stream);

/*
 * screen_generate -- one periodic n x n phase screen (Sec. 2.1: random noise filtered in the
 *   Fourier domain with the von Karman phase spectrum of given r0 and L0; L0 = INFINITY gives
 *   the Kolmogorov spectrum):
 *     screen[y][x] = Re sum_k (a_k + i b_k) sqrt(PSD(f_k)) df exp(+2 pi i (k_x x + k_y y) / n),
 *     PSD(f) = 0.023 r0^(-5/3) (|f|^2 + L0^-2)^(-11/6), df = 1 / (n pitch_m), the f = 0 sample
 *   zeroed; frequencies f_k = k / (n pitch_m) with k in [-n/2, n/2) per axis (DFT order).
 *   a_k, b_k: Box-Muller normals from the first two words of the Philox4x32-10 block with
 *   counter (k_y n + k_x, 0, stream_id low, stream_id high) and key (seed low, seed high),
 *   u = ((w >> 8) + 1/2) 2^-24, a = sqrt(-2 ln u0) cos(2 pi u1), b = sqrt(-2 ln u0) sin(2 pi u1).
 *   Radians at the wavelength r0 refers to.  n: a power of two in [16, 4096].  screen: device
 *   [n][n] (written).  work: device, >= 2 n^2 floats.  Asynchronous; deterministic.
 *   No subharmonics: they would break the periodicity the layers' wrap-around relies on.
 */
int screen_generate(int32_t n, double pitch_m, double r0_m, double L0_m, uint64_t seed,
                    uint64_t stream_id, float* screen, float* work, int64_t work_floats,
                    void* stream);

/* Message of the last failure on the calling thread ("" if none). */
const char* wfs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WFS_H */
