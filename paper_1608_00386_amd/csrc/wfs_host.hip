// Host side of libwfs: argument validation, geometry tables (pupil mask, valid subapertures,
// cone/frozen-flow affine maps, elongation parameters, binning phase tables), task tables and
// the C ABI entry points declared in include/wfs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <set>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdarg>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/wfs.h"
#include "wfs_internal.h"

namespace wfs {
hipError_t launch_forward(const FwdParams& p, int ns, hipStream_t st, const SideStream* side);
hipError_t launch_foot_entries(const FwdParams& p, FootEnt* out, int n_frames, hipStream_t st);
hipError_t launch_project(const FwdParams& p, float* phase, int lds, hipStream_t st);
int project_lds_bytes(int n_layers, int rows);
int project_max_groups();
int project_strip();
int project_rows();
hipError_t launch_step(int64_t* step_dev, int64_t value, int add, hipStream_t st);
hipError_t launch_adjoint(const AdjParams& a, int ns, bool clear_grad, bool clear,
                          hipStream_t st);
hipError_t launch_adjoint_gather(const FwdParams& f, const float* gpsi, float* grad,
                                 const int32_t* blk_start, hipStream_t st);
hipError_t launch_adjoint_gather_tab(const FwdParams& f, const float* gpsi, float* grad,
                                     int2* tab, const AdjSeg* segs, int n_segs, int max_n,
                                     const int64_t* tab_off, const int32_t* blk_start,
                                     hipStream_t st);
int adj_tab_rows();
int fft_adj_wave_lds_bytes(int n_fft, int n_pix);
hipError_t launch_adjoint_fft(const AdjParams& a, int lds_per_wave, hipStream_t st);
int adj_lds_bytes(int ns, int n_layers, int n_pix, bool gather);
hipError_t recon_work_floats(const float* R, int M, int N, const float* S, int B,
                             int64_t* floats);
hipError_t recon_stream_work(hipStream_t st, int64_t floats, float** out, bool* capturing);
int64_t recon_static_work_floats();
hipError_t recon_min_work_floats(const float* R, int M, int N, const float* S, int B,
                                 int64_t* floats);
hipError_t recon_static_work(float** out);
hipError_t recon_launch(const float* R, int M, int N, const float* S, int B, float* C,
                        int64_t ldc, float alpha, float beta, float* ws, int64_t ws_floats,
                        hipStream_t st, int* used_mfma);
hipError_t calib_poke(float* layers, const float* base, int64_t stride, int32_t h, int64_t act0,
                      int32_t n_chunk, float amp, hipStream_t st);
hipError_t calib_diff(const float* slopes, int32_t h, int32_t n_slopes, int32_t n_chunk,
                      float amp, float* im, int64_t ld_im, hipStream_t st);
int otf_lds_bytes(int ns, int n_layers, int n_pix, bool with_taps, int foot_floats,
                  int lag_parts = kOtfLagParts);
int foot_pitch(int ns);
int fft_wave_lds_bytes(int n_fft, int n_pix);
bool fft_supported(int n_sub, int n_fft, int bin);
}  // namespace wfs

using namespace wfs;

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

namespace wfs {
// Error reporting for the other translation units of the C ABI (same thread-local message).
int set_error(int code, const char* msg) {
  g_err = msg;
  return code;
}
}  // namespace wfs

static int hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? WFS_ENOMEM : WFS_EDEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                     \
  do {                                          \
    hipError_t _e = (expr);                     \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

// projection blocks of one realisation (device descriptors)
struct ProjTable {
  const int2* desc = nullptr;
  int32_t per_real = 0;
};

static void set_proj(FwdParams& p, const ProjTable& t) {
  p.proj_desc = t.desc;
  p.proj_per_real = t.per_real;
}

// One projection tile height offered by a plan: blocks of rows pupil rows (all sensors, and
// the FFT-path sensors alone) and the LDS bytes of a block.
struct ProjSet {
  ProjTable all, fft;
  int rows = 0, lds = 0, lds_fft = 0;
};

struct OtfGroup {
  int ns = 0, max_npix = 0, foot_floats = 0;
  std::vector<int> ids;
  TaskTable tasks{};
  int64_t n_tasks = 0;
  // LDS bytes per wave of this group's lag-domain waves in a launch without FFT-path blocks
  int lds_split = 0, lds_fused = 0, lds_foot = 0, lds_adj = 0;
  int lds_split_lp[2] = {0, 0};  // split field with the lag row in 2 / 3 passes
};

struct wfs_plan_s {
  int device = 0;
  int32_t n_layers = 0, n_sensors = 0, batch = 0;
  int64_t layer_stride = 0;
  double lambda_ref = 0, dt = 0;
  uint32_t flags = 0;
  std::vector<wfs_layer_desc> layers;
  std::vector<wfs_sensor_desc> sensors;
  std::vector<DevSensor> hsen;
  std::vector<int32_t> n_valid;
  std::vector<double> pix_scale;
  int32_t n_slopes = 0, n_valid_total = 0;
  int64_t phase_per_real = 0;
  int64_t pupil_per_real = 0;       // sum over sensors of n_pup^2
  float* d_gimg = nullptr;          // adjoint gather: [B][pupil_per_real], allocated on first use
  // device blob holding every table
  char* d_blob = nullptr;
  int64_t* d_step = nullptr;
  FwdParams base{};  // table pointers, sizes and schedule; per-call fields filled at launch
  int otf_ns = 0;    // lag-domain template instance of group 0 (0: no lag-domain sensor)
  int otf_max_npix = 0;
  // lag-domain sensors grouped by subaperture size, one spot launch per group: group 0's
  // launch also carries the FFT-path and pipelined projection blocks (its task table and LDS
  // sizes are the ones in `base` and below)
  std::vector<OtfGroup> groups;
  int64_t otf_tasks = 0, fft_tasks = 0;
  int adj_lds_per_wave = 0;
  std::vector<int32_t> gather_blk;  // adjoint gather: first tile of each layer (+ total)
  // table-driven adjoint gather (layers whose inverse stencil lists are short): first tile of
  // each such layer (+ total), the segments of the list tables, and the tables themselves
  std::vector<int32_t> gather_tab_blk;
  int adj_nseg = 0, adj_maxn = 0;
  int64_t adj_ent = 0;
  const AdjSeg* d_adj_segs = nullptr;
  const int64_t* d_adj_tab_off = nullptr;
  int2* d_adj_tab = nullptr;  // allocated on the first gather call, with d_gimg
  bool adj_clear_grad = true;  // the layer grids leave gaps inside the stride
  int lds_split = 0, lds_fused = 0;  // LDS bytes per lag-domain wave, per schedule
  int lds_split_otf = 0, lds_fused_otf = 0;  // same, in a launch without FFT-path blocks
  // the split field's figures with the lag row in 2 / 3 passes, and the current pass count
  int lds_split_lp[2] = {0, 0}, lds_split_otf_lp[2] = {0, 0};
  int lag_parts = kOtfLagParts;
  int proj_lds = 0;          // bytes of LDS per projection block (all sensors)
  int proj_lds_fft = 0;      // same, FFT-path sensors only
  ProjTable proj_all{}, proj_fft{};  // the projection blocks of the current tile height
  std::vector<ProjSet> proj_sets;    // every tile height the plan offers (rows ascending)
  int proj_set = 0;                  // the current one
  float* d_phase = nullptr;   // split-mode phase buffer [B][phase_per_real]
  float* d_phase2 = nullptr;  // second buffer (pipelined frames), same allocation
  int split = 0;             // 1: projection kernel + spot kernel; 0: fused gather
  int foot_ok = 0;           // every lag-domain sensor can stage its footprint, no FFT path
  int foot = 0;              // staged-footprint field (overrides split / fused gather)
  // wfs_forward_steps: 0 one wfs_forward per frame, 1 pipelined split frames, 2 one
  // staged-footprint launch for all frames, 3 split frames with the next frame's projection
  // on a second stream (1-3 only when the single-frame field is the split or the footprint
  // one: all four give the same bits)
  int frames = 0;
  int lds_foot = 0;          // LDS bytes per lag-domain wave with the staged footprint
  FootEnt* d_foot_ent = nullptr;  // stencil entries of up to foot_ent_cap frames
  int foot_ent_cap = 0;           // frames per footprint launch (longer runs take several)
  SideStream side{};         // FFT-path blocks run here concurrently (plans with both paths)
  // overlapped frames (frames == 3): frame k + 1 is projected here while frame k's spots run
  // on the caller's stream; proj_done[i] / spot_done[i]: the last projection into / spot
  // launch from phase buffer i
  struct {
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, proj_done[2] = {nullptr, nullptr},
               spot_done[2] = {nullptr, nullptr};
  } ovl;
  float* d_fft_adj = nullptr;    // FFT-path adjoint: per-chunk phase-gradient shares and the
  float* d_adj_fwd = nullptr;    // noise-free forward outputs it needs ([B][n_slopes + n_valid])
  int64_t fft_adj_per_real = 0;  // (both allocated on the first adjoint call)
  int fft_adj_lds = 0;           // LDS bytes per FFT-path adjoint wave
  float* d_fft_part = nullptr;   // FFT path: partial images of the spectrum chunks
  int32_t* d_fft_cnt = nullptr;  // and per-subaperture chunk counters (zero between launches)
  int64_t fft_part_per_real = 0, fft_cnt_per_real = 0;
  float4* d_na = nullptr;    // sodium-profile table (wfs_plan_na_profile), capacity na_cap
  int64_t na_cap = 0;
  std::vector<float4*> na_retired;  // outgrown tables: graphs captured earlier may hold them
};

static bool finite_d(double x) { return std::isfinite(x); }

static void destroy_ovl(wfs_plan_s* P) {
  for (int i = 0; i < 2; ++i) {
    if (P->ovl.proj_done[i]) (void)hipEventDestroy(P->ovl.proj_done[i]);
    if (P->ovl.spot_done[i]) (void)hipEventDestroy(P->ovl.spot_done[i]);
    P->ovl.proj_done[i] = P->ovl.spot_done[i] = nullptr;
  }
  if (P->ovl.fork) (void)hipEventDestroy(P->ovl.fork);
  if (P->ovl.stream) (void)hipStreamDestroy(P->ovl.stream);
  P->ovl.fork = nullptr;
  P->ovl.stream = nullptr;
}

// Makes projection tile height i of the plan the current one (host only: the descriptors of
// every height are on the device already, and each height gives the same bits).
static void use_lag_parts(wfs_plan_s* P, int lp) {
  const int i = lp == 3 ? 1 : 0;
  P->lag_parts = lp;
  P->lds_split = P->lds_split_lp[i];
  P->lds_split_otf = P->lds_split_otf_lp[i];
  for (OtfGroup& G : P->groups) G.lds_split = G.lds_split_lp[i];
  P->base.lag_parts = lp;
  P->base.lds_per_wave = P->lds_split;
  P->base.lds_per_wave_otf = P->lds_split_otf;
}

static void use_proj_set(wfs_plan_s* P, int i) {
  const ProjSet& q = P->proj_sets[i];
  P->proj_set = i;
  P->proj_all = q.all;
  P->proj_fft = q.fft;
  P->proj_lds = q.lds;
  P->proj_lds_fft = q.lds_fft;
  P->base.proj_lds = q.lds;
  set_proj(P->base, q.all);
}

// ------------------------------------------------------------------------------------------
// geometry
// ------------------------------------------------------------------------------------------

struct SensorGeom {
  int n_pup = 0;
  double dx = 0;
  std::vector<uint8_t> mask;  // [n_pup][n_pup]
  std::vector<DevSubap> subs; // valid subapertures, row-major
};

// Pupil pixels of pitch dx = D / n_pup centred at (i + 1/2 - n_pup/2) dx; lit when the centre
// radius is within [D_obs/2, D/2]; a subaperture is valid when its lit fraction >= valid_frac.
static SensorGeom sensor_geometry(const wfs_sensor_desc& s) {
  SensorGeom g;
  const int ns = s.n_sub;
  g.n_pup = s.n_sa * ns;
  g.dx = s.pupil_d_m / g.n_pup;
  g.mask.assign((size_t)g.n_pup * g.n_pup, 0);
  for (int j = 0; j < g.n_pup; ++j) {
    const double y = (j + 0.5 - g.n_pup / 2.0) * g.dx;
    for (int i = 0; i < g.n_pup; ++i) {
      const double x = (i + 0.5 - g.n_pup / 2.0) * g.dx;
      const double r = std::hypot(x, y);
      g.mask[(size_t)j * g.n_pup + i] = (r >= s.obs_d_m / 2.0 && r <= s.pupil_d_m / 2.0) ? 1 : 0;
    }
  }
  const double H = s.src_alt_m;
  const bool elong = s.na_fwhm_m > 0 && finite_d(H);
  const double sig_h = s.na_fwhm_m / (2.0 * std::sqrt(2.0 * std::log(2.0)));
  const double p_fft = s.lambda_m / (s.n_fft * g.dx);
  for (int a = 0; a < s.n_sa; ++a) {
    for (int b = 0; b < s.n_sa; ++b) {
      int cnt = 0;
      for (int r = 0; r < ns; ++r)
        for (int c = 0; c < ns; ++c) cnt += g.mask[(size_t)(a * ns + r) * g.n_pup + b * ns + c];
      if ((double)cnt / (double)(ns * ns) < s.valid_frac) continue;
      DevSubap d{};
      d.a = a;
      d.b = b;
      d.v = (int32_t)g.subs.size();
      const double cx = ((b + 0.5) * ns - g.n_pup / 2.0) * g.dx;
      const double cy = ((a + 0.5) * ns - g.n_pup / 2.0) * g.dx;
      const double bx = cx - s.launch_x_m, by = cy - s.launch_y_m;
      const double bl = std::hypot(bx, by);
      if (elong && bl > 0) {
        const double sig_px = bl * sig_h / (H * H) / p_fft;
        d.alpha = (float)(2.0 * M_PI * M_PI * sig_px * sig_px / ((double)s.n_fft * s.n_fft));
        d.ex = (float)(bx / bl);
        d.ey = (float)(by / bl);
        d.gam = (float)(bl / (H * H * p_fft * (double)s.n_fft));
      }
      g.subs.push_back(d);
    }
  }
  return g;
}

static int validate(const wfs_layer_desc* layers, int32_t n_layers, int64_t layer_stride,
                    const wfs_sensor_desc* sensors, int32_t n_sensors, int32_t batch,
                    double lambda_ref_m, double dt_s) {
  if (!layers || !sensors) return fail(WFS_EINVAL, "wfs_plan: null descriptor array");
  if (n_layers < 1 || n_layers > kMaxLayers)
    return fail(WFS_EINVAL, "wfs_plan: n_layers=%d outside [1, %d]", n_layers, kMaxLayers);
  if (n_sensors < 1 || n_sensors > kMaxSensors)
    return fail(WFS_EINVAL, "wfs_plan: n_sensors=%d outside [1, %d]", n_sensors, kMaxSensors);
  if (batch < 1 || batch > (1 << 20)) return fail(WFS_EINVAL, "wfs_plan: batch=%d", batch);
  if (layer_stride < 1) return fail(WFS_EINVAL, "wfs_plan: layer_stride=%lld", (long long)layer_stride);
  if (!(lambda_ref_m > 0) || !finite_d(lambda_ref_m))
    return fail(WFS_EINVAL, "wfs_plan: lambda_ref_m must be > 0");
  if (!(dt_s >= 0) || !finite_d(dt_s)) return fail(WFS_EINVAL, "wfs_plan: dt_s must be >= 0");
  for (int l = 0; l < n_layers; ++l) {
    const wfs_layer_desc& L = layers[l];
    if (L.nx < 2 || L.ny < 2 || L.nx > (1 << 20) || L.ny > (1 << 20) ||
        (int64_t)L.nx * L.ny > (1LL << 29))  // byte offsets within a layer fit 31 bits
      return fail(WFS_EINVAL, "layer %d: grid %dx%d (at most 2^29 pixels)", l, L.nx, L.ny);
    if (L.offset < 0 || L.offset + (int64_t)L.nx * L.ny > layer_stride)
      return fail(WFS_EINVAL, "layer %d: grid [%lld, +%lld) outside the stride %lld", l,
                  (long long)L.offset, (long long)L.nx * L.ny, (long long)layer_stride);
    if (!(L.pitch_m > 0) || !finite_d(L.pitch_m) || !finite_d(L.alt_m) || L.alt_m < 0 ||
        !finite_d(L.vx_mps) || !finite_d(L.vy_mps) || !std::isfinite(L.weight))
      return fail(WFS_EINVAL, "layer %d: non-finite or non-positive geometry", l);
    if (L.boundary != 0 && L.boundary != 1)
      return fail(WFS_EINVAL, "layer %d: boundary must be 0 or 1", l);
  }
  int64_t slopes = 0;
  for (int s = 0; s < n_sensors; ++s) {
    const wfs_sensor_desc& S = sensors[s];
    if (S.n_sa < 1 || S.n_sub < 1 || S.n_fft < 2 || S.bin < 1 || S.n_sa > 4095 || S.n_sub > 4080 ||
        (int64_t)S.n_sa * S.n_sub > 65536)
      return fail(WFS_EINVAL, "sensor %d: n_sa=%d n_sub=%d n_fft=%d bin=%d", s, S.n_sa, S.n_sub,
                  S.n_fft, S.bin);
    if (S.n_fft % 2) return fail(WFS_EINVAL, "sensor %d: n_fft=%d must be even", s, S.n_fft);
    if (S.n_fft % S.bin)
      return fail(WFS_EINVAL, "sensor %d: n_fft=%d not a multiple of bin=%d", s, S.n_fft, S.bin);
    if (S.n_fft < 2 * S.n_sub)
      return fail(WFS_EINVAL, "sensor %d: n_fft=%d < 2*n_sub=%d", s, S.n_fft, 2 * S.n_sub);
    if (!(S.lambda_m > 0) || !(S.pupil_d_m > 0) || !(S.obs_d_m >= 0) || S.obs_d_m >= S.pupil_d_m ||
        !finite_d(S.lambda_m) || !finite_d(S.pupil_d_m))
      return fail(WFS_EINVAL, "sensor %d: wavelength/pupil/obstruction", s);
    if (!(S.src_alt_m > 0)) return fail(WFS_EINVAL, "sensor %d: src_alt_m must be > 0", s);
    if (!(S.valid_frac > 0) || S.valid_frac > 1)
      return fail(WFS_EINVAL, "sensor %d: valid_frac must be in (0, 1]", s);
    if (!(S.photons >= 0) || !(S.read_noise_e >= 0) || !(S.na_fwhm_m >= 0) ||
        !finite_d(S.photons) || !finite_d(S.read_noise_e) || !finite_d(S.na_fwhm_m) ||
        !finite_d(S.theta_x_rad) || !finite_d(S.theta_y_rad) || !finite_d(S.launch_x_m) ||
        !finite_d(S.launch_y_m))
      return fail(WFS_EINVAL, "sensor %d: photons/noise/elongation/direction", s);
    if (!finite_d(S.tilt_x_rad) || !finite_d(S.tilt_y_rad))
      return fail(WFS_EINVAL, "sensor %d: non-finite tip-tilt offset", s);
    if (finite_d(S.src_alt_m))
      for (int l = 0; l < n_layers; ++l)
        if (!(layers[l].alt_m < S.src_alt_m))
          return fail(WFS_EINVAL, "sensor %d: layer %d at or above the LGS altitude", s, l);
    slopes += 2LL * S.n_sa * S.n_sa;
  }
  if (slopes * batch > (1LL << 31) - 1) return fail(WFS_EINVAL, "wfs_plan: too many slopes");
  return WFS_OK;
}

template <class T>
static size_t push_table(std::vector<char>& blob, const std::vector<T>& v) {
  size_t off = (blob.size() + 255) & ~size_t(255);
  blob.resize(off + v.size() * sizeof(T));
  if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
  return off;
}

static void fill_tasks(TaskTable& tt, const std::vector<int>& ids, const std::vector<int32_t>& nv) {
  std::memset(&tt, 0, sizeof tt);
  tt.n = (int32_t)ids.size();
  int32_t acc = 0;
  for (size_t k = 0; k < ids.size(); ++k) {
    tt.ids[k] = ids[k];
    tt.start[k] = acc;
    acc += nv[ids[k]];
  }
  tt.start[ids.size()] = acc;
  tt.per_real = acc;
}

static void default_schedule(wfs_plan_s* P) {
  const int64_t tasks = P->groups.empty() ? 0 : P->groups[0].n_tasks;
  const int64_t waves = tasks;
  P->base.otf_blocks = (int32_t)((waves + kWavesPerBlock - 1) / kWavesPerBlock);
  P->base.xcd_remap = (P->flags & WFS_FLAG_NO_XCD_REMAP) ? 0 : 1;
}

extern "C" {

const char* wfs_last_error(void) { return g_err.c_str(); }

int wfs_plan(const wfs_layer_desc* layers, int32_t n_layers, int64_t layer_stride,
             const wfs_sensor_desc* sensors, int32_t n_sensors, int32_t batch,
             double lambda_ref_m, double dt_s, uint32_t flags, wfs_plan_t* out) {
  g_err.clear();
  if (!out) return fail(WFS_EINVAL, "wfs_plan: null output handle");
  *out = nullptr;
  int rc = validate(layers, n_layers, layer_stride, sensors, n_sensors, batch, lambda_ref_m, dt_s);
  if (rc) return rc;
  if ((flags & WFS_FLAG_FORCE_OTF) && (flags & WFS_FLAG_FORCE_FFT))
    return fail(WFS_EINVAL, "wfs_plan: FORCE_OTF and FORCE_FFT together");

  auto* P = new wfs_plan_s();
  P->n_layers = n_layers;
  P->n_sensors = n_sensors;
  P->batch = batch;
  P->layer_stride = layer_stride;
  P->lambda_ref = lambda_ref_m;
  P->dt = dt_s;
  P->flags = flags;
  P->layers.assign(layers, layers + n_layers);
  P->sensors.assign(sensors, sensors + n_sensors);

  std::vector<DevLayer> dl(n_layers);
  for (int l = 0; l < n_layers; ++l) {
    const wfs_layer_desc& L = layers[l];
    dl[l].offset = L.offset;
    dl[l].nx = L.nx;
    dl[l].ny = L.ny;
    dl[l].weight = L.weight;
    dl[l].boundary = L.boundary;
    dl[l].inv_nx = 1.0 / L.nx;
    dl[l].inv_ny = 1.0 / L.ny;
  }

  std::vector<DevAffine> aff((size_t)n_sensors * n_layers);
  std::vector<DevSensor> ds(n_sensors);
  std::vector<DevSubap> subs;
  std::vector<uint8_t> masks;
  std::vector<float2> stab, wtab;
  std::vector<float> mtab;
  std::vector<int> otf_ids, fft_ids;
  std::vector<int32_t> subidx;
  std::vector<std::vector<int2>> proj_desc_s(n_sensors);  // projection blocks per sensor
  std::vector<int4> foot((size_t)n_sensors * n_layers, make_int4(0, 0, 0, 0));
  std::vector<FootCol> foot_cols;
  std::vector<FootAxis> foot_axis((size_t)n_sensors * n_layers * 2);
  bool foot_ok = true;
  int64_t foot_ent = 0;  // stencil entries of one frame (every footprint sensor, layer, axis)
  int32_t slope_off = 0, aux_off = 0;
  int64_t phase_off = 0, pupil_off = 0;
  int otf_ns = 0;
  for (int s = 0; s < n_sensors; ++s) {
    const wfs_sensor_desc& S = sensors[s];
    SensorGeom g = sensor_geometry(S);
    DevSensor& d = ds[s];
    std::memset(&d, 0, sizeof d);
    d.n_sa = S.n_sa;
    d.n_sub = S.n_sub;
    d.n_fft = S.n_fft;
    d.bin = S.bin;
    d.n_pix = S.n_fft / S.bin;
    d.inv_npix = 1.0f / (float)d.n_pix;
    d.n_pup = g.n_pup;
    d.n_valid = (int32_t)g.subs.size();
    d.valid_off = (int32_t)subs.size();
    d.slope_off = slope_off;
    d.aux_off = aux_off;
    d.mask_off = (int32_t)masks.size();
    d.phase_off = (int32_t)phase_off;
    d.pupil_off = (int32_t)std::min<int64_t>(pupil_off, (1LL << 31) - 1);
    d.noisy = S.photons > 0 ? 1 : 0;
    d.elong = (S.na_fwhm_m > 0 && finite_d(S.src_alt_m)) ? 1 : 0;
    d.kappa = (float)(lambda_ref_m / S.lambda_m);
    const double fph = S.photons > 0 ? S.photons : 1.0;
    d.flux_c = (float)(fph / ((double)S.n_fft * S.n_fft * (double)S.n_sub * S.n_sub));
    d.read_noise = (float)S.read_noise_e;
    d.ramp_x = (float)(0.5 / S.n_fft - S.tilt_x_rad * g.dx / S.lambda_m);
    d.ramp_y = (float)(0.5 / S.n_fft - S.tilt_y_rad * g.dx / S.lambda_m);
    // projection blocks: (group of project_rows() pupil rows, strip of project_strip()
    // columns) holding at least one pixel of a valid subaperture; packed row0 | strip << 16
    d.pad5 = 0;
    d.inv_nsub = 1.0f / (float)S.n_sub;
    d.subidx_off = (int32_t)subidx.size();
    {
      std::vector<int32_t> idx((size_t)S.n_sa * S.n_sa, -1);
      for (const DevSubap& q : g.subs) idx[(size_t)q.a * S.n_sa + q.b] = q.v;
      subidx.insert(subidx.end(), idx.begin(), idx.end());
      const int W = project_strip(), RG = project_rows();
      const int strips = (g.n_pup + W - 1) / W;
      for (int r0 = 0; r0 < g.n_pup; r0 += RG)
        for (int st = 0; st < strips; ++st) {
          bool any = false;
          for (int r = r0; r < std::min(g.n_pup, r0 + RG) && !any; ++r)
            for (int c = st * W; c < std::min(g.n_pup, (st + 1) * W) && !any; ++c)
              any = idx[(size_t)(r / S.n_sub) * S.n_sa + c / S.n_sub] >= 0;
          if (any) proj_desc_s[s].push_back(make_int2(r0 | (st << 16), s));
        }
    }
    if ((int64_t)masks.size() + (int64_t)g.mask.size() > (1LL << 31) - 1) {
      delete P;
      return fail(WFS_EINVAL, "wfs_plan: pupil masks too large");
    }
    masks.insert(masks.end(), g.mask.begin(), g.mask.end());
    subs.insert(subs.end(), g.subs.begin(), g.subs.end());
    slope_off += 2 * d.n_valid;
    aux_off += d.n_valid;
    phase_off += (int64_t)d.n_valid * S.n_sub * S.n_sub;
    pupil_off += (int64_t)g.n_pup * g.n_pup;
    P->n_valid.push_back(d.n_valid);
    P->pix_scale.push_back(S.bin * S.lambda_m / (S.n_fft * g.dx));

    // path choice
    const bool otf_ok = S.n_sub <= kOtfMaxNsub;
    const bool fft_ok = !d.elong && fft_supported(S.n_sub, S.n_fft, S.bin);
    int path;
    if (flags & WFS_FLAG_FORCE_OTF) path = otf_ok ? kPathOtf : -1;
    else if (flags & WFS_FLAG_FORCE_FFT) path = fft_ok ? kPathFft : -1;
    else path = otf_ok ? kPathOtf : (fft_ok ? kPathFft : -1);
    if (path < 0) {
      delete P;
      return fail(WFS_EUNSUPPORTED,
                  "sensor %d: n_sub=%d n_fft=%d bin=%d elongation=%d has no kernel path", s,
                  S.n_sub, S.n_fft, S.bin, d.elong);
    }
    if (path == kPathOtf) {
      if (!otf_ns) otf_ns = S.n_sub;
      otf_ids.push_back(s);
      size_t gi = 0;
      while (gi < P->groups.size() && P->groups[gi].ns != S.n_sub) ++gi;
      if (gi == P->groups.size()) {
        P->groups.emplace_back();
        P->groups.back().ns = S.n_sub;
      }
      P->groups[gi].ids.push_back(s);
      P->groups[gi].max_npix = std::max(P->groups[gi].max_npix, d.n_pix);
      if (gi == 0) P->otf_max_npix = P->groups[0].max_npix;
    } else {
      fft_ids.push_back(s);
    }
    d.path = path;
    // lag-domain tables: s(k) = (-1)^k sum_{d<bin} e^{2 pi i k d / N}, |k| < n_sub, and the
    // n_pix-point inverse twiddles e^{2 pi i t / n_pix}
    d.stab_off = (int32_t)stab.size();
    for (int k = -(S.n_sub - 1); k <= S.n_sub - 1; ++k) {
      double re = 0, im = 0;
      for (int q = 0; q < S.bin; ++q) {
        const double a = 2.0 * M_PI * (double)k * q / S.n_fft;
        re += std::cos(a);
        im += std::sin(a);
      }
      const double sg = (std::abs(k) % 2) ? -1.0 : 1.0;
      stab.push_back(make_float2((float)(sg * re), (float)(sg * im)));
    }
    // image operands for the matrix cores (n_pix <= 8): with C = cos, S = sin of
    // 2 pi (k n mod n_pix) / n_pix, F1 = [[C, S], [-S, C]] (Z = [Pr|Pi] F1 gives [Zr|Zi]) and
    // F2 = [C | -S] (B = F2 [Zr; Zi]), each 16 x 16 row-major, zero outside n_pix
    d.mtab_off = -1;
    if (d.n_pix <= 8) {
      d.mtab_off = (int32_t)mtab.size();
      const int np = d.n_pix;
      auto cs = [&](int a, int b2, bool sine) {
        if (a >= np || b2 >= np) return 0.0f;
        const double t = 2.0 * M_PI * ((a * b2) % np) / np;
        return (float)(sine ? std::sin(t) : std::cos(t));
      };
      for (int k = 0; k < 16; ++k)
        for (int n = 0; n < 16; ++n) {
          const int kk = k & 7, nn = n & 7;
          float v;
          if (k < 8) v = n < 8 ? cs(kk, nn, false) : cs(kk, nn, true);
          else v = n < 8 ? -cs(kk, nn, true) : cs(kk, nn, false);
          mtab.push_back(v);
        }
      for (int m = 0; m < 16; ++m)
        for (int k = 0; k < 16; ++k) {
          const int mm = m & 7, kk = k & 7;
          mtab.push_back(m >= 8 ? 0.0f : (k < 8 ? cs(mm, kk, false) : -cs(mm, kk, true)));
        }
    }
    d.wtab_off = (int32_t)wtab.size();
    for (int t = 0; t < d.n_pix; ++t) {
      const double a = 2.0 * M_PI * t / d.n_pix;
      wtab.push_back(make_float2((float)std::cos(a), (float)std::sin(a)));
    }
    // cone + frozen-flow affine maps: X = s x + theta h - v t, u = X / pitch + n/2 - 1/2
    const double H = S.src_alt_m;
    for (int l = 0; l < n_layers; ++l) {
      const wfs_layer_desc& L = layers[l];
      const double sc = finite_d(H) ? 1.0 - L.alt_m / H : 1.0;
      DevAffine& A = aff[(size_t)s * n_layers + l];
      const double x0 = (0.5 - g.n_pup / 2.0) * g.dx;
      A.ax = sc * g.dx / L.pitch_m;
      A.bx0 = (sc * x0 + S.theta_x_rad * L.alt_m) / L.pitch_m + L.nx / 2.0 - 0.5;
      A.dbx = -L.vx_mps * dt_s / L.pitch_m;
      A.ay = sc * g.dx / L.pitch_m;
      A.by0 = (sc * x0 + S.theta_y_rad * L.alt_m) / L.pitch_m + L.ny / 2.0 - 0.5;
      A.dby = -L.vy_mps * dt_s / L.pitch_m;
      A.inv_ax = 1.0 / A.ax;
      A.inv_ay = 1.0 / A.ay;
    }
    // staged footprint of one subaperture: n_sub consecutive pixels span (n_sub - 1)|a|
    // layer pixels, so their stencils touch at most ceil((n_sub - 1)|a|) + 2 grid lines per
    // axis (a margin covers the rounding of the FP64 coordinates)
    if (path == kPathOtf) {
      int cols = 0, floats = 0;
      bool ok = true;
      d.foot_ent_off = (int32_t)foot_ent;
      for (int l = 0; l < n_layers && ok; ++l) {
        const wfs_layer_desc& L = layers[l];
        const DevAffine& A = aff[(size_t)s * n_layers + l];
        const double ex = (S.n_sub - 1) * std::fabs(A.ax), ey = (S.n_sub - 1) * std::fabs(A.ay);
        if (!(ex < 64.0 && ey < 64.0)) {
          ok = false;
          break;
        }
        const int fw = (int)std::ceil(ex + 1e-7) + 2, fh = (int)std::ceil(ey + 1e-7) + 2;
        ok = fh <= S.n_sub + 2 && cols + fw <= kFootMaxCols &&
             (L.boundary != 0 || (fw <= L.nx && fh <= L.ny)) &&
             L.offset + (int64_t)L.nx * L.ny <= (1LL << 30);
        if (!ok) break;
        // the window goes to LDS column by column, each column in a slot of n_sub + 2 floats
        // rounded up to odd (rows fh.. of a slot are never read): a column's stores take
        // immediate offsets, and the lanes storing neighbouring columns hit distinct banks
        const int pitch = foot_pitch(S.n_sub);
        foot[(size_t)s * n_layers + l] = make_int4(fw, fh, floats, 0);
        for (int j = 0; j < fw; ++j)
          foot_cols.push_back(FootCol{(int32_t)L.offset, L.nx, L.ny, L.boundary, fw, fh,
                                      floats + j * pitch, (l << 8) | j});
        FootAxis& X = foot_axis[((size_t)s * n_layers + l) * 2];
        FootAxis& Y = foot_axis[((size_t)s * n_layers + l) * 2 + 1];
        X = FootAxis{A.ax, A.bx0, A.dbx, 1.0 / L.nx, L.nx, L.boundary, pitch, floats, 1.0f,
                     (int32_t)foot_ent, {0, 0}};
        Y = FootAxis{A.ay, A.by0, A.dby, 1.0 / L.ny, L.ny, L.boundary, 1, 0, L.weight,
                     (int32_t)(foot_ent + g.n_pup), {0, 0}};
        foot_ent += 2LL * g.n_pup;
        cols += fw;
        floats += fw * pitch;
      }
      if (ok) {
        d.foot_cols_off = (int32_t)foot_cols.size() - cols;
        d.foot_ncols = cols;
        d.foot_floats = floats;
        for (OtfGroup& G : P->groups)
          if (G.ns == S.n_sub) G.foot_floats = std::max(G.foot_floats, floats);
      } else {
        foot_ok = false;
      }
    }  // FFT-path sensors stage no footprint: they read the projected phase
  }
  // Adjoint gather by tables: a layer qualifies when, for every sensor and axis, the pupil
  // footprint meets each layer index in one periodic image only and at most kAdjKI pupil
  // indices touch it: floor(2 / a) + 1 (the coordinates a c + b in a window of two layer
  // pixels), one more for the rounding of the FP64 coordinates.
  std::vector<uint8_t> adj_tabled(n_layers, 1);
  std::vector<AdjSeg> adj_segs;
  std::vector<int64_t> adj_tab_off((size_t)n_sensors * n_layers, -1);
  for (int l = 0; l < n_layers; ++l) {
    const wfs_layer_desc& L = layers[l];
    for (int s = 0; s < n_sensors && adj_tabled[l]; ++s)
      for (int axis = 0; axis < 2; ++axis) {
        const DevAffine& A = aff[(size_t)s * n_layers + l];
        const double a = axis ? A.ay : A.ax;
        const int n = axis ? L.ny : L.nx;
        // one periodic image per layer pixel (the gather takes the pupil rows and columns
        // of a run of layer pixels as consecutive)
        const double images =
            L.boundary ? 1.0 : std::floor((a * (ds[s].n_pup - 1) + 2.0) / n) + 1.0;
        const double need = std::floor(2.0 / a) + 2.0;
        if (!(a > 0) || images != 1.0 || !(need <= kAdjKI)) adj_tabled[l] = 0;
      }
  }
  int64_t adj_ent = 0;
  for (int l = 0; l < n_layers; ++l) {
    if (!adj_tabled[l]) continue;
    for (int s = 0; s < n_sensors; ++s) {
      adj_tab_off[(size_t)s * n_layers + l] = adj_ent;
      adj_segs.push_back(AdjSeg{adj_ent, layers[l].nx, s, l, 0});
      adj_ent += (int64_t)layers[l].nx * kAdjKI;
      adj_segs.push_back(AdjSeg{adj_ent, layers[l].ny, s, l, 1});
      adj_ent += (int64_t)layers[l].ny * kAdjKI;
      P->adj_maxn = std::max(P->adj_maxn, std::max(layers[l].nx, layers[l].ny));
    }
  }
  P->adj_ent = adj_ent;
  P->adj_nseg = (int)adj_segs.size();
  if (adj_segs.size() > 65535) {  // one grid row per segment
    std::fill(adj_tabled.begin(), adj_tabled.end(), 0);
    adj_segs.clear();
    std::fill(adj_tab_off.begin(), adj_tab_off.end(), -1);
    P->adj_nseg = 0;
    P->adj_ent = 0;
  }
  {  // do the grids cover the stride without gaps (then the gather writes every float)?
    std::vector<std::pair<int64_t, int64_t>> ext;
    for (int l = 0; l < n_layers; ++l)
      ext.emplace_back(layers[l].offset, layers[l].offset + (int64_t)layers[l].nx * layers[l].ny);
    std::sort(ext.begin(), ext.end());
    int64_t end = 0;
    bool gap = false;
    for (const auto& e2 : ext) {
      if (e2.first > end) gap = true;
      end = std::max(end, e2.second);
    }
    P->adj_clear_grad = gap || end < layer_stride;
  }
  // FFT path with several spectrum chunks: per realisation, every such sensor's partial
  // images (Q^2 chunks of M x M floats = n_fft^2 per subaperture) and chunk counters
  int64_t fft_part = 0, fft_cnt = 0, fft_adj = 0;
  for (int s : fft_ids) {
    const int N = sensors[s].n_fft, M = N >= 32 ? 32 : N, Q = N / M;
    ds[s].fft_part_off = (int32_t)std::min<int64_t>(fft_part, (1LL << 31) - 1);
    ds[s].fft_cnt_off = (int32_t)fft_cnt;
    ds[s].fft_adj_off = (int32_t)std::min<int64_t>(fft_adj, (1LL << 31) - 1);
    if (Q > 1) {
      fft_part += (int64_t)ds[s].n_valid * N * N;
      fft_cnt += ds[s].n_valid;
      fft_adj += (int64_t)ds[s].n_valid * Q * Q * sensors[s].n_sub * sensors[s].n_sub;
    }
    P->fft_adj_lds = std::max(P->fft_adj_lds,
                              (fft_adj_wave_lds_bytes(N, N / sensors[s].bin) + 15) & ~15);
  }
  P->fft_adj_per_real = fft_adj;
  if (fft_part > (1LL << 31) - 1 || fft_adj > (1LL << 31) - 1) {
    delete P;
    return fail(WFS_EINVAL, "wfs_plan: FFT-path partial images too large");
  }
  P->fft_part_per_real = fft_part;
  P->fft_cnt_per_real = fft_cnt;
  // Projection tile heights: G groups of project_rows() rows per block, G = 1, 2, 4 where a
  // block's taps fit 32 KiB of LDS (taller blocks share each column tap among more pixels).
  // By default the tallest whose launch still has enough blocks to fill the chip at two per
  // CU and SIMD pair; wfs_plan_tune times them all.
  std::vector<int> proj_gs{1};
  int proj_g_default = 0;
  {
    int64_t n1 = 0;
    for (int s = 0; s < n_sensors; ++s) n1 += (int64_t)proj_desc_s[s].size();
    n1 *= batch;
    for (int G = 2; G <= project_max_groups(); G *= 2) {
      if (project_lds_bytes(n_layers, project_rows() * G) > 32768) break;
      proj_gs.push_back(G);
      if (n1 / G >= 4096) proj_g_default = (int)proj_gs.size() - 1;
    }
  }
  P->hsen = ds;
  P->n_slopes = slope_off;
  P->n_valid_total = aux_off;
  P->phase_per_real = phase_off;
  P->pupil_per_real = pupil_off;
  P->otf_ns = otf_ns;

  // Lag-domain tasks of each group interleaved by the subaperture's relative place in the
  // pupil (row, column, then sensor): the sensors of a realisation whose subapertures see
  // the same layer pixels run at about the same time on one XCD, so waves that gather the
  // layers (staged footprint, fused gather) meet those pixels in its L2.
  std::vector<int2> task_order;
  std::vector<size_t> order_off;
  for (OtfGroup& G : P->groups) {
    struct Key {
      double row, col;
      int s, v;
    };
    std::vector<Key> keys;
    for (int s : G.ids)
      for (int v = 0; v < P->n_valid[s]; ++v) {
        const DevSubap& q = subs[(size_t)ds[s].valid_off + v];
        keys.push_back(Key{(q.a + 0.5) / ds[s].n_sa, (q.b + 0.5) / ds[s].n_sa, s, v});
      }
    std::stable_sort(keys.begin(), keys.end(), [](const Key& x, const Key& y) {
      if (x.row != y.row) return x.row < y.row;
      if (x.col != y.col) return x.col < y.col;
      return x.s < y.s;
    });
    order_off.push_back(task_order.size());
    for (const Key& k : keys) task_order.push_back(make_int2(k.s, k.v));
  }
  if (task_order.empty()) task_order.push_back(make_int2(0, 0));

  // tables -> one device blob
  std::vector<char> blob;
  const size_t o_lay = push_table(blob, dl);
  const size_t o_aff = push_table(blob, aff);
  const size_t o_sen = push_table(blob, ds);
  const size_t o_sub = push_table(blob, subs);
  const size_t o_mask = push_table(blob, masks);
  const size_t o_stab = push_table(blob, stab);
  const size_t o_wtab = push_table(blob, wtab);
  const size_t o_mtab = push_table(blob, mtab);
  const size_t o_subidx = push_table(blob, subidx);
  const size_t o_foot = push_table(blob, foot);
  if (foot_cols.empty()) foot_cols.push_back(FootCol{});
  const size_t o_fcols = push_table(blob, foot_cols);
  const size_t o_faxis = push_table(blob, foot_axis);
  // Projection blocks of all sensors interleaved by their relative place in the pupil (row
  // group, then strip, then sensor): the sensors of a realisation read overlapping layer
  // regions (all of them the same ground-layer pixels), and blocks that are neighbours in
  // this order run at about the same time on the same XCD, so those reads meet in its L2
  // instead of each sensor's pass re-fetching the layers from memory.
  auto interleave = [&](const std::vector<std::vector<int2>>& lists, bool fft_only) {
    struct Key {
      double row, col;
      int s;
      int2 d;
    };
    std::vector<Key> keys;
    for (int s = 0; s < n_sensors; ++s) {
      if (fft_only && ds[s].path != kPathFft) continue;
      const double np = (double)ds[s].n_pup;
      for (const int2& d : lists[s])
        keys.push_back(Key{(double)(d.x & 0xFFFF) / np,
                           (double)(d.x >> 16) * project_strip() / np, s, d});
    }
    std::stable_sort(keys.begin(), keys.end(), [](const Key& a, const Key& b) {
      if (a.row != b.row) return a.row < b.row;
      if (a.col != b.col) return a.col < b.col;
      return a.s < b.s;
    });
    std::vector<int2> out;
    out.reserve(keys.size());
    for (const Key& k : keys) out.push_back(k.d);
    return out;
  };
  // blocks of G row groups: the G = 1 blocks merged by row group (sensor | log2 G << 24)
  std::vector<size_t> o_pall, o_pfft, n_pall, n_pfft;
  for (int G : proj_gs) {
    const int RT = project_rows() * G;
    int lg = 0;
    while ((1 << lg) < G) ++lg;
    std::vector<std::vector<int2>> lists(n_sensors);
    for (int s = 0; s < n_sensors; ++s) {
      std::set<std::pair<int, int>> seen;
      for (const int2& d : proj_desc_s[s]) {
        const int r0 = (d.x & 0xFFFF) / RT * RT, st = d.x >> 16;
        if (seen.insert({r0, st}).second)
          lists[s].push_back(make_int2(r0 | (st << 16), s | (lg << 24)));
      }
    }
    const std::vector<int2> desc_all = interleave(lists, false),
                            desc_fft = interleave(lists, true);
    o_pall.push_back(push_table(blob, desc_all));
    o_pfft.push_back(push_table(blob, desc_fft));
    n_pall.push_back(desc_all.size());
    n_pfft.push_back(desc_fft.size());
  }
  std::vector<int64_t> step0(1, 0);
  const size_t o_step = push_table(blob, step0);
  if (adj_segs.empty()) adj_segs.push_back(AdjSeg{});
  const size_t o_adjseg = push_table(blob, adj_segs);
  const size_t o_adjoff = push_table(blob, adj_tab_off);
  const size_t o_order = push_table(blob, task_order);
  blob.resize((blob.size() + 255) & ~size_t(255));

  hipError_t e = hipGetDevice(&P->device);
  if (e == hipSuccess) e = hipMalloc((void**)&P->d_blob, blob.size());
  if (e == hipSuccess) e = hipMemcpy(P->d_blob, blob.data(), blob.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    if (P->d_blob) (void)hipFree(P->d_blob);
    delete P;
    return hip_fail(e, "wfs_plan: table upload");
  }
  FwdParams& b = P->base;
  std::memset(&b, 0, sizeof b);
  b.lay = reinterpret_cast<const DevLayer*>(P->d_blob + o_lay);
  b.aff = reinterpret_cast<const DevAffine*>(P->d_blob + o_aff);
  b.sen = reinterpret_cast<const DevSensor*>(P->d_blob + o_sen);
  b.sub = reinterpret_cast<const DevSubap*>(P->d_blob + o_sub);
  b.mask = reinterpret_cast<const uint8_t*>(P->d_blob + o_mask);
  b.stab = reinterpret_cast<const float2*>(P->d_blob + o_stab);
  b.wtab = reinterpret_cast<const float2*>(P->d_blob + o_wtab);
  b.mtab = reinterpret_cast<const float*>(P->d_blob + o_mtab);
  b.subidx = reinterpret_cast<const int32_t*>(P->d_blob + o_subidx);
  b.foot = reinterpret_cast<const int4*>(P->d_blob + o_foot);
  b.foot_cols = reinterpret_cast<const FootCol*>(P->d_blob + o_fcols);
  b.foot_axis = reinterpret_cast<const FootAxis*>(P->d_blob + o_faxis);
  b.n_frames = 1;
  {
    bool any_fft = false;
    for (int s = 0; s < n_sensors; ++s) any_fft = any_fft || ds[s].path == kPathFft;
    for (size_t i = 0; i < proj_gs.size(); ++i) {
      ProjSet q;
      q.all.desc = reinterpret_cast<const int2*>(P->d_blob + o_pall[i]);
      q.all.per_real = (int32_t)n_pall[i];
      q.fft.desc = reinterpret_cast<const int2*>(P->d_blob + o_pfft[i]);
      q.fft.per_real = (int32_t)n_pfft[i];
      q.rows = project_rows() * proj_gs[i];
      q.lds = project_lds_bytes(n_layers, q.rows);
      q.lds_fft = any_fft ? q.lds : 0;
      P->proj_sets.push_back(q);
    }
    use_proj_set(P, proj_g_default);
  }
  P->d_step = reinterpret_cast<int64_t*>(P->d_blob + o_step);
  P->d_adj_segs = reinterpret_cast<const AdjSeg*>(P->d_blob + o_adjseg);
  P->d_adj_tab_off = reinterpret_cast<const int64_t*>(P->d_blob + o_adjoff);
  b.step_dev = P->d_step;
  b.layer_stride = layer_stride;
  b.n_layers = n_layers;
  b.n_sensors = n_sensors;
  b.batch = batch;
  b.n_slopes = P->n_slopes;
  b.n_valid_total = P->n_valid_total;
  P->otf_tasks = 0;
  for (size_t gi = 0; gi < P->groups.size(); ++gi) {
    OtfGroup& G = P->groups[gi];
    fill_tasks(G.tasks, G.ids, P->n_valid);
    G.tasks.order = reinterpret_cast<const int2*>(P->d_blob + o_order) + order_off[gi];
    G.n_tasks = (int64_t)G.tasks.per_real * batch;
    P->otf_tasks += G.n_tasks;
  }
  if (P->groups.empty()) fill_tasks(b.otf, otf_ids, P->n_valid);
  else b.otf = P->groups[0].tasks;
  {  // FFT path: one task (wave) per spectrum chunk, Q^2 per subaperture
    std::vector<int32_t> units(P->n_valid);
    for (int s : fft_ids) {
      const int Q = sensors[s].n_fft / (sensors[s].n_fft >= 32 ? 32 : sensors[s].n_fft);
      units[s] = P->n_valid[s] * Q * Q;
    }
    fill_tasks(b.fft, fft_ids, units);
  }
  set_proj(b, P->proj_all);
  b.phase_per_real = P->phase_per_real;
  b.pupil_per_real = P->pupil_per_real;
  b.phase_in = nullptr;
  {
    int64_t acc = 0, acc_tab = 0;
    const int th = adj_tab_rows();
    for (int l = 0; l < n_layers; ++l) {
      P->gather_blk.push_back((int32_t)acc);
      P->gather_tab_blk.push_back((int32_t)acc_tab);
      // adjoint gather tiles: 64 x th layer pixels for tabled layers, 64 x 16 for the others
      if (adj_tabled[l])
        acc_tab += (int64_t)((layers[l].nx + 63) / 64) * ((layers[l].ny + th - 1) / th);
      else
        acc += (int64_t)((layers[l].nx + 63) / 64) * ((layers[l].ny + 15) / 16);
    }
    P->gather_blk.push_back((int32_t)acc);
    P->gather_tab_blk.push_back((int32_t)acc_tab);
  }
  P->fft_tasks = (int64_t)b.fft.per_real * batch;
  if (P->otf_tasks > (1LL << 31) - 1 || P->fft_tasks > (1LL << 31) - 1) {
    (void)hipFree(P->d_blob);
    delete P;
    return fail(WFS_EINVAL, "wfs_plan: too many subaperture tasks");
  }
  // LDS: lag-domain waves and FFT workgroups share one dynamic allocation; the split
  // schedule's waves need no tap region (the fused gather does)
  int lds_fft = 0;  // per FFT-path wave
  for (int s : fft_ids)
    lds_fft = std::max(lds_fft, fft_wave_lds_bytes(sensors[s].n_fft,
                                                   sensors[s].n_fft / sensors[s].bin));
  auto wave_lds = [&](bool taps, bool with_fft, int lag_parts = kOtfLagParts) {
    int w = otf_ns ? otf_lds_bytes(otf_ns, n_layers, P->otf_max_npix, taps, 0, lag_parts) : 0;
    if (with_fft) w = std::max(w, lds_fft);
    return std::max(16, (w + 15) & ~15);
  };
  const int lds_wave = wave_lds(true, true);
  if (lds_wave * kWavesPerBlock > 65536) {
    (void)hipFree(P->d_blob);
    delete P;
    return fail(WFS_EUNSUPPORTED, "wfs_plan: %d bytes of LDS per workgroup exceed 64 KiB",
                lds_wave * kWavesPerBlock);
  }
  P->lds_fused = lds_wave;
  for (int i = 0; i < 2; ++i) {
    P->lds_split_lp[i] = wave_lds(false, true, 2 + i);
    P->lds_split_otf_lp[i] = wave_lds(false, false, 2 + i);
  }
  // every group's LDS per wave, in launches without FFT-path blocks (group 0's launch with
  // them takes the larger figures above)
  bool adj_ok = true;
  for (OtfGroup& G : P->groups) {
    auto r16 = [](int x) { return std::max(16, (x + 15) & ~15); };
    for (int i = 0; i < 2; ++i)
      G.lds_split_lp[i] = r16(otf_lds_bytes(G.ns, n_layers, G.max_npix, false, 0, 2 + i));
    G.lds_fused = r16(otf_lds_bytes(G.ns, n_layers, G.max_npix, true, 0));
    G.lds_foot = r16(otf_lds_bytes(G.ns, n_layers, G.max_npix, false, G.foot_floats));
    // the adjoint's form (gather unless asked for atomics), as wfs_adjoint decides it
    const bool adj_gather =
        !(flags & WFS_FLAG_ADJOINT_ATOMIC) && P->pupil_per_real < (1LL << 30);
    // (each wave lays out its own sensor's image size: take the largest over the sizes)
    int adj_max = 0;
    for (int np = 1; np <= G.max_npix; ++np)
      adj_max = std::max(adj_max, adj_lds_bytes(G.ns, n_layers, np, adj_gather));
    G.lds_adj = r16(adj_max);
    if (G.lds_fused * kWavesPerBlock > 65536) {
      (void)hipFree(P->d_blob);
      delete P;
      return fail(WFS_EUNSUPPORTED, "wfs_plan: %d bytes of LDS per workgroup exceed 64 KiB",
                  G.lds_fused * kWavesPerBlock);
    }
    foot_ok = foot_ok && G.lds_foot * kWavesPerBlock <= 65536;
    adj_ok = adj_ok && G.lds_adj * kWavesPerBlock <= 65536;
  }
  P->lds_foot = otf_ns ? P->groups[0].lds_foot : 0;
  P->foot_ok = otf_ns && foot_ok && foot_ent > 0 && foot_ent < (1LL << 31) / 64;
  if (P->foot_ok) {  // the stencil-entry table: 64 MiB at most, 1 to 256 frames
    const int64_t per = foot_ent * (int64_t)sizeof(FootEnt);
    P->foot_ent_cap = (int)std::max<int64_t>(1, std::min<int64_t>(256, (64LL << 20) / per));
    e = hipMalloc((void**)&P->d_foot_ent, (size_t)(per * P->foot_ent_cap));
    if (e != hipSuccess) {
      (void)hipFree(P->d_blob);
      delete P;
      return hip_fail(e, "wfs_plan: footprint stencil entries");
    }
    b.foot_ent = P->d_foot_ent;
    b.foot_ent_per_frame = (int32_t)foot_ent;
  }
  P->lds_fused_otf = wave_lds(true, false);
  {
    // the lag row in 3 passes where that lets more blocks share a CU and the split launch
    // runs more than two rounds of blocks (one 80 x 80 LGS: 1,158 blocks, 2 passes; eight
    // realisations of six: 55,584 blocks, 3 passes); wfs_plan_tune times both
    auto per_cu = [](int lds_wave) { return std::min(8, 163840 / (lds_wave * kWavesPerBlock)); };
    int64_t blocks = 0;
    for (const OtfGroup& G : P->groups) blocks += (G.n_tasks + kWavesPerBlock - 1) / kWavesPerBlock;
    int lp = kOtfLagParts;
    if (!P->groups.empty() &&
        per_cu(P->groups[0].lds_split_lp[1]) > per_cu(P->groups[0].lds_split_lp[0]) &&
        blocks > 2LL * 256 * per_cu(P->groups[0].lds_split_lp[0]))
      lp = 3;
    use_lag_parts(P, lp);
  }
  P->adj_lds_per_wave = otf_ns ? P->groups[0].lds_adj : 16;
  if (!adj_ok) P->adj_lds_per_wave = 0;  // adjoint unsupported
  // FFT blocks first, padded to a multiple of 8 so the lag-domain blocks keep their XCD order
  b.fft_blocks = (int32_t)((P->fft_tasks + kWavesPerBlock - 1) / kWavesPerBlock);
  default_schedule(P);
  if (P->phase_per_real > 0) {
    const size_t n = (size_t)P->phase_per_real * batch;
    e = hipMalloc((void**)&P->d_phase, sizeof(float) * 2 * n);
    if (e != hipSuccess) {
      (void)hipFree(P->d_blob);
      delete P;
      return hip_fail(e, "wfs_plan: phase buffers");
    }
    P->d_phase2 = P->d_phase + n;
  }
  P->base.proj_lds = P->proj_lds;
  P->split = (flags & WFS_FLAG_FUSED) ? 0 : 1;
  if (P->proj_lds > 65536) P->split = 0;  // taps of one subaperture exceed the LDS budget
  if (flags & (WFS_FLAG_SPLIT | WFS_FLAG_FUSED)) P->foot_ok = 0;
  // single frames: the projection kernel first (one footprint launch per frame exposes the
  // window loads of every wave at once); frames in a row: one footprint launch
  P->foot = (P->foot_ok && P->fft_tasks == 0 && (flags & WFS_FLAG_FOOTPRINT)) ? 1 : 0;
  // with FFT-path sensors their per-frame chain on the side stream can outlast the one
  // footprint launch (six 80 x 80 LGS and three 2 x 2 NGS at 8 realisations: 0.81 against
  // 0.57 ms per frame), so such plans take it by default only when asked
  // (WFS_FLAG_FOOTPRINT) or when the tuner finds it faster
  P->frames = (P->foot_ok && (P->fft_tasks == 0 || (flags & WFS_FLAG_FOOTPRINT)))
                  ? 2
                  : (P->split && P->d_phase ? 1 : 0);
  if (P->proj_lds_fft > 65536) {
    (void)hipFree(P->d_blob);
    if (P->d_phase) (void)hipFree(P->d_phase);
    delete P;
    return fail(WFS_EUNSUPPORTED, "wfs_plan: projection taps of an FFT-path sensor exceed 64 KiB");
  }
  if (P->fft_cnt_per_real > 0) {  // chunk partials and counters (counters start at zero)
    e = hipMalloc((void**)&P->d_fft_part,
                  sizeof(float) * (size_t)P->fft_part_per_real * P->batch);
    if (e == hipSuccess)
      e = hipMalloc((void**)&P->d_fft_cnt,
                    sizeof(int32_t) * (size_t)P->fft_cnt_per_real * P->batch);
    if (e == hipSuccess)
      e = hipMemset(P->d_fft_cnt, 0, sizeof(int32_t) * (size_t)P->fft_cnt_per_real * P->batch);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      if (P->d_fft_part) (void)hipFree(P->d_fft_part);
  if (P->d_foot_ent) (void)hipFree(P->d_foot_ent);
      if (P->d_fft_cnt) (void)hipFree(P->d_fft_cnt);
      (void)hipFree(P->d_blob);
      if (P->d_phase) (void)hipFree(P->d_phase);
      delete P;
      return hip_fail(e, "wfs_plan: FFT-path chunk buffers");
    }
    P->base.fft_part = P->d_fft_part;
    P->base.fft_cnt = P->d_fft_cnt;
    P->base.fft_part_per_real = P->fft_part_per_real;
    P->base.fft_cnt_per_real = (int32_t)P->fft_cnt_per_real;
  }
  if (P->d_phase) {  // overlapped frames: the projection stream and its events
    e = hipStreamCreateWithFlags(&P->ovl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->ovl.fork, hipEventDisableTiming);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
      e = hipEventCreateWithFlags(&P->ovl.proj_done[i], hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&P->ovl.spot_done[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      destroy_ovl(P);
      (void)hipFree(P->d_blob);
      (void)hipFree(P->d_phase);
      if (P->d_fft_part) (void)hipFree(P->d_fft_part);
      if (P->d_fft_cnt) (void)hipFree(P->d_fft_cnt);
      delete P;
      return hip_fail(e, "wfs_plan: projection stream");
    }
  }
  if (P->fft_tasks > 0 && P->otf_tasks > 0) {  // both paths: FFT-path blocks on a side stream
    e = hipStreamCreateWithFlags(&P->side.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->side.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->side.join, hipEventDisableTiming);
    if (e != hipSuccess) {
      if (P->side.join) (void)hipEventDestroy(P->side.join);
      if (P->side.fork) (void)hipEventDestroy(P->side.fork);
      if (P->side.stream) (void)hipStreamDestroy(P->side.stream);
      destroy_ovl(P);
      (void)hipFree(P->d_blob);
      if (P->d_phase) (void)hipFree(P->d_phase);
      if (P->d_fft_part) (void)hipFree(P->d_fft_part);
      if (P->d_fft_cnt) (void)hipFree(P->d_fft_cnt);
      delete P;
      return hip_fail(e, "wfs_plan: side stream");
    }
  }
  *out = P;
  return WFS_OK;
}

int wfs_plan_info(wfs_plan_t P, int32_t* n_slopes, int32_t* n_valid_total,
                  int32_t* n_valid_per_sensor, double* pix_scale_rad) {
  if (!P) return fail(WFS_EINVAL, "wfs_plan_info: null plan");
  if (n_slopes) *n_slopes = P->n_slopes;
  if (n_valid_total) *n_valid_total = P->n_valid_total;
  for (int s = 0; s < P->n_sensors; ++s) {
    if (n_valid_per_sensor) n_valid_per_sensor[s] = P->n_valid[s];
    if (pix_scale_rad) pix_scale_rad[s] = P->pix_scale[s];
  }
  return WFS_OK;
}

int wfs_plan_path(wfs_plan_t P, int32_t* path_per_sensor) {
  if (!P || !path_per_sensor) return fail(WFS_EINVAL, "wfs_plan_path: null argument");
  for (int s = 0; s < P->n_sensors; ++s) path_per_sensor[s] = P->hsen[s].path;
  return WFS_OK;
}

int wfs_plan_destroy(wfs_plan_t P) {
  if (!P) return fail(WFS_EINVAL, "wfs_plan_destroy: null plan");
  hipError_t e = hipDeviceSynchronize();
  if (P->d_blob) (void)hipFree(P->d_blob);
  if (P->d_phase) (void)hipFree(P->d_phase);
  if (P->d_gimg) (void)hipFree(P->d_gimg);
  if (P->d_na) (void)hipFree(P->d_na);
  if (P->d_adj_tab) (void)hipFree(P->d_adj_tab);
  if (P->d_fft_part) (void)hipFree(P->d_fft_part);
  if (P->d_fft_cnt) (void)hipFree(P->d_fft_cnt);
  if (P->d_fft_adj) (void)hipFree(P->d_fft_adj);
  if (P->d_adj_fwd) (void)hipFree(P->d_adj_fwd);
  for (float4* q : P->na_retired) (void)hipFree(q);
  if (P->side.join) (void)hipEventDestroy(P->side.join);
  if (P->side.fork) (void)hipEventDestroy(P->side.fork);
  if (P->side.stream) (void)hipStreamDestroy(P->side.stream);
  destroy_ovl(P);
  delete P;
  if (e != hipSuccess) return hip_fail(e, "wfs_plan_destroy");
  return WFS_OK;
}

static int check_device(wfs_plan_t P, const char* who) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, who);
  if (dev != P->device)
    return fail(WFS_EINVAL, "%s: current device %d is not the plan's device %d", who, dev,
                P->device);
  return WFS_OK;
}

int wfs_plan_na_profile(wfs_plan_t P, int32_t n_entries, int32_t n_peaks, const double* table) {
  if (!P) return fail(WFS_EINVAL, "wfs_plan_na_profile: null plan");
  if (n_entries == 0) {  // back to each sensor's single Gaussian
    P->base.na_entries = 0;
    P->base.na_peaks = 0;
    return WFS_OK;
  }
  if (n_entries < 0 || n_entries > (1 << 20))
    return fail(WFS_EINVAL, "wfs_plan_na_profile: n_entries=%d outside [0, 2^20]", n_entries);
  if (n_peaks < 1 || n_peaks > kMaxNaPeaks)
    return fail(WFS_EINVAL, "wfs_plan_na_profile: n_peaks=%d outside [1, %d]", n_peaks,
                kMaxNaPeaks);
  if (!table) return fail(WFS_EINVAL, "wfs_plan_na_profile: null table");
  const double to_sigma = 1.0 / (2.0 * std::sqrt(2.0 * std::log(2.0)));
  std::vector<float4> h((size_t)n_entries * n_peaks);
  for (int k = 0; k < n_entries; ++k) {
    const double* e = table + (size_t)k * n_peaks * 3;
    double wsum = 0.0;
    for (int j = 0; j < n_peaks; ++j) {
      const double dh = e[3 * j], fw = e[3 * j + 1], w = e[3 * j + 2];
      if (!finite_d(dh) || !finite_d(fw) || !finite_d(w) || fw < 0 || w < 0)
        return fail(WFS_EINVAL,
                    "wfs_plan_na_profile: entry %d peak %d: dh, fwhm, weight must be finite, "
                    "fwhm >= 0 and weight >= 0", k, j);
      wsum += w;
    }
    if (!(wsum > 0))
      return fail(WFS_EINVAL, "wfs_plan_na_profile: entry %d has no positive weight", k);
    for (int j = 0; j < n_peaks; ++j) {
      const double sig = e[3 * j + 1] * to_sigma;
      h[(size_t)k * n_peaks + j] = make_float4((float)(2.0 * M_PI * M_PI * sig * sig),
                                               (float)e[3 * j], (float)(e[3 * j + 2] / wsum),
                                               0.0f);
    }
  }
  int rc = check_device(P, "wfs_plan_na_profile");
  if (rc) return rc;
  // no launch may still read the table being replaced
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "wfs_plan_na_profile: synchronise");
  const int64_t need = (int64_t)h.size();
  if (need > P->na_cap) {
    float4* q = nullptr;
    e = hipMalloc((void**)&q, sizeof(float4) * (size_t)need);
    if (e != hipSuccess) return fail(WFS_ENOMEM, "wfs_plan_na_profile: %lld peaks", (long long)need);
    if (P->d_na) P->na_retired.push_back(P->d_na);
    P->d_na = q;
    P->na_cap = need;
  }
  e = hipMemcpy(P->d_na, h.data(), sizeof(float4) * h.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "wfs_plan_na_profile: upload");
  P->base.na_tab = P->d_na;
  P->base.na_entries = n_entries;
  P->base.na_peaks = n_peaks;
  return WFS_OK;
}

static int check_step(int64_t step, const char* who) {
  if (step < 0 && step != WFS_STEP_DEVICE)
    return fail(WFS_EINVAL, "%s: step=%lld (>= 0 or WFS_STEP_DEVICE)", who, (long long)step);
  return WFS_OK;
}

static FwdParams call_params(wfs_plan_t P, const float* layers, int64_t step, uint64_t seed,
                             float* slopes, float* aux) {
  FwdParams p = P->base;
  p.layers = layers;
  p.step = step < 0 ? 0 : step;
  p.use_dev_step = step == WFS_STEP_DEVICE ? 1 : 0;
  p.seed_lo = (uint32_t)(seed & 0xFFFFFFFFu);
  p.seed_hi = (uint32_t)(seed >> 32);
  p.noise_on = 1;
  p.slopes = slopes;
  p.aux = aux;
  return p;
}

// The spot launch of every lag-domain group (subaperture size) for `p`, which is set up for
// group 0 (its tasks and LDS per wave, the FFT-path and projection blocks); the other groups
// follow on `st` with their own tasks and LDS and neither FFT-path nor projection blocks.
static hipError_t launch_groups(wfs_plan_t P, const FwdParams& p, hipStream_t st,
                                const SideStream* side) {
  hipError_t e = launch_forward(p, P->otf_ns ? P->otf_ns : 2, st, side);
  for (size_t g = 1; g < P->groups.size() && e == hipSuccess; ++g) {
    const OtfGroup& G = P->groups[g];
    FwdParams q = p;
    q.otf = G.tasks;
    q.otf_blocks = (int32_t)((G.n_tasks + kWavesPerBlock - 1) / kWavesPerBlock);
    q.fft_blocks = 0;
    q.proj_blocks = 0;
    q.lds_per_wave = p.otf_from_phase == 2   ? G.lds_foot
                     : p.otf_from_phase == 1 ? G.lds_split
                                             : G.lds_fused;
    q.lds_per_wave_otf = q.lds_per_wave;
    e = launch_forward(q, G.ns, st, nullptr);
  }
  return e;
}

// fused: one launch; split: projection into the plan's phase buffer, then the spot launch
static hipError_t launch_fwd_modes(wfs_plan_t P, FwdParams p, hipStream_t st) {
  if (P->foot) {  // staged footprint: the spot launch alone (no FFT-path sensor here)
    p.otf_from_phase = 2;
    p.n_frames = 1;
    p.lds_per_wave = P->lds_foot;
    p.lds_per_wave_otf = P->lds_foot;
    hipError_t e = launch_foot_entries(p, P->d_foot_ent, 1, st);
    if (e != hipSuccess) return e;
    return launch_groups(P, p, st, &P->side);
  }
  const bool split = P->split && P->d_phase;
  if (split || P->fft_tasks > 0) {  // FFT-path sensors always read the projected phase
    set_proj(p, split ? P->proj_all : P->proj_fft);
    hipError_t e = launch_project(p, P->d_phase, split ? P->proj_lds : P->proj_lds_fft, st);
    if (e != hipSuccess) return e;
    p.phase_in = P->d_phase;
  }
  p.otf_from_phase = split ? 1 : 0;
  p.lds_per_wave = split ? P->lds_split : P->lds_fused;
  p.lds_per_wave_otf = split ? P->lds_split_otf : P->lds_fused_otf;
  return launch_groups(P, p, st, &P->side);
}

int wfs_forward(wfs_plan_t P, const float* layers, int64_t step, uint64_t seed, float* slopes,
                float* aux, void* stream) {
  if (!P) return fail(WFS_EINVAL, "wfs_forward: null plan");
  if (!layers || !slopes) return fail(WFS_EINVAL, "wfs_forward: null layers or slopes");
  int rc = check_step(step, "wfs_forward");
  if (rc) return rc;
  rc = check_device(P, "wfs_forward");
  if (rc) return rc;
  FwdParams p = call_params(P, layers, step, seed, slopes, aux);
  hipError_t e = launch_fwd_modes(P, p, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "wfs_forward: launch");
  return WFS_OK;
}

// Frames step0 .. step0 + n - 1 (or the device counter + k), outputs of frame k at slopes +
// k * (slopes of one frame).  Staged footprint: one launch for all frames.  Pipelined (split
// schedule only): project frame 0; then launch k computes the spots of frame k from phase
// buffer k % 2 and projects frame k + 1 into the other buffer.  Overlapped: the projection of
// frame k + 1 (into buffer (k + 1) % 2, once the spots of frame k - 1 have read it) runs on
// the plan's projection stream while the spots of frame k (after its projection) run on st;
// the projection kernel is bound by the vector L1's access rate, the spot kernel by vector
// issue, so the two share the chip.
static hipError_t run_steps(wfs_plan_t P, const float* layers, int64_t step0, int n,
                            uint64_t seed, float* slopes, float* aux, int frames,
                            hipStream_t st) {
  const bool pipelined = frames == 1;
  const int64_t ns_per = (int64_t)P->n_slopes * P->batch;
  const int64_t na_per = (int64_t)P->n_valid_total * P->batch;
  auto frame = [&](int k) {
    const int64_t s = step0 == WFS_STEP_DEVICE ? WFS_STEP_DEVICE : step0 + k;
    FwdParams p = call_params(P, layers, s, seed, slopes + k * ns_per, aux ? aux + k * na_per : nullptr);
    if (s == WFS_STEP_DEVICE) p.step = k;
    return p;
  };
  hipError_t e = hipSuccess;
  // footprint launches of every lag-domain frame, as many frames a launch as the stencil-entry
  // table holds, each after the launch that fills the table
  auto foot_frames = [&]() {
    hipError_t ef = hipSuccess;
    for (int c0 = 0; c0 < n && ef == hipSuccess; c0 += P->foot_ent_cap) {
      FwdParams q = frame(c0);
      q.otf_from_phase = 2;
      q.n_frames = std::min(P->foot_ent_cap, n - c0);
      q.lds_per_wave = P->lds_foot;
      q.lds_per_wave_otf = P->lds_foot;
      q.fft_blocks = 0;
      ef = launch_foot_entries(q, P->d_foot_ent, q.n_frames, st);
      if (ef == hipSuccess) ef = launch_groups(P, q, st, nullptr);
    }
    return ef;
  };
  if (frames == 2) {
    if (P->base.fft_blocks == 0) return foot_frames();
    // FFT-path sensors read the projected phase: frame by frame on the side stream (their
    // projection into the plan's phase buffer, then their launch), concurrently with the one
    // footprint launch of every lag-domain frame on st
    hipStream_t fs = P->side.stream ? P->side.stream : st;
    if (fs != st) {
      e = hipEventRecord(P->side.fork, st);
      if (e == hipSuccess) e = hipStreamWaitEvent(fs, P->side.fork, 0);
    }
    for (int k = 0; k < n && e == hipSuccess; ++k) {
      FwdParams a = frame(k);
      set_proj(a, P->proj_fft);
      e = launch_project(a, P->d_phase, P->proj_lds_fft, fs);
      if (e != hipSuccess) break;
      a.phase_in = P->d_phase;
      a.otf_from_phase = 1;
      a.otf_blocks = 0;
      a.proj_blocks = 0;
      a.lds_per_wave = P->lds_split;
      e = launch_forward(a, P->otf_ns ? P->otf_ns : 2, fs, nullptr);
    }
    if (e == hipSuccess) e = foot_frames();
    if (e == hipSuccess && fs != st) {
      e = hipEventRecord(P->side.join, fs);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, P->side.join, 0);
    }
    return e;
  }
  if (frames == 3 && P->ovl.stream && P->d_phase) {
    float* buf[2] = {P->d_phase, P->d_phase2};
    hipStream_t ps = P->ovl.stream;
    auto project_into = [&](int k) {
      FwdParams q = frame(k);
      set_proj(q, P->proj_all);
      hipError_t r = launch_project(q, buf[k & 1], P->proj_lds, ps);
      if (r == hipSuccess) r = hipEventRecord(P->ovl.proj_done[k & 1], ps);
      return r;
    };
    e = hipEventRecord(P->ovl.fork, st);  // the projections follow everything queued on st
    if (e == hipSuccess) e = hipStreamWaitEvent(ps, P->ovl.fork, 0);
    if (e == hipSuccess) e = project_into(0);
    for (int k = 0; k < n && e == hipSuccess; ++k) {
      if (k + 1 < n) {
        if (k >= 1) e = hipStreamWaitEvent(ps, P->ovl.spot_done[(k - 1) & 1], 0);
        if (e == hipSuccess) e = project_into(k + 1);
        if (e != hipSuccess) break;
      }
      e = hipStreamWaitEvent(st, P->ovl.proj_done[k & 1], 0);
      if (e != hipSuccess) break;
      FwdParams p = frame(k);
      p.phase_in = buf[k & 1];
      p.otf_from_phase = 1;
      p.proj_blocks = 0;
      p.lds_per_wave = P->lds_split;
      p.lds_per_wave_otf = P->lds_split_otf;
      e = launch_groups(P, p, st, &P->side);
      if (e == hipSuccess) e = hipEventRecord(P->ovl.spot_done[k & 1], st);
    }
    // the last projection is joined by the wait before the last spot launch
    return e;
  }
  if (!pipelined) {
    for (int k = 0; k < n && e == hipSuccess; ++k) e = launch_fwd_modes(P, frame(k), st);
    return e;
  }
  float* buf[2] = {P->d_phase, P->d_phase2};
  {
    FwdParams p = frame(0);
    set_proj(p, P->proj_all);
    e = launch_project(p, buf[0], P->proj_lds, st);
  }
  for (int k = 0; k < n && e == hipSuccess; ++k) {
    FwdParams p = frame(k);
    p.phase_in = buf[k & 1];
    p.otf_from_phase = 1;
    if (k + 1 < n) {
      set_proj(p, P->proj_all);
      p.proj_blocks = P->proj_all.per_real * P->batch;
      p.phase_out = buf[(k + 1) & 1];
    }
    e = launch_groups(P, p, st, &P->side);
  }
  return e;
}

int wfs_forward_steps(wfs_plan_t P, const float* layers, int64_t step0, int32_t n_steps,
                      uint64_t seed, float* slopes, float* aux, void* stream) {
  if (!P) return fail(WFS_EINVAL, "wfs_forward_steps: null plan");
  if (!layers || !slopes) return fail(WFS_EINVAL, "wfs_forward_steps: null layers or slopes");
  if (n_steps < 1) return fail(WFS_EINVAL, "wfs_forward_steps: n_steps=%d < 1", n_steps);
  int rc = check_step(step0, "wfs_forward_steps");
  if (rc) return rc;
  if (step0 >= 0 && step0 > INT64_MAX - n_steps)
    return fail(WFS_EINVAL, "wfs_forward_steps: step overflow");
  rc = check_device(P, "wfs_forward_steps");
  if (rc) return rc;
  hipError_t e = run_steps(P, layers, step0, n_steps, seed, slopes, aux, P->frames,
                           (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "wfs_forward_steps: launch");
  return WFS_OK;
}

int wfs_spots(wfs_plan_t P, const float* phase, int64_t step, uint64_t seed, float* slopes,
              float* aux, void* stream) {
  if (!P) return fail(WFS_EINVAL, "wfs_spots: null plan");
  if (!phase || !slopes) return fail(WFS_EINVAL, "wfs_spots: null phase or slopes");
  int rc = check_step(step, "wfs_spots");
  if (rc) return rc;
  rc = check_device(P, "wfs_spots");
  if (rc) return rc;
  FwdParams p = call_params(P, nullptr, step, seed, slopes, aux);
  p.phase_in = phase;
  p.otf_from_phase = 1;
  hipError_t e = launch_groups(P, p, (hipStream_t)stream, &P->side);
  if (e != hipSuccess) return hip_fail(e, "wfs_spots: launch");
  return WFS_OK;
}

int wfs_plan_schedule(wfs_plan_t P, int32_t* field, int32_t* frames, int32_t* xcd_remap,
                      int32_t* fft_launch, int32_t* proj_rows, int32_t* lag_passes) {
  if (!P) return fail(WFS_EINVAL, "wfs_plan_schedule: null plan");
  const bool split = P->split && P->d_phase;
  if (field) *field = P->foot ? 2 : (split ? 1 : 0);
  if (frames) *frames = P->frames;
  if (xcd_remap) *xcd_remap = P->base.xcd_remap;
  if (fft_launch) *fft_launch = P->base.fft_inline;
  if (proj_rows) *proj_rows = P->proj_sets[P->proj_set].rows;
  if (lag_passes) *lag_passes = P->lag_parts;
  return WFS_OK;
}

int wfs_plan_set_schedule(wfs_plan_t P, int32_t field, int32_t frames, int32_t xcd_remap,
                          int32_t fft_launch, int32_t proj_rows, int32_t lag_passes) {
  if (!P) return fail(WFS_EINVAL, "wfs_plan_set_schedule: null plan");
  if (field < -1 || field > 2 || frames < -1 || frames > 3 || xcd_remap < -1 ||
      xcd_remap > 1 || fft_launch < -1 || fft_launch > 1 || proj_rows < -1 ||
      !(lag_passes == -1 || lag_passes == 2 || lag_passes == 3))
    return fail(WFS_EINVAL, "wfs_plan_set_schedule: field=%d frames=%d xcd_remap=%d "
                "fft_launch=%d proj_rows=%d lag_passes=%d out of range", field, frames,
                xcd_remap, fft_launch, proj_rows, lag_passes);
  int ps = P->proj_set;
  if (proj_rows >= 0) {
    ps = -1;
    for (size_t i = 0; i < P->proj_sets.size(); ++i)
      if (P->proj_sets[i].rows == proj_rows) ps = (int)i;
    if (ps < 0)
      return fail(WFS_EUNSUPPORTED,
                  "wfs_plan_set_schedule: the plan offers no projection blocks of %d rows "
                  "(%d to %d, doubling, where a block's taps fit 32 KiB of LDS)",
                  proj_rows, P->proj_sets.front().rows, P->proj_sets.back().rows);
  }
  const int cur_field = P->foot ? 2 : ((P->split && P->d_phase) ? 1 : 0);
  const int f = field < 0 ? cur_field : field;
  const int fr = frames < 0 ? P->frames : frames;
  const bool phase_ok = P->d_phase && P->proj_lds <= 65536;
  if (f == 1 && !phase_ok)
    return fail(WFS_EUNSUPPORTED, "wfs_plan_set_schedule: no phase buffer for the split field");
  if (f == 2 && !(P->foot_ok && P->fft_tasks == 0))
    return fail(WFS_EUNSUPPORTED,
                "wfs_plan_set_schedule: a sensor cannot take the footprint field for single "
                "frames");
  if ((fr == 1 || fr == 3) && !phase_ok)
    return fail(WFS_EUNSUPPORTED, "wfs_plan_set_schedule: no phase buffer for pipelined frames");
  if (fr == 2 && !P->foot_ok)
    return fail(WFS_EUNSUPPORTED,
                "wfs_plan_set_schedule: a lag-domain sensor cannot stage its footprint");
  if (fr != 0 && f == 0)
    return fail(WFS_EUNSUPPORTED,
                "wfs_plan_set_schedule: frames in a row need the split or footprint field");
  P->split = f == 1 ? 1 : (f == 0 ? 0 : P->split);
  P->foot = f == 2;
  P->frames = fr;
  if (xcd_remap >= 0) P->base.xcd_remap = xcd_remap;
  if (fft_launch >= 0) P->base.fft_inline = fft_launch;
  use_proj_set(P, ps);
  if (lag_passes > 0) use_lag_parts(P, lag_passes);
  return WFS_OK;
}

int wfs_plan_footprint(wfs_plan_t P, int64_t step, int64_t* distinct_layer_pixels,
                       int64_t* phase_pixels) {
  if (!P) return fail(WFS_EINVAL, "wfs_plan_footprint: null plan");
  if (step < 0) return fail(WFS_EINVAL, "wfs_plan_footprint: step < 0");
  int64_t total = 0;
  for (int l = 0; l < P->n_layers; ++l) {
    const wfs_layer_desc& L = P->layers[l];
    std::vector<uint8_t> hit((size_t)L.nx * L.ny, 0);
    for (int s = 0; s < P->n_sensors; ++s) {
      const wfs_sensor_desc& S = P->sensors[s];
      SensorGeom g = sensor_geometry(S);
      const double H = S.src_alt_m;
      const double sc = finite_d(H) ? 1.0 - L.alt_m / H : 1.0;
      const double t = (double)step * P->dt;
      auto idx = [&](double c, int n, std::vector<int>& out) {
        out.clear();
        const double f = std::floor(c);
        for (int k = 0; k < 2; ++k) {
          long long i = (long long)f + k;
          if (L.boundary == 0) {
            i %= n;
            if (i < 0) i += n;
          } else if (i < 0 || i >= n) {
            continue;
          }
          out.push_back((int)i);
        }
      };
      std::vector<int> us, vs;
      const int ns = S.n_sub;
      for (const DevSubap& q : g.subs)
        for (int r = 0; r < ns; ++r) {
          const double y = ((q.a * ns + r) + 0.5 - g.n_pup / 2.0) * g.dx;
          const double Y = sc * y + S.theta_y_rad * L.alt_m - L.vy_mps * t;
          idx(Y / L.pitch_m + L.ny / 2.0 - 0.5, L.ny, vs);
          for (int c = 0; c < ns; ++c) {
            const double x = ((q.b * ns + c) + 0.5 - g.n_pup / 2.0) * g.dx;
            const double X = sc * x + S.theta_x_rad * L.alt_m - L.vx_mps * t;
            idx(X / L.pitch_m + L.nx / 2.0 - 0.5, L.nx, us);
            for (int vv : vs)
              for (int uu : us) hit[(size_t)vv * L.nx + uu] = 1;
          }
        }
    }
    for (uint8_t v : hit) total += v;
  }
  if (distinct_layer_pixels) *distinct_layer_pixels = total;
  if (phase_pixels) *phase_pixels = P->phase_per_real;
  return WFS_OK;
}

int wfs_project(wfs_plan_t P, const float* layers, int64_t step, float* phase, void* stream) {
  if (!P) return fail(WFS_EINVAL, "wfs_project: null plan");
  if (!layers || !phase) return fail(WFS_EINVAL, "wfs_project: null layers or phase");
  int rc = check_step(step, "wfs_project");
  if (rc) return rc;
  rc = check_device(P, "wfs_project");
  if (rc) return rc;
  if (P->proj_lds > 65536)
    return fail(WFS_EUNSUPPORTED, "wfs_project: %d bytes of LDS per block exceed 64 KiB",
                P->proj_lds);
  FwdParams p = call_params(P, layers, step, 0, nullptr, nullptr);
  set_proj(p, P->proj_all);
  hipError_t e = launch_project(p, phase, P->proj_lds, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "wfs_project: launch");
  return WFS_OK;
}

int wfs_set_step(wfs_plan_t P, int64_t step, void* stream) {
  if (!P) return fail(WFS_EINVAL, "wfs_set_step: null plan");
  if (step < 0) return fail(WFS_EINVAL, "wfs_set_step: step=%lld < 0", (long long)step);
  int rc = check_device(P, "wfs_set_step");
  if (rc) return rc;
  hipError_t e = launch_step(P->d_step, step, 0, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "wfs_set_step: launch");
  return WFS_OK;
}

int wfs_advance_step(wfs_plan_t P, int64_t delta, void* stream) {
  if (!P) return fail(WFS_EINVAL, "wfs_advance_step: null plan");
  int rc = check_device(P, "wfs_advance_step");
  if (rc) return rc;
  hipError_t e = launch_step(P->d_step, delta, 1, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "wfs_advance_step: launch");
  return WFS_OK;
}

int wfs_adjoint(wfs_plan_t P, const float* layers, const float* grad_slopes,
                const float* fwd_slopes, const float* fwd_aux, int64_t step, float* grad_layers,
                void* stream) {
  if (!P) return fail(WFS_EINVAL, "wfs_adjoint: null plan");
  if (!layers || !grad_slopes || !grad_layers)
    return fail(WFS_EINVAL, "wfs_adjoint: null layers, grad_slopes or grad_layers");
  if ((fwd_slopes == nullptr) != (fwd_aux == nullptr))
    return fail(WFS_EINVAL, "wfs_adjoint: give both fwd_slopes and fwd_aux, or neither");
  int rc = check_step(step, "wfs_adjoint");
  if (rc) return rc;
  rc = check_device(P, "wfs_adjoint");
  if (rc) return rc;
  if (P->otf_tasks > 0 && P->adj_lds_per_wave == 0)
    return fail(WFS_EUNSUPPORTED, "wfs_adjoint: lag-domain adjoint needs more than 64 KiB of LDS");
  const bool fft = P->fft_tasks > 0;
  if (fft && ((P->flags & WFS_FLAG_ADJOINT_ATOMIC) || P->pupil_per_real >= (1LL << 30)))
    return fail(WFS_EUNSUPPORTED,
                "wfs_adjoint: FFT-path sensors take the gather form only (no atomic scatter)");
  if (fft && !P->d_phase)
    return fail(WFS_EUNSUPPORTED, "wfs_adjoint: FFT-path sensors need the plan's phase buffer");
  AdjParams a;
  a.f = call_params(P, layers, step, 0, nullptr, nullptr);
  a.f.noise_on = 0;
  a.grad_slopes = grad_slopes;
  a.fwd_slopes = fwd_slopes;
  a.fwd_aux = fwd_aux;
  a.grad_layers = grad_layers;
  // gather mode (default): phase gradients into the second phase buffer, then the layer
  // gather; atomic mode: each pupil pixel scatters its taps
  const bool gather = !(P->flags & WFS_FLAG_ADJOINT_ATOMIC) &&
                      P->pupil_per_real < (1LL << 30);  // 32-bit byte offsets in the images
  if (gather && !P->d_gimg) {  // phase-gradient images, allocated on the first gather call
    hipError_t ea = hipMalloc((void**)&P->d_gimg,
                              sizeof(float) * (size_t)P->pupil_per_real * P->batch);
    if (ea != hipSuccess) {
      P->d_gimg = nullptr;
      return hip_fail(ea, "wfs_adjoint: phase-gradient images");
    }
  }
  if (fft && !P->d_adj_fwd) {  // FFT path: chunk shares and the forward outputs it needs
    hipError_t ea = hipMalloc((void**)&P->d_adj_fwd,
                              sizeof(float) * (size_t)(P->n_slopes + P->n_valid_total) * P->batch);
    if (ea == hipSuccess && P->fft_adj_per_real > 0)
      ea = hipMalloc((void**)&P->d_fft_adj,
                     sizeof(float) * (size_t)P->fft_adj_per_real * P->batch);
    if (ea != hipSuccess) {
      if (P->d_adj_fwd) (void)hipFree(P->d_adj_fwd);
      P->d_adj_fwd = nullptr;
      P->d_fft_adj = nullptr;
      return hip_fail(ea, "wfs_adjoint: FFT-path buffers");
    }
  }
  if (gather && P->adj_ent > 0 && !P->d_adj_tab) {  // and the gather's stencil lists
    hipError_t ea = hipMalloc((void**)&P->d_adj_tab, sizeof(int2) * (size_t)P->adj_ent);
    if (ea != hipSuccess) {
      P->d_adj_tab = nullptr;
      return hip_fail(ea, "wfs_adjoint: stencil lists");
    }
  }
  a.gpsi = gather ? P->d_gimg : nullptr;
  a.f.lds_per_wave = P->adj_lds_per_wave;
  hipError_t e = hipSuccess;
  if ((P->split || P->foot) && P->d_phase) {  // subaperture fields from the projection kernel's phase
    set_proj(a.f, P->proj_all);
    e = launch_project(a.f, P->d_phase, P->proj_lds, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "wfs_adjoint: projection launch");
    a.f.phase_in = P->d_phase;
    a.f.otf_from_phase = 1;
  }
  if (fft) {
    // FFT-path sensors need the noise-free forward outputs (run them when not given) and
    // the projected phase of their pixels
    if (!a.fwd_slopes) {
      FwdParams q = call_params(P, layers, step, 0, P->d_adj_fwd,
                                P->d_adj_fwd + (int64_t)P->n_slopes * P->batch);
      q.noise_on = 0;
      e = launch_fwd_modes(P, q, (hipStream_t)stream);
      if (e != hipSuccess) return hip_fail(e, "wfs_adjoint: forward for the FFT-path sensors");
      a.fwd_slopes = P->d_adj_fwd;
      a.fwd_aux = P->d_adj_fwd + (int64_t)P->n_slopes * P->batch;
    }
    if (!a.f.phase_in) {
      set_proj(a.f, P->proj_fft);
      e = launch_project(a.f, P->d_phase, P->proj_lds_fft, (hipStream_t)stream);
      if (e != hipSuccess) return hip_fail(e, "wfs_adjoint: projection launch");
      a.f.phase_in = P->d_phase;
    }
  }
  a.fft_adj_part = P->d_fft_adj;
  a.fft_adj_per_real = P->fft_adj_per_real;
  e = launch_adjoint(a, P->otf_ns ? P->otf_ns : 2, P->adj_clear_grad, true, (hipStream_t)stream);
  for (size_t g = 1; g < P->groups.size() && e == hipSuccess; ++g) {
    AdjParams ag = a;  // the other subaperture sizes add their sensors' shares
    ag.f.otf = P->groups[g].tasks;
    ag.f.lds_per_wave = P->groups[g].lds_adj;
    e = launch_adjoint(ag, P->groups[g].ns, false, false, (hipStream_t)stream);
  }
  if (e != hipSuccess) return hip_fail(e, "wfs_adjoint: launch");
  if (fft) {
    e = launch_adjoint_fft(a, P->fft_adj_lds, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "wfs_adjoint: FFT-path launch");
  }
  if (gather) {
    e = launch_adjoint_gather_tab(a.f, P->d_gimg, grad_layers, P->d_adj_tab, P->d_adj_segs,
                                  P->adj_nseg, P->adj_maxn, P->d_adj_tab_off,
                                  P->gather_tab_blk.data(), (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "wfs_adjoint: tabled gather launch");
    e = launch_adjoint_gather(a.f, P->d_gimg, grad_layers, P->gather_blk.data(),
                              (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "wfs_adjoint: gather launch");
  }
  return WFS_OK;
}

int wfs_plan_tune(wfs_plan_t P, const float* layers, int32_t iters, double* best_us,
                  void* stream) {
  if (!P || !layers) return fail(WFS_EINVAL, "wfs_plan_tune: null argument");
  if (iters < 1 || iters > 10000) return fail(WFS_EINVAL, "wfs_plan_tune: iters=%d", iters);
  int rc = check_device(P, "wfs_plan_tune");
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const int nf = std::max(2, iters);  // frames of the multi-frame candidates
  float *slopes = nullptr, *aux = nullptr;
  HIP_TRY(hipMalloc((void**)&slopes,
                    sizeof(float) * (size_t)std::max(1, P->n_slopes) * P->batch * nf),
          "wfs_plan_tune: scratch");
  hipError_t e = hipMalloc((void**)&aux,
                           sizeof(float) * (size_t)std::max(1, P->n_valid_total) * P->batch * nf);
  if (e != hipSuccess) {
    (void)hipFree(slopes);
    return hip_fail(e, "wfs_plan_tune: scratch");
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  auto elapsed_ms = [&]() {
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return (double)ms;
  };
  const FwdParams keep = P->base;
  const int keep_split = P->split, keep_foot = P->foot, keep_frames = P->frames;
  const int keep_ps = P->proj_set, keep_lp = P->lag_parts;
  // candidates (field, frames, block order, FFT-path blocks in the lag-domain launch,
  // projection tile height), timed on nf frames in a row (the stepping loop the plan serves);
  // only schedules whose single frames and frames in a row give the same bits: the gather
  // field steps frame by frame, the split and footprint fields share their bits with
  // pipelined and one-launch frames; every tile height gives the same bits
  struct Cand {
    int field, frames, remap, inl, ps, lp;
  };
  std::vector<Cand> cands;
  const bool has_fft = P->fft_tasks > 0, mixed = P->fft_tasks > 0 && P->otf_tasks > 0;
  const bool phase_ok = P->d_phase && P->proj_lds <= 65536;
  const bool foot1 = P->foot_ok && !has_fft;  // footprint field for single frames
  const uint32_t fl = P->flags;
  const int n_ps = (int)P->proj_sets.size();
  // the tile heights of the projection kernel, for a schedule that launches it (the split
  // field, and the FFT-path sensors of any field)
  // and, for the split field's spot kernel, the lag row in 2 or 3 passes
  auto add = [&](Cand c) {
    const bool proj = c.field == 1 || has_fft;
    const bool split_spots = c.field == 1 || c.frames == 1 || c.frames == 3;
    for (int ps = 0; ps < (proj ? n_ps : 1); ++ps)
      for (int lp = 2; lp <= (split_spots ? 3 : 2); ++lp) {
        c.ps = proj ? ps : keep_ps;
        c.lp = split_spots ? lp : keep_lp;
        cands.push_back(c);
      }
  };
  for (int remap = 0; remap < 2; ++remap)
    for (int inl = 0; inl < (mixed ? 2 : 1); ++inl) {
      if (!(fl & (WFS_FLAG_SPLIT | WFS_FLAG_FOOTPRINT))) add({0, 0, remap, inl, 0, 0});
      if (phase_ok && !(fl & WFS_FLAG_FUSED)) {
        if (!((fl & WFS_FLAG_FOOTPRINT) && foot1)) {
          add({1, 0, remap, inl, 0, 0});
          add({1, 1, remap, inl, 0, 0});
          if (P->ovl.stream) add({1, 3, remap, inl, 0, 0});
        }
      }
      if (inl == 0 && P->foot_ok && !(fl & (WFS_FLAG_FUSED | WFS_FLAG_SPLIT)) &&
          (foot1 || phase_ok))
        add({foot1 ? 2 : 1, 2, remap, 0, 0, 0});
    }
  auto apply = [&](const Cand& c) {
    P->base = keep;
    P->base.xcd_remap = c.remap;
    P->base.fft_inline = c.inl;
    use_proj_set(P, c.ps);
    use_lag_parts(P, c.lp);
    P->split = c.field == 1;
    P->foot = c.field == 2;
    P->frames = c.frames;
  };
  // every candidate once (after a warm-up), then the four fastest three more times each: the
  // fastest minimum wins (single timings of a few frames differ by several per cent)
  auto time_cand = [&](size_t i, bool warm) {
    apply(cands[i]);
    if (warm) e = run_steps(P, layers, 0, nf, 1, slopes, aux, P->frames, st);
    if (e != hipSuccess) return 1e30;
    (void)hipEventRecord(e0, st);
    e = run_steps(P, layers, 0, nf, 1, slopes, aux, P->frames, st);
    (void)hipEventRecord(e1, st);
    const double ms = elapsed_ms();
    return e == hipSuccess ? ms : 1e30;
  };
  std::vector<std::pair<double, int>> first;
  for (size_t i = 0; i < cands.size() && e == hipSuccess; ++i)
    first.push_back({time_cand(i, true), (int)i});
  std::sort(first.begin(), first.end());
  double best_t = 1e30;
  int best_i = -1;
  for (size_t r = 0; r < first.size() && r < 4 && e == hipSuccess; ++r) {
    double t = first[r].first;
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep)
      t = std::min(t, time_cand((size_t)first[r].second, rep == 0));
    if (e == hipSuccess && t < best_t) {
      best_t = t;
      best_i = first[r].second;
    }
  }
  double single_us = 0.0;
  if (e == hipSuccess && best_i >= 0) {
    Cand c = cands[best_i];
    apply(c);
    // single frames of the chosen schedule: the split and footprint fields share their bits,
    // keep the faster for one wfs_forward
    auto time_single = [&]() {
      FwdParams q = call_params(P, layers, 0, 1, slopes, aux);
      hipError_t r = launch_fwd_modes(P, q, st);
      (void)hipEventRecord(e0, st);
      for (int it = 0; it < iters && r == hipSuccess; ++it) r = launch_fwd_modes(P, q, st);
      (void)hipEventRecord(e1, st);
      e = r;
      return 1000.0 * elapsed_ms() / iters;
    };
    single_us = time_single();
    if (e == hipSuccess && c.frames != 0 && foot1 && phase_ok && !(fl & WFS_FLAG_SPLIT)) {
      Cand other = c;
      other.field = c.field == 2 ? 1 : 2;
      apply(other);
      const double us2 = time_single();
      if (e == hipSuccess && us2 < single_us) single_us = us2;
      else apply(c);
    }
  }
  if (e == hipSuccess && best_i < 0) e = hipErrorInvalidValue;  // no schedule could run
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(slopes);
  (void)hipFree(aux);
  if (e != hipSuccess) {
    P->base = keep;
    use_proj_set(P, keep_ps);
    use_lag_parts(P, keep_lp);
    P->split = keep_split;
    P->foot = keep_foot;
    P->frames = keep_frames;
    return hip_fail(e, "wfs_plan_tune: launch");
  }
  if (best_us) *best_us = single_us;
  return WFS_OK;
}

int recon_apply(const float* R, int32_t M, int32_t N, const float* S, int32_t B, float* C,
                int64_t ldc, float alpha, float beta, void* stream) {
  if (!R || !S || !C) return fail(WFS_EINVAL, "recon_apply: null R, S or C");
  if (M < 1 || N < 1 || B < 1)
    return fail(WFS_EINVAL, "recon_apply: M=%d N=%d B=%d must be >= 1", M, N, B);
  if (ldc < M) return fail(WFS_EINVAL, "recon_apply: ldc=%lld < M=%d", (long long)ldc, M);
  if ((int64_t)M * N > (1LL << 40)) return fail(WFS_EINVAL, "recon_apply: R too large");
  if (!std::isfinite(alpha) || !std::isfinite(beta))
    return fail(WFS_EINVAL, "recon_apply: non-finite alpha or beta");
  hipStream_t st = (hipStream_t)stream;
  int64_t floats = 0;
  hipError_t e = recon_work_floats(R, M, N, S, B, &floats);
  if (e != hipSuccess) return hip_fail(e, "recon_apply");
  float* ws = nullptr;
  bool capturing = false;
  e = recon_stream_work(st, floats, &ws, &capturing);
  if (capturing)
    return fail(WFS_EINVAL,
                "recon_apply: the stream is capturing a graph and its workspace must grow to "
                "%lld floats: call recon_apply once with this size (or larger) on this stream "
                "before the capture",
                (long long)floats);
  if (e != hipSuccess) return hip_fail(e, "recon_apply: workspace");
  int mfma = 0;
  e = recon_launch(R, M, N, S, B, C, ldc, alpha, beta, ws, floats, st, &mfma);
  if (e != hipSuccess) return hip_fail(e, "recon_apply");
  return WFS_OK;
}

int recon_apply_noalloc(const float* R, int32_t M, int32_t N, const float* S, int32_t B,
                        float* C, int64_t ldc, float alpha, float beta, void* stream) {
  if (!R || !S || !C) return fail(WFS_EINVAL, "recon_apply_noalloc: null R, S or C");
  if (M < 1 || N < 1 || B < 1)
    return fail(WFS_EINVAL, "recon_apply_noalloc: M=%d N=%d B=%d must be >= 1", M, N, B);
  if (ldc < M)
    return fail(WFS_EINVAL, "recon_apply_noalloc: ldc=%lld < M=%d", (long long)ldc, M);
  if ((int64_t)M * N > (1LL << 40)) return fail(WFS_EINVAL, "recon_apply_noalloc: R too large");
  if (!std::isfinite(alpha) || !std::isfinite(beta))
    return fail(WFS_EINVAL, "recon_apply_noalloc: non-finite alpha or beta");
  int64_t need = 0;
  hipError_t e = recon_min_work_floats(R, M, N, S, B, &need);
  if (e != hipSuccess) return hip_fail(e, "recon_apply_noalloc");
  const int64_t cap = recon_static_work_floats();
  if (need > cap)
    return fail(WFS_EINVAL,
                "recon_apply_noalloc: M=%d rows x %d realisations per tile need %lld floats of "
                "partial sums, above the fixed workspace of %lld floats (M * min(B, 16) <= "
                "%lld)",
                M, (int)(need / M), (long long)need, (long long)cap,
                (long long)cap);
  float* ws = nullptr;
  e = recon_static_work(&ws);
  if (e != hipSuccess) return hip_fail(e, "recon_apply_noalloc: workspace address");
  int mfma = 0;
  e = recon_launch(R, M, N, S, B, C, ldc, alpha, beta, ws, cap, (hipStream_t)stream, &mfma);
  if (e != hipSuccess) return hip_fail(e, "recon_apply_noalloc");
  return WFS_OK;
}

// Calibration workspace: a [B][layer_stride] layer batch, then [B][n_slopes] slopes and
// [B][n_valid_total] fluxes, each region starting on a 64-float boundary.
static int64_t round64(int64_t x) { return (x + 63) / 64 * 64; }

static int64_t calib_floats(wfs_plan_t P, int64_t* o_slopes, int64_t* o_aux) {
  const int64_t B = P->batch;
  const int64_t a = round64(B * P->layer_stride);
  const int64_t b = a + round64(B * P->n_slopes);
  if (o_slopes) *o_slopes = a;
  if (o_aux) *o_aux = b;
  return b + round64(B * P->n_valid_total);
}

int wfs_calibrate_work(wfs_plan_t P, int64_t* work_floats) {
  if (!P || !work_floats) return fail(WFS_EINVAL, "wfs_calibrate_work: null argument");
  *work_floats = calib_floats(P, nullptr, nullptr);
  return WFS_OK;
}

int wfs_calibrate(wfs_plan_t P, const float* base, int64_t act_offset, int32_t n_act,
                  float amplitude, int64_t step, uint64_t seed, float* im, int64_t ld_im,
                  float* ref_slopes, float* work, int64_t work_floats, void* stream) {
  if (!P) return fail(WFS_EINVAL, "wfs_calibrate: null plan");
  if (!work) return fail(WFS_EINVAL, "wfs_calibrate: null work");
  if (P->batch < 2 || P->batch % 2)
    return fail(WFS_EINVAL, "wfs_calibrate: plan batch %d must be even and >= 2", P->batch);
  if (n_act < 0) return fail(WFS_EINVAL, "wfs_calibrate: n_act=%d < 0", n_act);
  if (n_act > 0 && !im) return fail(WFS_EINVAL, "wfs_calibrate: null im");
  if (act_offset < 0 || act_offset + n_act > P->layer_stride)
    return fail(WFS_EINVAL, "wfs_calibrate: actuators [%lld, %lld) outside the layer stride %lld",
                (long long)act_offset, (long long)(act_offset + n_act),
                (long long)P->layer_stride);
  if (!std::isfinite(amplitude) || amplitude == 0.0f)
    return fail(WFS_EINVAL, "wfs_calibrate: amplitude must be finite and non-zero");
  if (ld_im < P->n_slopes)
    return fail(WFS_EINVAL, "wfs_calibrate: ld_im=%lld < n_slopes=%d", (long long)ld_im,
                P->n_slopes);
  int rc = check_step(step, "wfs_calibrate");
  if (rc) return rc;
  if (step == WFS_STEP_DEVICE)
    return fail(WFS_EINVAL, "wfs_calibrate: step must be an explicit step >= 0");
  const int32_t h = P->batch / 2;
  const int64_t chunks = ((int64_t)n_act + h - 1) / h;
  if (chunks > INT32_MAX || step > INT64_MAX - chunks)
    return fail(WFS_EINVAL, "wfs_calibrate: step overflow");
  int64_t o_s = 0, o_a = 0;
  const int64_t need = calib_floats(P, &o_s, &o_a);
  if (work_floats < need)
    return fail(WFS_EINVAL, "wfs_calibrate: work holds %lld floats, needs %lld",
                (long long)work_floats, (long long)need);
  rc = check_device(P, "wfs_calibrate");
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  float* wl = work;
  float* ws = work + o_s;
  float* wa = work + o_a;
  hipError_t e = hipSuccess;
  if (ref_slopes) {  // realisation 0 of an unpoked batch
    if ((e = calib_poke(wl, base, P->layer_stride, h, act_offset, 0, amplitude, st)) !=
        hipSuccess)
      return hip_fail(e, "wfs_calibrate: poke");
    rc = wfs_forward(P, wl, step, seed, ws, wa, stream);
    if (rc) return rc;
    e = hipMemcpyAsync(ref_slopes, ws, (size_t)P->n_slopes * sizeof(float),
                       hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "wfs_calibrate: reference slopes");
  }
  for (int64_t c = 0; c < chunks; ++c) {
    const int32_t j0 = (int32_t)(c * h);
    const int32_t nc = std::min<int32_t>(h, n_act - j0);
    if ((e = calib_poke(wl, base, P->layer_stride, h, act_offset + j0, nc, amplitude, st)) !=
        hipSuccess)
      return hip_fail(e, "wfs_calibrate: poke");
    // every chunk sees the layers at the calibration step; only its noise draws move on
    FwdParams p = call_params(P, wl, step, seed, ws, wa);
    p.noise_dstep = (int32_t)c;
    if ((e = launch_fwd_modes(P, p, st)) != hipSuccess)
      return hip_fail(e, "wfs_calibrate: forward");
    if ((e = calib_diff(ws, h, P->n_slopes, nc, amplitude, im + (int64_t)j0 * ld_im, ld_im,
                        st)) != hipSuccess)
      return hip_fail(e, "wfs_calibrate: difference");
  }
  return WFS_OK;
}

}  // extern "C"
