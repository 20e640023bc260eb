"""Plain FP64 numpy oracle of the Shack-Hartmann wavefront-sensor path.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg may use it.

The paper (Arcidiacono et al., "The numerical simulation tool for the MAORY multiconjugate
adaptive optics system") describes the chain in prose only:
  * Sec. 2.1  static (frozen-flow) phase screens at several altitudes;
  * Sec. 2.2  the open-loop wavefront of each guide star as the geometric projection of the
              screens, the laser guide star being at a finite distance (cone effect);
  * Sec. 2.7  X/Y slopes computed by the wavefront-sensor modules from the residual phase
              (open loop minus DM), slopes times the control matrix giving differential
              coefficients added to the mirror, a pure integrator, the sodium layer;
  * Sec. 1    six LGS feeding as many Shack-Hartmann sensors, three NGS;
  * Sec. 2.3  extra aberrations, among them an extra tip and tilt per NGS sensor;
  * Sec. 2.7  also the temporal evolution of the sodium layer.
Everything inside the Shack-Hartmann model (pupil sampling rule, spot formation by a
zero-padded FFT with a half-pixel centring ramp, Gaussian or multi-peak time-varying sodium
elongation, per-sensor tip-tilt offsets, binning, photon
and read noise, centre of gravity) is one reading of that prose; each function below states
the reading it implements.  Arrays are row-major [y][x]; x runs along columns.

Nothing here is blocked, fused or reordered for speed: it is the definition, with a library
FFT (numpy.fft) and matmul as primitives, vectorised over subapertures only.
"""

import math

import numpy as np

from .philox import philox4x32_10, uniforms_from_words

FWHM_TO_SIGMA = 1.0 / (2.0 * math.sqrt(2.0 * math.log(2.0)))


# --------------------------------------------------------------------------------------------
# Geometry (pupil sampling of Sec. 2: a square grid of pupil pixels; subapertures are square
# blocks of n_sub x n_sub pixels; a subaperture is used if enough of it is illuminated)
# --------------------------------------------------------------------------------------------

def pupil_geometry(sensor):
    """Pupil grid, binary amplitude and the list of valid subapertures.

    n_pup = n_sa * n_sub pixels of pitch dx = D / n_pup; pixel centres
    x_i = (i + 1/2 - n_pup/2) dx.  A = 1 where D_obs/2 <= r <= D/2.  Subaperture (a, b) covers
    rows a*n_sub.. and columns b*n_sub..; it is valid when the mean of A over it is
    >= valid_frac.  Valid subapertures are listed in row-major (a, b) order.
    """
    n_sa, n_sub = int(sensor["n_sa"]), int(sensor["n_sub"])
    n_pup = n_sa * n_sub
    D, Dobs = float(sensor["pupil_d_m"]), float(sensor["obs_d_m"])
    dx = D / n_pup
    xc = (np.arange(n_pup) + 0.5 - n_pup / 2.0) * dx
    X, Y = np.meshgrid(xc, xc)
    r = np.hypot(X, Y)
    A = ((r >= Dobs / 2.0) & (r <= D / 2.0)).astype(np.float64)
    frac = A.reshape(n_sa, n_sub, n_sa, n_sub).mean(axis=(1, 3))
    valid = np.argwhere(frac >= float(sensor["valid_frac"]))
    return dict(n_pup=n_pup, dx=dx, xc=xc, A=A, frac=frac, valid=valid)


def subap_centres(sensor, geo):
    """(x, y) in metres of the centre of each valid subaperture."""
    n_sub, n_pup, dx = int(sensor["n_sub"]), geo["n_pup"], geo["dx"]
    a, b = geo["valid"][:, 0], geo["valid"][:, 1]
    return np.stack([((b + 0.5) * n_sub - n_pup / 2.0) * dx,
                     ((a + 0.5) * n_sub - n_pup / 2.0) * dx], axis=1)


def pixel_scale(sensor):
    """Radians per binned detector pixel: bin * lambda / (n_fft * dx)."""
    dx = float(sensor["pupil_d_m"]) / (int(sensor["n_sa"]) * int(sensor["n_sub"]))
    return int(sensor["bin"]) * float(sensor["lambda_m"]) / (int(sensor["n_fft"]) * dx)


def n_slopes(cfg):
    return sum(2 * len(pupil_geometry(s)["valid"]) for s in cfg["sensors"])


# --------------------------------------------------------------------------------------------
# Projection (Sec. 2.1 frozen flow + Sec. 2.2 geometric projection, cone effect for the LGS)
# --------------------------------------------------------------------------------------------

def _layer_coords(L, sensor, geo, step, dt):
    """Continuous layer-pixel coordinates (u per column, v per row) of the pupil pixels.

    A pupil point x seen towards a source at altitude H in direction theta crosses the layer
    at altitude h at  s x + theta h  with  s = 1 - h/H  (s = 1 for a star at infinity); the
    frozen-flow screen moved by v t, so it is sampled at  X = s x + theta h - v t.
    u = X / pitch + n/2 - 1/2 (pixel centres of the layer grid at (j + 1/2 - n/2) pitch).
    """
    H = float(sensor["src_alt_m"])
    h = float(L["alt_m"])
    s = 1.0 - h / H if math.isfinite(H) else 1.0
    t = step * dt
    X = s * geo["xc"] + sensor["theta_x_rad"] * h - L["vx_mps"] * t
    Y = s * geo["xc"] + sensor["theta_y_rad"] * h - L["vy_mps"] * t
    u = X / L["pitch_m"] + L["nx"] / 2.0 - 0.5
    v = Y / L["pitch_m"] + L["ny"] / 2.0 - 0.5
    return u, v


def _bilinear_taps(c, n, boundary):
    """Floor-based linear-interpolation taps along one axis: (i0, i1, w0, w1, ok0, ok1)."""
    c0 = np.floor(c)
    f = c - c0
    c0 = c0.astype(np.int64)
    if boundary == 0:  # periodic screen
        return c0 % n, (c0 + 1) % n, 1.0 - f, f, np.ones_like(f, bool), np.ones_like(f, bool)
    ok0 = (c0 >= 0) & (c0 < n)
    ok1 = (c0 + 1 >= 0) & (c0 + 1 < n)
    return np.clip(c0, 0, n - 1), np.clip(c0 + 1, 0, n - 1), 1.0 - f, f, ok0, ok1


def project(layer_buf, cfg, sensor, step):
    """Pupil phase psi [n_pup][n_pup] in radians at the sensor wavelength.

    psi = (lambda_ref / lambda) * sum_l w_l * bilinear_l(u, v), bilinear with u0 = floor(u),
    indices periodic (screens, boundary 0) or zero outside the grid (DM grids, boundary 1).
    """
    geo = pupil_geometry(sensor)
    psi = np.zeros((geo["n_pup"], geo["n_pup"]))
    for L in cfg["layers"]:
        u, v = _layer_coords(L, sensor, geo, step, cfg["dt_s"])
        grid = np.asarray(layer_buf[L["offset"]:L["offset"] + L["nx"] * L["ny"]],
                          dtype=np.float64).reshape(L["ny"], L["nx"])
        iu0, iu1, wu0, wu1, ou0, ou1 = _bilinear_taps(u, L["nx"], L["boundary"])
        iv0, iv1, wv0, wv1, ov0, ov1 = _bilinear_taps(v, L["ny"], L["boundary"])
        val = np.zeros_like(psi)
        for iv, wv, ov in ((iv0, wv0, ov0), (iv1, wv1, ov1)):
            for iu, wu, ou in ((iu0, wu0, ou0), (iu1, wu1, ou1)):
                g = grid[np.ix_(iv, iu)] * (ov[:, None] & ou[None, :])
                val += wv[:, None] * wu[None, :] * g
        psi += L["weight"] * val
    return psi * (cfg["lambda_ref_m"] / sensor["lambda_m"])


def project_transpose(g_psi, cfg, sensor, step, out):
    """Adjoint of ``project``: accumulate d(loss)/d(layer buffer) into ``out`` (flat)."""
    geo = pupil_geometry(sensor)
    kappa = cfg["lambda_ref_m"] / sensor["lambda_m"]
    for L in cfg["layers"]:
        u, v = _layer_coords(L, sensor, geo, step, cfg["dt_s"])
        iu0, iu1, wu0, wu1, ou0, ou1 = _bilinear_taps(u, L["nx"], L["boundary"])
        iv0, iv1, wv0, wv1, ov0, ov1 = _bilinear_taps(v, L["ny"], L["boundary"])
        acc = np.zeros(L["nx"] * L["ny"])
        for iv, wv, ov in ((iv0, wv0, ov0), (iv1, wv1, ov1)):
            for iu, wu, ou in ((iu0, wu0, ou0), (iu1, wu1, ou1)):
                w = wv[:, None] * wu[None, :] * (ov[:, None] & ou[None, :])
                idx = iv[:, None] * L["nx"] + iu[None, :]
                np.add.at(acc, idx.ravel(), (w * g_psi).ravel())
        out[L["offset"]:L["offset"] + acc.size] += kappa * L["weight"] * acc
    return out


# --------------------------------------------------------------------------------------------
# Shack-Hartmann spots (Sec. 2.7: the sensor turns the residual phase into X/Y slopes)
# --------------------------------------------------------------------------------------------

def subap_fields(psi, geo, sensor):
    """E[m, n] = A exp(i (psi - pi (m + n) / N)) on the n_sub x n_sub corner of an N x N zero
    array, one per valid subaperture ([nv][N][N] complex).  The half-pixel ramp centres the
    diffraction spot of a flat wavefront between the four central detector pixels."""
    n, N = int(sensor["n_sub"]), int(sensor["n_fft"])
    m = np.arange(n)
    ramp = -math.pi * (m[:, None] + m[None, :]) / N
    valid = geo["valid"]
    E = np.zeros((len(valid), N, N), dtype=np.complex128)
    for k, (a, b) in enumerate(valid):
        ph = psi[a * n:(a + 1) * n, b * n:(b + 1) * n]
        amp = geo["A"][a * n:(a + 1) * n, b * n:(b + 1) * n]
        E[k, :n, :n] = amp * np.exp(1j * (ph + ramp))
    return E


def flux(sensor):
    """Photons per fully lit subaperture per frame (1 when the sensor is noise-free)."""
    return float(sensor["photons"]) if sensor["photons"] > 0 else 1.0


def spots(E, sensor):
    """F = DFT2(E) (kernel exp(-2 pi i (k m + l n) / N)); I = F_ph |F|^2 / (N^2 n_sub^2)."""
    n, N = int(sensor["n_sub"]), int(sensor["n_fft"])
    F = np.fft.fft2(E, axes=(1, 2))
    I = flux(sensor) * (F.real ** 2 + F.imag ** 2) / (N * N * n * n)
    return F, I


def na_profile_at(cfg, step):
    """Sodium profile of the frame at time step ``step``: entry step mod T of the plan's table
    cfg["na_profile"] (T entries, each a list of peaks (dh, fwhm, weight)), or None when the
    configuration has no table (each LGS then keeps its own single Gaussian).

    Reading of "the sodium layer temporal evolution" (Sec. 2.7): the profile is a time series
    sampled once per frame and repeated with period T; a peak dh metres above the LGS focus
    altitude H, of width fwhm, carries the fraction weight / sum(weights) of the return."""
    table = cfg.get("na_profile")
    if not table:
        return None
    return table[int(step) % len(table)]


def elongation_kernel(sensor, geo, profile=None):
    """Sodium-profile transfer function per valid subaperture ([nv][N][N]).

    Reading of the paper's "sodium layer" (Sec. 2.7): a Gaussian profile of FWHM na_fwhm at
    the LGS altitude H seen from a subaperture at baseline b (centre minus launch position)
    is elongated along e = b/|b| with angular sigma |b| sigma_h / H^2 (first-order parallax),
    i.e. sigma_px = that / (lambda / (N dx)) FFT pixels.  Its transfer function is
    K[ky, kx] = exp(-2 pi^2 sigma_px^2 ((kx~ e_x + ky~ e_y) / N)^2), kx~ the signed frequency
    (k for k < N/2, k - N otherwise).  No elongation (K = 1) for NGS or na_fwhm = 0.

    With a multi-peak ``profile`` (list of (dh, fwhm, weight), see na_profile_at) instead of
    the sensor's single Gaussian: peak j is seen at the angle |b| dh_j / H^2 from the focus
    along e (further from the launch for dh > 0) with the width |b| sigma_j / H^2, so
    K = sum_j w_j exp(-2 pi^2 sigma_px,j^2 u^2) exp(-2 pi i mu_px,j u), u = (kx~ e_x +
    ky~ e_y) / N, w_j the normalised weights and mu_px,j the shift in FFT pixels (complex,
    Hermitian: the spot stays real and moves by mu along e).
    """
    N = int(sensor["n_fft"])
    nv = len(geo["valid"])
    H = float(sensor["src_alt_m"])
    if not (sensor["na_fwhm_m"] > 0 and math.isfinite(H)):
        return np.ones((nv, N, N))
    c = subap_centres(sensor, geo)
    bx = c[:, 0] - sensor["launch_x_m"]
    by = c[:, 1] - sensor["launch_y_m"]
    blen = np.hypot(bx, by)
    p_fft = sensor["lambda_m"] / (N * geo["dx"])
    with np.errstate(invalid="ignore", divide="ignore"):
        ex = np.where(blen > 0, bx / blen, 0.0)
        ey = np.where(blen > 0, by / blen, 0.0)
    k = np.arange(N)
    ks = np.where(k < N // 2, k, k - N).astype(np.float64)
    proj = (ks[None, None, :] * ex[:, None, None] + ks[None, :, None] * ey[:, None, None]) / N
    if profile is None:
        sig_h = sensor["na_fwhm_m"] * FWHM_TO_SIGMA
        sig_px = blen * sig_h / (H * H) / p_fft
        return np.exp(-2.0 * math.pi ** 2 * sig_px[:, None, None] ** 2 * proj ** 2)
    w = np.array([float(pk[2]) for pk in profile])
    w = w / w.sum()
    K = np.zeros((nv, N, N), dtype=np.complex128)
    for (dh, fwhm, _), wj in zip(profile, w):
        sig_px = blen * (float(fwhm) * FWHM_TO_SIGMA) / (H * H) / p_fft
        mu_px = blen * float(dh) / (H * H) / p_fft
        K += wj * np.exp(-2.0 * math.pi ** 2 * sig_px[:, None, None] ** 2 * proj ** 2
                         - 2j * math.pi * mu_px[:, None, None] * proj)
    return K


def tilt_phase(sensor, geo):
    """Extra tip-tilt of one sensor, [n_pup][n_pup] radians at its wavelength.

    Reading of the NGS WFS mispositioning modelled as an extra tip and tilt aberration
    (Sec. 2.3): a sensor offset by the angles (tilt_x, tilt_y) on the sky sees the phase
    2 pi (tilt_x x + tilt_y y) / lambda at the pupil coordinates (x, y) of its pixel centres,
    added to the projected phase (zero when the sensor has no such keys)."""
    tx = float(sensor.get("tilt_x_rad", 0.0))
    ty = float(sensor.get("tilt_y_rad", 0.0))
    n_pup, dx = geo["n_pup"], geo["dx"]
    xc = (np.arange(n_pup) + 0.5 - n_pup / 2.0) * dx
    return 2.0 * math.pi * (tx * xc[None, :] + ty * xc[:, None]) / float(sensor["lambda_m"])


def elongate(I, K):
    """Circular convolution with the sodium profile: I_e = Re IDFT2(DFT2(I) K).  (With
    conj(K) it is the adjoint map: the correlation with the same profile.)"""
    return np.real(np.fft.ifft2(np.fft.fft2(I, axes=(1, 2)) * K, axes=(1, 2)))


def bin_spots(I_e, b):
    """Detector image: S = fftshift(I_e), then b x b block sums -> [nv][N/b][N/b]."""
    S = np.fft.fftshift(I_e, axes=(1, 2))
    nv, N = S.shape[0], S.shape[1]
    n_pix = N // b
    return S.reshape(nv, n_pix, b, n_pix, b).sum(axis=(2, 4))


def noise_normals(n_pix, subap_idx, realisation, sensor_index, step, seed):
    """Standard normals (z1, z2) per binned pixel, [nv][n_pix][n_pix] each.

    Philox4x32-10 with key (seed lo, seed hi) and counter
    (pixel-pair j, subaperture index, (realisation << 8) | sensor index, step); one block
    serves pixels 2j and 2j+1 (row-major pixel order) through two Box-Muller pairs:
    z1 = sqrt(-2 ln u_a) cos(2 pi u_b), z2 = sqrt(-2 ln u_a) sin(2 pi u_b).
    """
    n_pix2 = n_pix * n_pix
    n_pairs = (n_pix2 + 1) // 2
    j = np.arange(n_pairs, dtype=np.uint64)[None, :]
    v = np.asarray(subap_idx, dtype=np.uint64)[:, None]
    c2 = np.uint64(((int(realisation) << 8) | int(sensor_index)) & 0xFFFFFFFF)
    c3 = np.uint64(int(step) & 0xFFFFFFFF)
    w = philox4x32_10(j, v, c2, c3, int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF)
    u = [uniforms_from_words(x) for x in w]
    r_a = np.sqrt(-2.0 * np.log(u[0]))
    r_b = np.sqrt(-2.0 * np.log(u[2]))
    z1 = np.empty((len(subap_idx), 2 * n_pairs))
    z2 = np.empty_like(z1)
    z1[:, 0::2] = r_a * np.cos(2 * math.pi * u[1])
    z2[:, 0::2] = r_a * np.sin(2 * math.pi * u[1])
    z1[:, 1::2] = r_b * np.cos(2 * math.pi * u[3])
    z2[:, 1::2] = r_b * np.sin(2 * math.pi * u[3])
    shape = (len(subap_idx), n_pix, n_pix)
    return z1[:, :n_pix2].reshape(shape), z2[:, :n_pix2].reshape(shape)


def add_noise(B, sensor, realisation, sensor_index, step, seed):
    """B' = B + sqrt(max(B, 0)) z1 + sigma_ro z2 (Gaussian photon and read noise), applied when
    the sensor has a photon budget (photons > 0)."""
    if not sensor["photons"] > 0:
        return B
    z1, z2 = noise_normals(B.shape[1], np.arange(B.shape[0]), realisation, sensor_index, step,
                           seed)
    return B + np.sqrt(np.maximum(B, 0.0)) * z1 + float(sensor["read_noise_e"]) * z2


def centroid(B):
    """Centre of gravity in binned pixels: c_x = sum (p - (n-1)/2) B / sum B, same for y;
    (0, 0) when sum B <= 0.  Returns (c_x, c_y, sum B)."""
    n_pix = B.shape[1]
    x = np.arange(n_pix) - (n_pix - 1) / 2.0
    S = B.sum(axis=(1, 2))
    sx = (B * x[None, None, :]).sum(axis=(1, 2))
    sy = (B * x[None, :, None]).sum(axis=(1, 2))
    ok = S > 0
    cx = np.where(ok, sx / np.where(ok, S, 1.0), 0.0)
    cy = np.where(ok, sy / np.where(ok, S, 1.0), 0.0)
    return cx, cy, S


def sensor_slopes(layer_buf, cfg, s_idx, step, seed, realisation, noise=True, trace=None,
                  noise_step=None):
    """Slopes of one sensor for one realisation: [c_x over valid subaps || c_y], and sum B'.
    The noise is drawn with the step counter ``noise_step`` (default: ``step``, the frame's
    own time step)."""
    sensor = cfg["sensors"][s_idx]
    geo = pupil_geometry(sensor)
    psi = project(layer_buf, cfg, sensor, step) + tilt_phase(sensor, geo)
    E = subap_fields(psi, geo, sensor)
    F, I = spots(E, sensor)
    K = elongation_kernel(sensor, geo, na_profile_at(cfg, step))
    I_e = elongate(I, K)
    B = bin_spots(I_e, int(sensor["bin"]))
    if noise:
        B = add_noise(B, sensor, realisation, s_idx, step if noise_step is None else noise_step,
                      seed)
    cx, cy, S = centroid(B)
    if trace is not None:
        trace.update(psi=psi, E=E, F=F, I=I, K=K, I_e=I_e, B=B, geo=geo)
    return np.concatenate([cx, cy]), S


def forward(layers, cfg, step, seed=42, noise=True, realisations=None, noise_step=None):
    """Slopes [B][N_s] and sum-of-pixels aux [B][n_valid_total] of every sensor, sensors in
    plan order, realisation-major.  ``layers`` is [B][layer_stride].  ``noise_step``: step
    counter of the noise draws when it differs from the frame's time step."""
    layers = np.atleast_2d(np.asarray(layers, dtype=np.float64))
    if realisations is None:
        realisations = range(layers.shape[0])
    slopes, aux = [], []
    for bi, r in enumerate(realisations):
        s_r, a_r = [], []
        for s_idx in range(len(cfg["sensors"])):
            s, S = sensor_slopes(layers[bi], cfg, s_idx, step, seed, r, noise,
                                 noise_step=noise_step)
            s_r.append(s)
            a_r.append(S)
        slopes.append(np.concatenate(s_r))
        aux.append(np.concatenate(a_r))
    return np.array(slopes), np.array(aux)


# --------------------------------------------------------------------------------------------
# Adjoint of the noise-free forward (slopes -> layer screens)
# --------------------------------------------------------------------------------------------

def _sensor_adjoint(layer_buf, cfg, s_idx, step, g_slopes, out):
    sensor = cfg["sensors"][s_idx]
    tr = {}
    sensor_slopes(layer_buf, cfg, s_idx, step, 0, 0, noise=False, trace=tr)
    geo, E, F, K, B = tr["geo"], tr["E"], tr["F"], tr["K"], tr["B"]
    n, N, b = int(sensor["n_sub"]), int(sensor["n_fft"]), int(sensor["bin"])
    nv = len(geo["valid"])
    n_pix = N // b
    cx, cy, S = centroid(B)
    gx, gy = g_slopes[:nv], g_slopes[nv:2 * nv]
    x = np.arange(n_pix) - (n_pix - 1) / 2.0
    ok = S > 0
    Ss = np.where(ok, S, 1.0)
    # d c_x / d B[q, p] = (x_p - c_x) / S ; d c_y / d B[q, p] = (y_q - c_y) / S
    g_B = (gx[:, None, None] * (x[None, None, :] - cx[:, None, None])
           + gy[:, None, None] * (x[None, :, None] - cy[:, None, None])) / Ss[:, None, None]
    g_B *= ok[:, None, None]
    g_S = np.repeat(np.repeat(g_B, b, axis=1), b, axis=2)  # adjoint of the block sum
    g_Ie = np.fft.ifftshift(g_S, axes=(1, 2))  # adjoint of fftshift
    g_I = elongate(g_Ie, np.conj(K))  # adjoint of the convolution: the correlation
    c_I = flux(sensor) / (N * N * n * n)
    G = (N * N) * np.fft.ifft2(g_I * F, axes=(1, 2))  # D^H (g_I . F)
    g_sub = 2.0 * c_I * np.imag(np.conj(E) * G)[:, :n, :n]
    g_psi = np.zeros((geo["n_pup"], geo["n_pup"]))
    for k, (a, bb) in enumerate(geo["valid"]):
        g_psi[a * n:(a + 1) * n, bb * n:(bb + 1) * n] = g_sub[k]
    project_transpose(g_psi, cfg, sensor, step, out)


def adjoint(layers, cfg, step, grad_slopes):
    """d(loss)/d(layers) given d(loss)/d(slopes) of the noise-free forward; [B][layer_stride]."""
    layers = np.atleast_2d(np.asarray(layers, dtype=np.float64))
    grad_slopes = np.atleast_2d(np.asarray(grad_slopes, dtype=np.float64))
    out = np.zeros_like(layers)
    for bi in range(layers.shape[0]):
        o = 0
        for s_idx, sensor in enumerate(cfg["sensors"]):
            nv = len(pupil_geometry(sensor)["valid"])
            _sensor_adjoint(layers[bi], cfg, s_idx, step, grad_slopes[bi, o:o + 2 * nv],
                            out[bi])
            o += 2 * nv
    return out


def loss(layers, cfg, step, target):
    """L = sum (s - s*)^2 over the noise-free slopes."""
    s, _ = forward(layers, cfg, step, noise=False)
    return float(((s - target) ** 2).sum())


# --------------------------------------------------------------------------------------------
# Reconstructor and integrator (Sec. 2.6-2.7)
# --------------------------------------------------------------------------------------------

def recon(R, S):
    """C[b] = R S[b] in FP64: R [M][N] row-major, S [B][N] -> C [B][M]."""
    R = np.asarray(R, dtype=np.float64)
    S = np.atleast_2d(np.asarray(S, dtype=np.float64))
    return S @ R.T


def closed_loop_step(layers, cfg, R, step, seed=42, noise=True, realisations=None):
    """One integrator step: slopes of the residual phase (DM grids enter the projection with
    weight -1), C = R s, and the DM actuators a <- a + g C (rows beyond the actuator count are
    computed and dropped).  ``realisations`` numbers the rows of ``layers`` for the noise
    (default 0 .. B-1).  Returns (new layers, slopes)."""
    layers = np.atleast_2d(np.asarray(layers, dtype=np.float64)).copy()
    s, _ = forward(layers, cfg, step, seed, noise, realisations=realisations)
    C = recon(R, s)
    n_act = sum(L["nx"] * L["ny"] for L in cfg["layers"] if L["weight"] < 0)
    o = cfg["dm_offset"]
    layers[:, o:o + n_act] += cfg["gain"] * C[:, :n_act]
    return layers, s
