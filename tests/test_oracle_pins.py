"""Pins of the FP64 oracle against facts other than itself: known-answer vectors, brute-force
DFTs, closed forms, invariants, exact geometry and finite differences.

Each test is chosen so that a plausible slip in the oracle (a dropped term, a wrong sign or
index, a transposed operand, a wrong normalisation) fails at least one of them.
"""

import math
import os

import numpy as np
import pytest

import oracle
import synth
from synth.configs import ARCSEC

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------------------------------
# helpers: tiny systems
# ------------------------------------------------------------------------------------------

def _sys(sensor, layers, dt=0.002, lam_ref=None):
    cfg = dict(layers=layers, sensors=[sensor], batch=1,
               lambda_ref_m=lam_ref if lam_ref else sensor["lambda_m"], dt_s=dt)
    offs, stride = synth.layer_offsets(layers)
    for L, o in zip(layers, offs):
        L["offset"] = o
    cfg["layer_stride"] = stride
    return cfg


def _ngs(n_sa, n_sub, N, b, D=None, obs=0.0, lam=0.6e-6, photons=0.0, ro=0.0, tx=0.0, ty=0.0):
    D = D if D is not None else float(n_sa * n_sub)
    return dict(theta_x_rad=tx, theta_y_rad=ty, src_alt_m=math.inf, lambda_m=lam, pupil_d_m=D,
                obs_d_m=obs, n_sa=n_sa, n_sub=n_sub, n_fft=N, bin=b, valid_frac=0.5,
                na_fwhm_m=0.0, launch_x_m=0.0, launch_y_m=0.0, photons=photons,
                read_noise_e=ro)


def _lgs(n_sa, n_sub, N, b, D, obs=0.0, fwhm=10e3, tx=0.0, ty=0.0, H=90e3):
    s = _ngs(n_sa, n_sub, N, b, D=D, obs=obs, lam=589e-9, tx=tx, ty=ty)
    s.update(src_alt_m=H, na_fwhm_m=fwhm)
    return s


def _layer(n, pitch, alt=0.0, vx=0.0, vy=0.0, w=1.0, boundary=0):
    return dict(nx=n, ny=n, pitch_m=pitch, alt_m=alt, vx_mps=vx, vy_mps=vy, weight=w,
                boundary=boundary)


def _random_layers(cfg, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(cfg["layer_stride"]) * scale


# ------------------------------------------------------------------------------------------
# Philox4x32-10: published known-answer vectors
# ------------------------------------------------------------------------------------------

def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert oracle.philox4x32_10_scalar(ctr, key) == out
        vec = oracle.philox4x32_10(*[np.array([c]) for c in ctr], key[0], key[1])
        assert [int(v[0]) for v in vec] == out


def test_philox_vectorised_equals_scalar():
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2 ** 32, size=(4, 50), dtype=np.uint64)
    key = (0x12345678, 0x9abcdef0)
    vec = oracle.philox4x32_10(*ctr, *key)
    for i in range(50):
        ref = oracle.philox4x32_10_scalar([int(c[i]) for c in ctr], key)
        assert [int(v[i]) for v in vec] == ref


def test_noise_statistics():
    """Box-Muller normals: mean 0, variance 1, uncorrelated z1/z2; B' has variance B + s^2."""
    z1, z2 = oracle.noise_normals(8, np.arange(4000), realisation=3, sensor_index=2, step=7,
                                  seed=42)
    for z in (z1, z2):
        assert abs(z.mean()) < 0.01
        assert abs(z.var() - 1.0) < 0.01
    assert abs(np.mean(z1 * z2)) < 0.01
    # distinct counters give distinct draws
    z1b, _ = oracle.noise_normals(8, np.arange(4000), realisation=3, sensor_index=2, step=8,
                                  seed=42)
    assert abs(np.corrcoef(z1.ravel(), z1b.ravel())[0, 1]) < 0.01
    sensor = _ngs(1, 4, 16, 2, photons=100.0, ro=3.0)
    B = np.full((4000, 8, 8), 50.0)
    Bn = oracle.add_noise(B, sensor, 0, 0, 0, 42)
    assert abs((Bn - B).mean()) < 0.05
    assert abs((Bn - B).var() / (50.0 + 9.0) - 1.0) < 0.01


# ------------------------------------------------------------------------------------------
# Spots: brute-force DFT, closed form, Parseval
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("n,N", [(2, 4), (3, 6), (4, 8), (3, 8)])
def test_spot_against_brute_force_dft(n, N):
    """I = F_ph |sum_mn A e^{i(psi - pi(m+n)/N)} e^{-2 pi i (km + ln)/N}|^2 / (N^2 n^2), summed
    term by term (the corner pixels of the single subaperture are dark)."""
    sensor = _ngs(1, n, N, 1, photons=7.0)
    geo = oracle.pupil_geometry(sensor)
    A = geo["A"]
    rng = np.random.default_rng(n * 10 + N)
    psi = rng.standard_normal((n, n)) * 2.0
    E = oracle.subap_fields(psi, geo, sensor)
    _, I = oracle.spots(E, sensor)
    ref = np.zeros((N, N))
    for k in range(N):
        for l in range(N):
            acc = 0j
            for m in range(n):
                for q in range(n):
                    ph = psi[m, q] - math.pi * (m + q) / N - 2 * math.pi * (k * m + l * q) / N
                    acc += A[m, q] * complex(math.cos(ph), math.sin(ph))
            ref[k, l] = 7.0 * abs(acc) ** 2 / (N * N * n * n)
    np.testing.assert_allclose(I[0], ref, rtol=0, atol=1e-12)


def test_flat_spot_dirichlet_closed_form():
    """Flat, fully lit n x n subaperture: I[k, l] = F_ph D(k) D(l) / (N^2 n^2) with
    D(k) = sin^2(pi (k + 1/2) n / N) / sin^2(pi (k + 1/2) / N)."""
    n, N = 5, 16
    sensor = _ngs(4, n, N, 4, obs=0.0, photons=3.0)
    geo = oracle.pupil_geometry(sensor)
    psi = np.zeros((4 * n, 4 * n))
    E = oracle.subap_fields(psi, geo, sensor)
    _, I = oracle.spots(E, sensor)
    k = np.arange(N)
    D = np.sin(math.pi * (k + 0.5) * n / N) ** 2 / np.sin(math.pi * (k + 0.5) / N) ** 2
    ref = 3.0 * D[:, None] * D[None, :] / (N * N * n * n)
    inner = [i for i, (a, b) in enumerate(geo["valid"]) if a in (1, 2) and b in (1, 2)]
    assert len(inner) == 4
    for i in inner:
        np.testing.assert_allclose(I[i], ref, rtol=1e-12, atol=1e-15)


def test_parseval_flux():
    """sum I = F_ph * (lit pixels) / n^2; elongation (K[0] = 1) and binning keep the flux."""
    cfg = synth.small_lgs(n_sa=6, n_sub=4, n_fft=8, bin_=2, noise=True)
    cfg["sensors"][0]["photons"] = 250.0
    sensor = cfg["sensors"][0]
    buf = synth.make_layers(cfg, 0).astype(np.float64)
    tr = {}
    oracle.sensor_slopes(buf, cfg, 0, 0, 42, 0, noise=False, trace=tr)
    geo = tr["geo"]
    n = sensor["n_sub"]
    lit = np.array([geo["A"][a * n:(a + 1) * n, b * n:(b + 1) * n].sum() for a, b in geo["valid"]])
    np.testing.assert_allclose(tr["I"].sum(axis=(1, 2)), 250.0 * lit / n ** 2, rtol=1e-12)
    np.testing.assert_allclose(tr["I_e"].sum(axis=(1, 2)), tr["I"].sum(axis=(1, 2)), rtol=1e-12)
    np.testing.assert_allclose(tr["B"].sum(axis=(1, 2)), tr["I"].sum(axis=(1, 2)), rtol=1e-12)
    assert np.all(tr["K"][:, 0, 0] == 1.0)


# ------------------------------------------------------------------------------------------
# Slopes: flat -> 0, shift theorem, symmetries
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["ngs", "lgs", "ngs_small"])
def test_flat_wavefront_gives_zero_slopes(kind):
    """Zero for every subaperture, partly lit ones included (point symmetry of |F|)."""
    if kind == "ngs":
        cfg = synth.config0()
    elif kind == "ngs_small":
        cfg = _sys(_ngs(5, 3, 8, 2, obs=1.5), [_layer(32, 1.0)])
    else:
        cfg = synth.small_lgs(n_sa=8, n_sub=5, n_fft=10, bin_=2)
    s, aux = oracle.forward(np.zeros((1, cfg["layer_stride"])), cfg, 0, noise=False)
    assert np.abs(s).max() < 1e-12
    assert aux.min() > 0


def _tilt_system(n_sa=4, n=4, N=16, b=4, k0=4):
    """NGS at lambda = lambda_ref, layer at h = 0 with the pupil pitch and a planar screen whose
    phase advances by 2 pi k0 / N per pupil pixel along x."""
    sensor = _ngs(n_sa, n, N, b)
    n_pup = n_sa * n
    dx = sensor["pupil_d_m"] / n_pup
    nl = n_pup + 16
    cfg = _sys(sensor, [_layer(nl, dx)])
    u = np.arange(nl, dtype=np.float64)
    plane = np.tile(2 * math.pi * k0 / N * u, (nl, 1))
    return cfg, plane.ravel()


def test_shift_theorem_integer_tilt():
    """A tilt of k0 FFT pixels rolls the spot by k0; for k0 = j b the binned spot rolls by j and
    the slopes equal the centre of gravity of the rolled flat image."""
    N, b, k0 = 16, 4, 4
    cfg, plane = _tilt_system(N=N, b=b, k0=k0)
    flat = np.zeros(cfg["layer_stride"])
    tr0, tr1 = {}, {}
    oracle.sensor_slopes(flat, cfg, 0, 0, 0, 0, noise=False, trace=tr0)
    s1, _ = oracle.sensor_slopes(plane, cfg, 0, 0, 0, 0, noise=False, trace=tr1)
    np.testing.assert_allclose(tr1["I"], np.roll(tr0["I"], k0, axis=2), atol=1e-12)
    np.testing.assert_allclose(tr1["B"], np.roll(tr0["B"], k0 // b, axis=2), atol=1e-12)
    B_roll = np.roll(tr0["B"], k0 // b, axis=2)
    n_pix = N // b
    x = np.arange(n_pix) - (n_pix - 1) / 2
    cx = (B_roll * x[None, None, :]).sum(axis=(1, 2)) / B_roll.sum(axis=(1, 2))
    nv = len(tr0["geo"]["valid"])
    np.testing.assert_allclose(s1[:nv], cx, atol=1e-12)
    np.testing.assert_allclose(s1[nv:], 0.0, atol=1e-12)


def test_small_tilt_moves_centroid_the_right_way():
    """A positive phase gradient along x moves the spot towards +x (and nothing along y)."""
    N, b = 16, 2
    cfg, plane = _tilt_system(N=N, b=b, k0=1)
    s, _ = oracle.sensor_slopes(plane * 0.25, cfg, 0, 0, 0, 0, noise=False)
    nv = len(s) // 2
    assert np.all(s[:nv] > 0.02)
    assert np.abs(s[nv:]).max() < 1e-12


def test_antisymmetry_and_transpose():
    """s(-phi) = -s(phi); transposing the screen swaps (s_x, s_y) between mirrored subaps."""
    sensor = _ngs(6, 4, 8, 2, obs=2.0)
    cfg = _sys(sensor, [_layer(24, 1.0)])
    buf = _random_layers(cfg, 5, scale=0.7)
    sp, _ = oracle.forward(buf[None], cfg, 0, noise=False)
    sm, _ = oracle.forward(-buf[None], cfg, 0, noise=False)
    np.testing.assert_allclose(sm, -sp, atol=1e-12)
    # the layer (24 px, pitch 1) and the pupil (24 px, pitch 1) coincide pixel for pixel
    bufT = buf.reshape(24, 24).T.ravel()
    sT, _ = oracle.forward(bufT[None], cfg, 0, noise=False)
    valid = oracle.pupil_geometry(sensor)["valid"]
    nv = len(valid)
    pos = {(a, b): i for i, (a, b) in enumerate(valid)}
    perm = np.array([pos[(b, a)] for a, b in valid])
    np.testing.assert_allclose(sT[0, :nv], sp[0, nv:][perm], atol=1e-12)
    np.testing.assert_allclose(sT[0, nv:], sp[0, :nv][perm], atol=1e-12)


def test_lgs_antisymmetry_with_elongation():
    cfg = synth.small_lgs(n_sa=6, n_sub=4, n_fft=8, bin_=2, n_layers=2)
    buf = synth.make_layers(cfg, 0).astype(np.float64) * 0.3
    sp, _ = oracle.forward(buf[None], cfg, 0, noise=False)
    sm, _ = oracle.forward(-buf[None], cfg, 0, noise=False)
    np.testing.assert_allclose(sm, -sp, atol=1e-12)
    assert np.abs(sp).max() > 1e-3


# ------------------------------------------------------------------------------------------
# Elongation
# ------------------------------------------------------------------------------------------

def test_elongation_of_a_point_is_a_gaussian_along_the_baseline():
    """A delta spot elongated along e = (1, 0) becomes a (periodised) sampled Gaussian of sigma
    sigma_px along x, untouched along y; the y-marginal of any image is unchanged."""
    N = 32
    sig = 2.5  # transfer function ~4e-14 at Nyquist: no frequency aliasing at 1e-9
    k = np.arange(N)
    ks = np.where(k < N // 2, k, k - N)
    K = np.exp(-2 * math.pi ** 2 * sig ** 2 * (ks[None, :] / N) ** 2)[None]
    K = np.broadcast_to(K, (1, N, N))
    I = np.zeros((1, N, N))
    I[0, 3, 5] = 1.0
    Ie = oracle.elongate(I, K)[0]
    d = np.arange(N) - 5
    g = sum(np.exp(-(d + j * N) ** 2 / (2 * sig ** 2)) for j in (-2, -1, 0, 1, 2))
    g /= math.sqrt(2 * math.pi) * sig
    np.testing.assert_allclose(Ie[3], g, atol=1e-9)
    assert np.abs(np.delete(Ie, 3, axis=0)).max() < 1e-12
    rng = np.random.default_rng(0)
    J = rng.random((1, N, N))
    np.testing.assert_allclose(oracle.elongate(J, K)[0].sum(axis=1), J[0].sum(axis=1), rtol=1e-12)


def test_elongation_geometry():
    """sigma_px = |b| sigma_h / H^2 / (lambda / (N dx)) along the launch-to-subap baseline."""
    sensor = _lgs(8, 4, 16, 2, D=8.0, fwhm=5e3)
    geo = oracle.pupil_geometry(sensor)
    K = oracle.elongation_kernel(sensor, geo)
    c = oracle.subap_centres(sensor, geo)
    N, dx = 16, 8.0 / 32
    for i in range(len(c)):
        bx, by = c[i]
        bl = math.hypot(bx, by)
        sig = bl * 5e3 / (2 * math.sqrt(2 * math.log(2))) / 90e3 ** 2 / (589e-9 / (N * dx))
        # along the baseline direction, frequency (1, 0) projected: e_x / N
        ref = math.exp(-2 * math.pi ** 2 * sig ** 2 * (bx / bl / N) ** 2)
        assert abs(K[i, 0, 1] - ref) < 1e-14
        # perpendicular frequency to e gives K = 1 when e is axis-aligned
        if abs(by) < 1e-12:
            assert abs(K[i, 1, 0] - 1.0) < 1e-14


def test_subap_centres_hand_computed():
    """8 x 8 subapertures of 1 m (8 m pupil, 4 px each): the centre of subaperture (row a,
    column b) is x = b + 1/2 - 4, y = a + 1/2 - 4 metres, worked out by hand for five named
    subapertures (x follows the column, y the row; a swapped axis or a half-subaperture shift
    changes at least one of them)."""
    sensor = _ngs(8, 4, 16, 2, D=8.0)
    geo = oracle.pupil_geometry(sensor)
    c = oracle.subap_centres(sensor, geo)
    where = {(int(a), int(b)): i for i, (a, b) in enumerate(geo["valid"])}
    expect = {(3, 7): (3.5, -0.5), (0, 3): (-0.5, -3.5), (7, 4): (0.5, 3.5),
              (4, 0): (-3.5, 0.5), (0, 2): (-1.5, -3.5)}
    for ab, xy in expect.items():
        assert ab in where, ab
        np.testing.assert_allclose(c[where[ab]], xy, atol=1e-14)
    # the corner subapertures lie outside the 8 m circle: not valid
    assert (0, 0) not in where and (7, 7) not in where


def _spot_variances(sensor):
    """x and y second moments (FFT pixels^2) of the elongated, fftshifted spot of a flat
    wavefront, per valid subaperture."""
    cfg = _sys(sensor, [_layer(64, 0.25)])
    tr = {}
    oracle.sensor_slopes(np.zeros(cfg["layer_stride"]), cfg, 0, 0, 0, 0, noise=False, trace=tr)
    S = np.fft.fftshift(tr["I_e"], axes=(1, 2))
    N = S.shape[1]
    x = np.arange(N) - (N - 1) / 2.0
    tot = S.sum(axis=(1, 2))
    vx = (S * x[None, None, :] ** 2).sum(axis=(1, 2)) / tot
    vy = (S * x[None, :, None] ** 2).sum(axis=(1, 2)) / tot
    where = {(int(a), int(b)): i for i, (a, b) in enumerate(tr["geo"]["valid"])}
    return where, vx, vy


def test_elongation_follows_the_launch_baseline():
    """Sodium elongation stretches each spot along the line from the launch position to the
    subaperture (Sec. 2.7 sodium layer, centre-launch reading).  With the launch at the pupil
    centre a subaperture on the +x side of the pupil has the larger x variance and one on the
    +y side the larger y variance; moving the launch onto a subaperture removes its
    elongation (equal variances: the flat spot of a fully lit square subaperture is
    symmetric) and turns its neighbour one row down (+y) into a y-elongated spot."""
    sensor = _lgs(8, 4, 32, 4, D=8.0, fwhm=3e3)
    where, vx, vy = _spot_variances(sensor)
    for ab in ((3, 7), (4, 7), (3, 0)):      # on the x axis: elongated along x
        i = where[ab]
        assert vx[i] > 2.0 * vy[i], (ab, vx[i], vy[i])
    for ab in ((0, 3), (7, 4)):              # on the y axis: elongated along y
        i = where[ab]
        assert vy[i] > 2.0 * vx[i], (ab, vx[i], vy[i])
    sensor = dict(sensor, launch_x_m=3.5, launch_y_m=-0.5)  # launch at subaperture (3, 7)
    where, vx, vy = _spot_variances(sensor)
    i = where[(3, 7)]
    assert abs(vx[i] - vy[i]) < 1e-9 * vx[i]
    i = where[(4, 7)]                         # baseline (0, +1 m)
    assert vy[i] > vx[i] + 1.0 and abs(vx[i] - vx[where[(3, 7)]]) < 1e-9 * vx[i]


# ------------------------------------------------------------------------------------------
# Projection geometry
# ------------------------------------------------------------------------------------------

def test_projection_exact_on_planes_with_cone_offaxis_and_wind():
    """A screen equal to its own u (or v) pixel coordinate returns, at each pupil pixel, the
    coordinate where the line from that pupil point to the LGS crosses the layer, shifted
    against the wind by v t: bilinear interpolation is exact on planes."""
    n_sa, n = 4, 5
    D = 10.0
    H = 20e3
    tx, ty = 30 * ARCSEC, -45 * ARCSEC
    sensor = _lgs(n_sa, n, 10, 2, D=D, tx=tx, ty=ty, H=H)
    nl, pitch, h = 64, 0.3, 5e3
    vx, vy, step, dt = 7.0, -3.0, 11, 0.002
    lay = [_layer(nl, pitch, alt=h, vx=vx, vy=vy)]
    cfg = _sys(sensor, lay, dt=dt)
    uu = np.tile(np.arange(nl, dtype=float), (nl, 1))
    geo = oracle.pupil_geometry(sensor)
    xc = geo["xc"]
    # line from pupil point (x, y, 0) to source (tx H, ty H, H) at height h
    X = xc + (tx * H - xc) * h / H - vx * step * dt
    Y = xc + (ty * H - xc) * h / H - vy * step * dt
    u_ref = X / pitch + (nl - 1) / 2.0
    v_ref = Y / pitch + (nl - 1) / 2.0
    assert u_ref.min() > 1 and u_ref.max() < nl - 2 and v_ref.min() > 1 and v_ref.max() < nl - 2
    kappa = cfg["lambda_ref_m"] / sensor["lambda_m"]
    pu = oracle.project(uu.ravel(), cfg, sensor, step) / kappa
    pv = oracle.project(uu.T.ravel(), cfg, sensor, step) / kappa
    np.testing.assert_allclose(pu, np.tile(u_ref, (len(xc), 1)), atol=1e-9)
    np.testing.assert_allclose(pv, np.tile(v_ref[:, None], (1, len(xc))), atol=1e-9)


def test_frozen_flow_moves_the_screen_with_the_wind():
    """After t with v t = 3 pixels along x, the sensor sees the screen rolled by +3 pixels."""
    sensor = _ngs(4, 4, 8, 2, obs=0.0)
    pitch = 1.0
    dt = 0.01
    lay = [_layer(32, pitch, vx=3 * pitch / (5 * dt), vy=0.0)]
    cfg = _sys(sensor, lay, dt=dt)
    buf = _random_layers(cfg, 3)
    psi5 = oracle.project(buf, cfg, sensor, 5)
    rolled = np.roll(buf.reshape(32, 32), 3, axis=1).ravel()
    psi0 = oracle.project(rolled, cfg, sensor, 0)
    np.testing.assert_allclose(psi5, psi0, atol=1e-12)


def test_periodic_and_zero_boundaries():
    sensor = _ngs(2, 4, 8, 2)
    n_pup = 8
    # layer smaller than the pupil footprint: periodic wraps, zero boundary clips
    lay = [_layer(4, 1.0)]
    cfg = _sys(sensor, lay)
    buf = np.arange(16, dtype=float)
    psi = oracle.project(buf, cfg, sensor, 0)
    # pupil pixel i samples layer coordinate i - 2 (mod 4)
    ref = buf.reshape(4, 4)[np.ix_((np.arange(n_pup) - 2) % 4, (np.arange(n_pup) - 2) % 4)]
    np.testing.assert_allclose(psi, ref * (cfg["lambda_ref_m"] / sensor["lambda_m"]), atol=1e-12)
    lay[0]["boundary"] = 1
    psi = oracle.project(buf, cfg, sensor, 0)
    inside = (np.arange(n_pup) >= 2) & (np.arange(n_pup) < 6)
    assert np.all(psi[~inside, :] == 0) and np.all(psi[:, ~inside] == 0)


def test_periodic_wrap_equals_tiled_screen():
    """Sampling a periodic n x n screen at fractional, partly negative coordinates equals
    sampling the 3x3-tiled screen (no wrap needed) at the same physical points."""
    sensor = _ngs(3, 5, 10, 2, D=15.0 * 0.7, tx=3e-5, ty=-2e-5)
    lay = [_layer(8, 0.61, alt=3e4, vx=2.3, vy=-1.1)]
    cfg = _sys(sensor, lay)
    buf = _random_layers(cfg, 9)
    psi = oracle.project(buf, cfg, sensor, 4)
    big = np.tile(buf.reshape(8, 8), (3, 3))
    lay3 = [_layer(24, 0.61, alt=3e4, vx=2.3, vy=-1.1)]
    cfg3 = _sys(sensor, lay3)
    psi3 = oracle.project(big.ravel(), cfg3, sensor, 4)
    np.testing.assert_allclose(psi, psi3, atol=1e-12)
    geo = oracle.pupil_geometry(sensor)
    u, _ = oracle.wfs_oracle._layer_coords(lay[0], sensor, geo, 4, cfg["dt_s"])
    assert u.min() < -1.2 and u.max() > 8.5  # really wraps on both sides, off the grid


def test_dm_layer_cancels_equal_turbulence():
    """A DM grid (weight -1) holding the same surface as a turbulence layer gives a flat
    residual, hence zero slopes (the residual is open loop minus DM)."""
    sensor = _ngs(4, 4, 8, 2, obs=1.0)
    lay = [_layer(16, 1.0), _layer(16, 1.0, w=-1.0, boundary=1)]
    cfg = _sys(sensor, lay)
    rng = np.random.default_rng(0)
    scr = rng.standard_normal(256)
    buf = np.concatenate([scr, scr])
    s, _ = oracle.forward(buf[None], cfg, 0, noise=False)
    assert np.abs(s).max() < 1e-12


# ------------------------------------------------------------------------------------------
# Reconstructor
# ------------------------------------------------------------------------------------------

def test_recon_exact_on_integers():
    rng = np.random.default_rng(2)
    R = rng.integers(-4, 5, size=(7, 13)).astype(np.float64)
    S = rng.integers(-3, 4, size=(3, 13)).astype(np.float64)
    C = oracle.recon(R, S)
    for b in range(3):
        for i in range(7):
            assert C[b, i] == sum(R[i, j] * S[b, j] for j in range(13))


# ------------------------------------------------------------------------------------------
# Adjoint: dot products and finite differences
# ------------------------------------------------------------------------------------------

def test_projection_dot_product():
    """<P x, y> = <x, P^T y> for periodic and zero-boundary layers with cone and wind."""
    sensor = _lgs(4, 5, 10, 2, D=10.0, tx=20 * ARCSEC, H=30e3)
    lay = [_layer(40, 0.3, alt=4e3, vx=3.0, vy=1.0),
           _layer(12, 1.0, alt=1e3, w=-1.0, boundary=1)]
    cfg = _sys(sensor, lay)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(cfg["layer_stride"])
    y = rng.standard_normal((20, 20))
    Px = oracle.project(x, cfg, sensor, 3)
    PTy = oracle.project_transpose(y, cfg, sensor, 3, np.zeros_like(x))
    assert abs((Px * y).sum() - (x * PTy).sum()) < 1e-10 * abs((Px * y).sum())


def test_binning_and_elongation_adjoints():
    rng = np.random.default_rng(8)
    N, b = 16, 4
    I = rng.standard_normal((2, N, N))
    g = rng.standard_normal((2, N // b, N // b))
    Bx = oracle.bin_spots(I, b)
    up = np.fft.ifftshift(np.repeat(np.repeat(g, b, axis=1), b, axis=2), axes=(1, 2))
    assert abs((Bx * g).sum() - (I * up).sum()) < 1e-12
    sensor = _lgs(8, 4, N, b, D=8.0)
    K = oracle.elongation_kernel(sensor, oracle.pupil_geometry(sensor))[:2]
    J = rng.standard_normal((2, N, N))
    assert abs((oracle.elongate(I, K) * J).sum() - (I * oracle.elongate(J, K)).sum()) < 1e-12


def _fd_setup():
    cfg = synth.small_lgs(n_sa=4, n_sub=4, n_fft=8, bin_=2, n_layers=2, n=32, pitch=0.5,
                          n_sensors=2)
    x0 = synth.make_layers(cfg, 1).astype(np.float64)[None] * 0.5
    truth = synth.make_layers(cfg, 0).astype(np.float64)[None] * 0.5
    target, _ = oracle.forward(truth, cfg, 2, noise=False)
    return cfg, x0, target


def test_adjoint_against_central_differences():
    """Gradient of L = sum (s - s*)^2 against central differences (h = 1e-4) along random
    directions and single pixels."""
    cfg, x0, target = _fd_setup()
    step = 2
    s0, _ = oracle.forward(x0, cfg, step, noise=False)
    g = oracle.adjoint(x0, cfg, step, 2.0 * (s0 - target))
    rng = np.random.default_rng(11)
    h = 1e-4
    dirs = [rng.standard_normal(x0.shape) for _ in range(6)]
    # single pixels inside the footprint (where the gradient is large)
    for idx in np.argsort(-np.abs(g[0]))[:6]:
        d = np.zeros_like(x0)
        d[0, idx] = 1.0
        dirs.append(d)
    for d in dirs:
        fd = (oracle.loss(x0 + h * d, cfg, step, target)
              - oracle.loss(x0 - h * d, cfg, step, target)) / (2 * h)
        an = float((g * d).sum())
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_closed_loop_step_integrates():
    """a <- a + g R s on the DM actuators; turbulence layers untouched."""
    cfg = synth.config4(batch=1)
    cfg = dict(cfg)
    # shrink to one small sensor so the step is quick
    cfg["sensors"] = [synth.small_lgs(n_sa=4, n_sub=4, n_fft=8, bin_=2)["sensors"][0]]
    cfg["sensors"][0].update(pupil_d_m=39.0, obs_d_m=11.0)
    ns = oracle.n_slopes(cfg)
    rng = np.random.default_rng(4)
    R = rng.standard_normal((cfg["n_act_rows"], ns))
    buf = np.zeros((1, cfg["layer_stride"]))
    buf[0, :1024] = rng.standard_normal(1024)
    new, s = oracle.closed_loop_step(buf, cfg, R, 0, noise=False)
    C = R @ s[0]
    o = cfg["dm_offset"]
    n_act = 40 * 40 + 42 * 42 + 45 * 45
    assert n_act == 5389
    np.testing.assert_allclose(new[0, o:o + n_act], 0.4 * C[:n_act], atol=1e-12)
    np.testing.assert_array_equal(new[0, :o], buf[0, :o])
    np.testing.assert_array_equal(new[0, o + n_act:], buf[0, o + n_act:])


def test_workload_geometry_counts():
    """80x80 subaps on the 39 m / 11 m pupil with the 50 % rule: 4,632 valid; config 2 gives
    55,608 slopes per realisation; 52 valid subaps for the 8 m NGS."""
    assert len(oracle.pupil_geometry(synth.config1()["sensors"][0])["valid"]) == 4632
    assert oracle.n_slopes(synth.config2()) == 55608
    assert len(oracle.pupil_geometry(synth.config0()["sensors"][0])["valid"]) == 52
    cfg = synth.config1()
    assert abs(cfg["sensors"][0]["pupil_d_m"] / 800 - 0.04875) < 1e-15
