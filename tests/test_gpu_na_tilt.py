"""GPU parity, against the FP64 oracle, of the time-varying multi-peak sodium profile (Sec. 2.7,
the sodium layer's temporal evolution) and of per-sensor tip-tilt offsets (Sec. 2.3, NGS WFS
mispositioning): forward slopes in every field schedule, frames in a row, the adjoint, and a
cleared profile giving back the single Gaussian bit for bit."""

import numpy as np
import pytest

import oracle
import synth
from wfs_cases import CASES, layers_for, slope_tolerance

pytestmark = pytest.mark.gpu

# three frames of a drifting profile (dh above the focus, FWHM, weight): a thin peak, a
# single-peak entry (padded with zero-weight peaks on the device), peaks below and above
PROFILE = [
    [(-150.0, 100.0, 0.5), (120.0, 200.0, 0.3), (0.0, 0.0, 0.2)],
    [(50.0, 300.0, 1.0)],
    [(-300.0, 50.0, 0.2), (0.0, 150.0, 0.6), (250.0, 80.0, 0.2)],
]


def _gpu():
    import torch
    import paper_1608_00386_amd as W
    return torch, W


def _flags(W, mode):
    return {"split": W.WFS_FLAG_SPLIT, "fused": W.WFS_FLAG_FUSED,
            "footprint": W.WFS_FLAG_FOOTPRINT}[mode]


def _p_fft(s):
    dx = s["pupil_d_m"] / (s["n_sa"] * s["n_sub"])
    return s["lambda_m"] / (s["n_fft"] * dx)


def _with_tilts(cfg, pixels):
    """Tip-tilt offsets of (px, py) FFT pixels per sensor, cycling through ``pixels``."""
    for k, s in enumerate(cfg["sensors"]):
        px, py = pixels[k % len(pixels)]
        s["tilt_x_rad"] = px * _p_fft(s)
        s["tilt_y_rad"] = py * _p_fft(s)
    return cfg


def _check(cfg, x, s_gpu, a_gpu, step, seed=42):
    s_ref, a_ref = oracle.forward(x.astype(np.float64), cfg, step, seed, noise=True)
    tol = slope_tolerance(cfg)
    err = np.abs(s_gpu - s_ref)
    worst = float((err / tol[None, :]).max())
    assert worst <= 1.0, f"slope error {worst:.3g} x tolerance (max abs {err.max():.3g})"
    np.testing.assert_allclose(a_gpu, a_ref, rtol=2e-5, atol=1e-4 * np.abs(a_ref).max())


def _forward(cfg, x, step, flags):
    torch, W = _gpu()
    plan = W.Plan(cfg, flags=flags, batch=x.shape[0])
    s, a = plan.forward(torch.from_numpy(x).cuda(), step=step, seed=42)
    torch.cuda.synchronize()
    return s.cpu().numpy().astype(np.float64), a.cpu().numpy().astype(np.float64), plan


@pytest.mark.parametrize("name", ["lgs_n4_N8_b2", "lgs_n10_N32_b4_noise",
                                  "lgs_n5_N10_b2_2sens_batch3"])
@pytest.mark.parametrize("step", [0, 1, 2, 4])
@pytest.mark.parametrize("mode", ["split", "fused", "footprint"])
def test_na_profile_forward_matches_oracle(name, step, mode):
    torch, W = _gpu()
    cfg = CASES[name]()
    cfg["na_profile"] = PROFILE
    x = layers_for(cfg)
    s, a, plan = _forward(cfg, x, step, _flags(W, mode))
    _check(cfg, x, s, a, step)
    # the profile really acts: the single Gaussian gives other slopes
    s_g, _ = oracle.forward(x.astype(np.float64), dict(cfg, na_profile=None), step, 42)
    assert np.abs(s - s_g).max() > 1e-2


def test_na_profile_frames_in_a_row_equal_single_frames():
    """wfs_forward_steps over a profile period and beyond: bit for bit the single frames."""
    torch, W = _gpu()
    cfg = CASES["lgs_n10_N32_b4_noise"]()
    cfg["na_profile"] = PROFILE
    x = torch.from_numpy(layers_for(cfg)).cuda()
    for flags in (0, W.WFS_FLAG_SPLIT):
        plan = W.Plan(cfg, flags=flags)
        many, _ = plan.forward_steps(x, 5, 7)
        for k in range(7):
            one, _ = plan.forward(x, step=5 + k)
            assert torch.equal(many[k], one), (flags, k)


def test_cleared_profile_is_the_single_gaussian_bit_for_bit():
    torch, W = _gpu()
    cfg = CASES["lgs_n10_N32_b4_noise"]()
    x = torch.from_numpy(layers_for(cfg)).cuda()
    plain = W.Plan(cfg)
    ref, _ = plain.forward(x, step=3)
    ref = ref.clone()
    plan = W.Plan(dict(cfg, na_profile=PROFILE))
    with_profile, _ = plan.forward(x, step=3)
    assert not torch.equal(with_profile, ref)
    plan.set_na_profile(None)
    again, _ = plan.forward(x, step=3)
    assert torch.equal(again, ref)
    # a longer table (one more entry: period 4) replaces the first one in a new device buffer
    longer = PROFILE + [[(75.0, 120.0, 1.0), (-75.0, 120.0, 1.0)]]
    plan.set_na_profile(longer)
    s7, a7 = plan.forward(x, step=7)
    _check(dict(cfg, na_profile=longer), x.cpu().numpy(), s7.cpu().numpy().astype(np.float64),
           a7.cpu().numpy().astype(np.float64), 7)


def test_na_profile_rejects_bad_tables():
    torch, W = _gpu()
    plan = W.Plan(CASES["lgs_n4_N8_b2"]())
    for bad in ([[(0.0, -1.0, 1.0)]], [[(0.0, 1.0, 0.0)]], [[(float("nan"), 1.0, 1.0)]],
                [[(0.0, 1.0, 1.0)] * 9]):
        with pytest.raises(W.WfsError) as e:
            plan.set_na_profile(bad)
        assert e.value.code == -1


TILTS = [(0.37, -1.25), (-2.5, 0.8)]


@pytest.mark.parametrize("name", ["cfg0", "ngs_n6_N12_b4_oddpix", "fft_ngs_n14_N32_b4",
                                  "fft_ngs_n64_N128_b4", "mixed_lgs_ngs_batch2",
                                  "dm_two_ngs_batch2", "lgs_n5_N10_b2_2sens_batch3"])
@pytest.mark.parametrize("mode", ["split", "fused", "footprint"])
def test_tip_tilt_forward_matches_oracle(name, mode):
    torch, W = _gpu()
    cfg = _with_tilts(CASES[name](), TILTS)
    x = layers_for(cfg)
    s, a, plan = _forward(cfg, x, 6, _flags(W, mode))
    _check(cfg, x, s, a, 6)
    s0, _ = oracle.forward(x.astype(np.float64), _with_tilts(CASES[name](), [(0.0, 0.0)]), 6)
    assert np.abs(s - s0).max() > 1e-2  # the offsets move the spots


def test_tip_tilt_of_whole_binned_pixels_on_a_flat_wavefront():
    """Flat phase and a tilt of exactly b FFT pixels (one binned pixel) along x: the slopes
    follow the rolled diffraction spot, on both kernel paths."""
    torch, W = _gpu()
    for name in ("cfg0", "fft_ngs_n14_N32_b4"):
        cfg = CASES[name]()
        b = cfg["sensors"][0]["bin"]
        cfg = _with_tilts(cfg, [(float(b), 0.0)])
        x = np.zeros((1, cfg["layer_stride"]), np.float32)
        s, a, _ = _forward(cfg, x, 0, 0)
        _check(cfg, x, s, a, 0)
        nv = s.shape[1] // 2
        assert np.all(s[0, :nv] > 0.5) and np.abs(s[0, nv:]).max() < 1e-5


@pytest.mark.parametrize("mode", ["split", "fused", "footprint"])
def test_adjoint_with_profile_and_tilt_matches_oracle(mode):
    torch, W = _gpu()
    cfg = _with_tilts(CASES["lgs_n5_N10_b2_2sens_batch3"](), TILTS)
    cfg["na_profile"] = PROFILE
    for s in cfg["sensors"]:
        s["photons"] = 0.0
        s["read_noise_e"] = 0.0
    x = layers_for(cfg, scale=0.5)
    g = synth.random_field((cfg["batch"], oracle.n_slopes(cfg)), seed=9)
    plan = W.Plan(cfg, flags=_flags(W, mode))
    for step in (1, 5):
        out = plan.adjoint(torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda(), step=step)
        got = out.cpu().numpy().astype(np.float64)
        ref = oracle.adjoint(x.astype(np.float64), cfg, step, g.astype(np.float64))
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert rel <= 1e-4, (step, rel)
        assert np.abs(got - ref).max() <= 1e-3 * np.abs(ref).max()
