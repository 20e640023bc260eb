"""GPU parity of the full-size workloads against the FP64 oracle, element by element:

* one step of the batched system (six LGS on the 60" ring + three NGS on the 80" triangle,
  eight realisations, photon and read noise), realisations 0 and 7 at a step where every
  layer has wrapped;
* the adjoint of the six-LGS loss ||s(phi) - s*||^2 with the target from a seeded truth, at the
  full ten 1024^2 layers;
* one closed-loop step of the system with three DMs and the 5,400 x 55,608 reconstructor
  (integrator gain 0.4), the oracle restarted from the GPU's state;
* a ten-step closed-loop trajectory (noise on, frozen flow moving) of a reduced system with a
  calibrated reconstructor, the GPU and the oracle each on their own trajectory;
* a sensor so dark that many subapertures see a non-positive pixel sum (the (0, 0) branch).

Bars: slopes within 1e-4 of the spot FWHM in binned pixels (per sensor), gradients rel-L2 <=
1e-4 and max <= 1e-3 max|g|, reconstructor outputs within 1e-4 of sum_j |R_ij s_j| plus the
slope bar carried through R."""

import numpy as np
import pytest

import oracle
import synth
from test_oracle_calib import _system
from wfs_cases import slope_tolerance

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    import paper_1608_00386_amd as W
    return torch, W


def _slope_errors(got, want, tol):
    return np.abs(np.asarray(got, np.float64) - want) / tol


def test_batched_config_step_matches_oracle():
    torch, W = _gpu()
    cfg = synth.config2(batch=8)
    x = synth.make_batch(cfg, range(8))
    step = 1500  # 3 s of frozen flow: every layer has moved by 15-90 m (> one period)
    plan = W.Plan(cfg)
    xt = torch.from_numpy(x).cuda()
    s, a = plan.forward(xt, step=step, seed=42)
    s = s.cpu().numpy()
    a = a.cpu().numpy()
    rows = [0, 7]
    want, aux = oracle.forward(x[rows].astype(np.float64), cfg, step, 42, True, realisations=rows)
    tol = slope_tolerance(cfg)
    err = _slope_errors(s[rows], want, tol)
    assert err.max() <= 1.0, f"config-2 slopes: {err.max():.3g} of the bar"
    np.testing.assert_allclose(a[rows], aux, rtol=2e-5, atol=1e-3)
    # the tuned schedule gives the same bits when it keeps a field that shares them (split or
    # footprint); the per-pixel gather has its own bits, held to the same bar
    plan.tune(xt, iters=2)
    s2, _ = plan.forward(xt, step=step, seed=42)
    s2 = s2.cpu().numpy()
    if plan.schedule()["field"] != "gather":
        assert np.array_equal(s2, s)
    else:
        assert _slope_errors(s2[rows], want, tol).max() <= 1.0


def test_adjoint_batched_system_with_ngs_matches_oracle():
    """Gradient through every sensor of the batched system (six LGS on the lag-domain path and
    three 2 x 2 NGS of 64-pixel subapertures on the FFT path, sixteen spectrum chunks each),
    one realisation, noise off, at full size."""
    torch, W = _gpu()
    cfg = synth.config2(batch=1)
    for s in cfg["sensors"]:
        s["photons"] = 0.0
        s["read_noise_e"] = 0.0
    x = synth.make_batch(cfg, [1])
    step = 40
    g = synth.random_field((1, oracle.n_slopes(cfg)), seed=12)
    want = oracle.adjoint(x.astype(np.float64), cfg, step, g.astype(np.float64))
    plan = W.Plan(cfg, batch=1)
    assert 1 in plan.paths and 0 in plan.paths
    got = plan.adjoint(torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda(), step=step)
    got = got.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    mx = np.abs(got - want).max() / np.abs(want).max()
    assert rel <= 1e-4 and mx <= 1e-3, f"rel-L2 {rel:.3g}, max {mx:.3g}"


@pytest.mark.parametrize("saved", [False, True])
def test_adjoint_full_size_matches_oracle(saved):
    """Gradient of L = ||s(phi) - s*||^2 over the six LGS at full size: s* the noise-free
    slopes of the truth (realisation 0), phi realisation 1; dL/ds = 2 (s - s*) from the
    oracle's own slopes."""
    torch, W = _gpu()
    cfg = synth.config3()
    truth = synth.make_batch(cfg, [cfg["truth_realisation"]])
    guess = synth.make_batch(cfg, [cfg["guess_realisation"]])
    step = 40
    s_t, _ = oracle.forward(truth.astype(np.float64), cfg, step, noise=False)
    s_g, _ = oracle.forward(guess.astype(np.float64), cfg, step, noise=False)
    g = 2.0 * (s_g - s_t)
    want = oracle.adjoint(guess.astype(np.float64), cfg, step, g)
    plan = W.Plan(cfg)
    xt = torch.from_numpy(guess).cuda()
    gt = torch.from_numpy(g.astype(np.float32)).cuda()
    if saved:
        fs, fa = plan.forward(xt, step=step)
        got = plan.adjoint(xt, gt, step=step, fwd_slopes=fs, fwd_aux=fa)
    else:
        got = plan.adjoint(xt, gt, step=step)
    got = got.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    mx = np.abs(got - want).max() / np.abs(want).max()
    assert rel <= 1e-4 and mx <= 1e-3, f"rel-L2 {rel:.3g}, max {mx:.3g}"


def test_closed_loop_step_full_size_matches_oracle_restarted_from_gpu_state():
    torch, W = _gpu()
    cfg = synth.config4(batch=8)
    B = cfg["batch"]
    x = synth.make_batch(cfg, range(B))
    o, ldc = cfg["dm_offset"], cfg["layer_stride"]
    n_act = sum(L["nx"] * L["ny"] for L in cfg["layers"] if L["weight"] < 0)
    x[:, o:o + n_act] = synth.random_field((B, n_act), seed=23) * 0.3  # a DM shape in place
    plan = W.Plan(cfg)
    M = cfg["n_act_rows"]
    R = synth.make_reconstructor(M, plan.n_slopes)
    Rt = torch.from_numpy(R).cuda()
    xt = torch.from_numpy(x).cuda()
    dm = xt[:, o:]
    step = 321
    for k in range(3):  # a few steps in, so the DMs hold the loop's own shape
        s, _ = plan.forward(xt, step=step + k, seed=42)
        W.recon_apply(Rt, s, dm, alpha=cfg["gain"], beta=1.0, ldc=ldc)
    state = xt.cpu().numpy()
    k = step + 3
    s, _ = plan.forward(xt, step=k, seed=42)
    W.recon_apply(Rt, s, dm, alpha=cfg["gain"], beta=1.0, ldc=ldc)
    after = xt.cpu().numpy()
    s = s.cpu().numpy()
    rows = [0, 7]
    new, s_o = oracle.closed_loop_step(state[rows].astype(np.float64), cfg, R, k, seed=42,
                                       noise=True, realisations=rows)
    tol = slope_tolerance(cfg)
    err = _slope_errors(s[rows], s_o, tol)
    assert err.max() <= 1.0, f"slopes {err.max():.3g} of the bar"
    # DM update: |g R (s_gpu - s_o)| <= g sum_j |R_ij| tol_j, plus 1e-4 of g sum_j |R_ij s_j|
    Ra = np.abs(R[:n_act].astype(np.float64))
    g = abs(cfg["gain"])
    bound = g * (Ra @ tol)[None, :] + 1e-4 * g * (np.abs(s_o) @ Ra.T) + 1e-6
    d = np.abs(after[rows, o:o + n_act] - new[:, o:o + n_act])
    assert (d / bound).max() <= 1.0, f"DM update {(d / bound).max():.3g} of the bar"
    # the rest of each realisation's buffer is untouched (rows beyond the actuators land in
    # padding that no layer reads)
    assert np.array_equal(after[:, :o], state[:, :o])


def test_closed_loop_trajectory_ten_steps_matches_oracle():
    """Ten integrator steps a <- a - g R s (g = 0.4, noise on, the screen moving with the wind)
    with R the oracle's regularised least-squares matrix of the system's DM: the GPU and the
    oracle run their own trajectories from the same start.  Their DM states differ by e_k; the
    slopes then differ by D^T e_k (D the oracle's interaction matrix) plus at most the slope
    bar, and each DM update by g R times the slope difference plus the reconstructor bar."""
    torch, W = _gpu()
    cfg, a0, n_act = _system(turbulence=True, wind=(12.0, -7.0))
    for sen in cfg["sensors"]:
        sen["photons"] = 2000.0
        sen["read_noise_e"] = 2.0
    cfg = dict(cfg, batch=2)
    im = oracle.interaction_matrix(cfg, a0, n_act, 0.05, batch=8)
    R = oracle.regularised_lse(im, 0.05).astype(np.float32)
    R64 = R.astype(np.float64)
    rng = np.random.default_rng(17)
    x = np.zeros((2, cfg["layer_stride"]), np.float32)
    x[:, :a0] = (rng.standard_normal((2, a0)) * 0.15).astype(np.float32)
    loop = dict(cfg, dm_offset=a0, gain=-0.4)
    plan = W.Plan(cfg)
    xt = torch.from_numpy(x).cuda()
    Rt = torch.from_numpy(R).cuda()
    dm = xt[:, a0:a0 + n_act]
    xo = x.astype(np.float64)
    tol = slope_tolerance(cfg)
    norms = []
    for k in range(10):
        e = xt.cpu().numpy()[:, a0:a0 + n_act].astype(np.float64) - xo[:, a0:a0 + n_act]
        s, _ = plan.forward(xt, step=k, seed=9)
        W.recon_apply(Rt, s, dm, alpha=-0.4, beta=1.0, ldc=cfg["layer_stride"])
        xo_next, s_o = oracle.closed_loop_step(xo, loop, R64, k, seed=9, noise=True)
        s_g = s.cpu().numpy().astype(np.float64)
        lin = e @ im  # D^T e for each realisation
        slope_err = np.abs(s_g - s_o - lin) / (tol + 1e-2 * np.abs(lin))
        assert slope_err.max() <= 1.0, f"step {k}: slopes {slope_err.max():.3g} of the bar"
        e_next = (xt.cpu().numpy()[:, a0:a0 + n_act].astype(np.float64)
                  - xo_next[:, a0:a0 + n_act])
        upd = e_next - e + 0.4 * (s_g - s_o) @ R64.T
        bound = 0.4 * 1e-4 * (np.abs(s_o) @ np.abs(R64).T) + 1e-6 * (1 + np.abs(xo_next[:, a0:a0 + n_act]))
        assert (np.abs(upd) / bound).max() <= 1.0, f"step {k}: DM {(np.abs(upd) / bound).max():.3g}"
        assert np.abs(e_next).max() <= 1e-3
        norms.append(np.linalg.norm(s_o))
        xo = xo_next
    assert norms[-1] < norms[0]  # the loop closes


def test_dark_sensor_non_positive_pixel_sums_give_zero_slopes():
    """Photons 1e-3 per subaperture and 5 e- read noise: the pixel sum of a subaperture is
    mostly noise, and about half of them are <= 0.  Where the oracle's sum is clearly negative
    the GPU gives exactly (0, 0); where it is clearly positive the slopes agree within the slope
    bar plus the FP32 rounding of the sums, 4e-6 (sum |x B'| + |c| sum |B'|) / sum B'."""
    torch, W = _gpu()
    cfg = synth.small_lgs(n_sa=12, n_sub=10, n_fft=32, bin_=4, n_layers=2, n=256, pitch=0.25,
                          noise=True)
    sen = cfg["sensors"][0]
    sen["photons"] = 1e-3
    sen["read_noise_e"] = 5.0
    x = synth.make_batch(cfg, [0])
    plan = W.Plan(cfg)
    s, a = plan.forward(torch.from_numpy(x).cuda(), step=2, seed=42)
    s = s.cpu().numpy()[0].astype(np.float64)
    a = a.cpu().numpy()[0].astype(np.float64)
    tr = {}
    want, S = oracle.sensor_slopes(x[0].astype(np.float64), cfg, 0, 2, 42, 0, noise=True,
                                   trace=tr)
    Bp = tr["B"]
    nv = len(S)
    n_pix = Bp.shape[1]
    xq = np.arange(n_pix) - (n_pix - 1) / 2.0
    np.testing.assert_allclose(a, S, rtol=0, atol=1e-4 * np.abs(Bp).sum(axis=(1, 2)).max())
    neg = S < -1.0
    pos = S > 1.0
    assert neg.sum() >= nv // 5 and pos.sum() >= nv // 5
    assert np.all(s[:nv][neg] == 0.0) and np.all(s[nv:][neg] == 0.0)
    absx = np.abs(Bp * xq[None, None, :]).sum(axis=(1, 2))
    absy = np.abs(Bp * xq[None, :, None]).sum(axis=(1, 2))
    absb = np.abs(Bp).sum(axis=(1, 2))
    t0 = slope_tolerance(cfg)
    tx = t0[:nv] + 4e-6 * (absx + np.abs(want[:nv]) * absb) / np.abs(S)
    ty = t0[nv:] + 4e-6 * (absy + np.abs(want[nv:]) * absb) / np.abs(S)
    assert np.all(np.abs(s[:nv] - want[:nv])[pos] <= tx[pos])
    assert np.all(np.abs(s[nv:] - want[nv:])[pos] <= ty[pos])


def test_noisy_slopes_backward_uses_the_noise_free_adjoint():
    """wfs_slopes on a noisy LGS: the forward carries noise, the backward is the adjoint of the
    noise-free model (the oracle's adjoint at the same layers)."""
    torch, W = _gpu()
    cfg = synth.small_lgs(n_sa=12, n_sub=10, n_fft=32, bin_=4, n_layers=3, n=256, pitch=0.25,
                          noise=True)
    x = synth.make_batch(cfg, [0]) * 0.5
    plan = W.Plan(cfg)
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    s = W.wfs_slopes(xt, plan, step=6, seed=3)
    noisy_want, _ = oracle.forward(x.astype(np.float64), cfg, 6, 3, noise=True)
    err = _slope_errors(s.detach().cpu().numpy(), noisy_want, slope_tolerance(cfg))
    assert err.max() <= 1.0
    gs = synth.random_field(tuple(s.shape), seed=4)
    s.backward(torch.from_numpy(gs).cuda())
    want = oracle.adjoint(x.astype(np.float64), cfg, 6, gs.astype(np.float64))
    got = xt.grad.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert rel <= 1e-4 and np.abs(got - want).max() <= 1e-3 * np.abs(want).max()
