"""GPU parity of wfs_calibrate (push-pull interaction matrix, reference slopes) and wfs_tlse
(regularised least-squares control matrix) against the FP64 oracle, and closed-loop
convergence with the calibrated reconstructor.

Interaction-matrix bar: each GPU slope is within t = 1e-4 of the spot FWHM (binned pixels) of
the oracle's, so a push-pull column (s+ - s-) / (2a) is within t / a."""

import numpy as np
import pytest

import oracle
import synth
from test_oracle_calib import _system
from wfs_cases import dm_case, slope_tolerance

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    import paper_1608_00386_amd as W
    return torch, W


def _noisy(cfg):
    for s in cfg["sensors"]:
        s["photons"] = 800.0
        s["read_noise_e"] = 2.0
    return cfg


def _case(name):
    """(calibration config, first actuator, actuators, base or None, noise)."""
    from paper_1608_00386_amd import calib
    if name == "ngs_lgs_dm7":
        cfg, a0, n = _system()
        return dict(cfg, batch=8), a0, n, None, False
    if name == "ngs_lgs_dm7_noisy":
        cfg, a0, n = _system()
        return _noisy(dict(cfg, batch=8)), a0, n, None, True
    if name == "ngs_lgs_dm7_onsky":
        cfg, a0, n = _system(turbulence=True)
        base = np.random.default_rng(3).standard_normal(cfg["layer_stride"]) * 0.3
        base[a0:] = 0.0
        return dict(cfg, batch=6), a0, n, base.astype(np.float32), False
    if name == "ngs_lgs_dm7_onsky_wind_noisy":
        # a base screen moving with the wind and noisy sensors: every chunk sees the screen
        # at the calibration step and draws its own noise
        cfg, a0, n = _system(turbulence=True, wind=(35.0, -20.0))
        base = np.random.default_rng(3).standard_normal(cfg["layer_stride"]) * 0.3
        base[a0:] = 0.0
        return _noisy(dict(cfg, batch=6)), a0, n, base.astype(np.float32), True
    if name == "two_ngs_dm11":
        ccfg, n = calib.dm_config(dm_case(), batch=16)
        return ccfg, 0, n, None, False
    raise KeyError(name)


@pytest.mark.parametrize("name", ["ngs_lgs_dm7", "ngs_lgs_dm7_noisy", "ngs_lgs_dm7_onsky",
                                  "ngs_lgs_dm7_onsky_wind_noisy", "two_ngs_dm11"])
def test_calibrate_matches_oracle(name):
    torch, W = _gpu()
    cfg, a0, n, base, noise = _case(name)
    amp = 0.5
    plan = W.Plan(cfg)
    bt = torch.from_numpy(base).cuda() if base is not None else None
    im, ref = plan.calibrate(a0, n, amplitude=amp, step=3, seed=7, base=bt)
    got = im.cpu().numpy().astype(np.float64)
    b64 = base.astype(np.float64) if base is not None else None
    want = oracle.interaction_matrix(cfg, a0, n, amp, batch=cfg["batch"], step=3, seed=7,
                                     noise=noise, base=b64)
    tol = slope_tolerance(cfg) / amp
    err = np.abs(got - want) / tol[None, :]
    assert err.max() <= 1.0, f"IM error {err.max():.3g} of the bar"
    r_want = oracle.reference_slopes(cfg, step=3, seed=7, noise=noise, base=b64)
    r_err = np.abs(ref.cpu().numpy() - r_want) / slope_tolerance(cfg)
    assert r_err.max() <= 1.0


def test_calibrate_rows_of_unseen_actuators_are_exactly_zero():
    torch, W = _gpu()
    cfg, a0, n, _, _ = _case("ngs_lgs_dm7")
    im, _ = W.Plan(cfg).calibrate(a0, n, amplitude=0.5)
    iy, ix = np.divmod(np.arange(n), 7)
    ring = (ix == 0) | (ix == 6) | (iy == 0) | (iy == 6)
    ring |= np.isin(ix, (1, 5)) & np.isin(iy, (1, 5))
    got = im.cpu().numpy()
    assert np.all(got[ring] == 0.0)
    assert np.all(np.abs(got[~ring]).max(axis=1) > 1e-3)


def test_calibrate_is_deterministic_and_chunk_independent_without_noise():
    """The same rows, bit for bit, from a run twice and from plans of other batch sizes (the
    noise-free forward of a realisation does not depend on its neighbours or the step)."""
    torch, W = _gpu()
    cfg, a0, n, _, _ = _case("ngs_lgs_dm7")
    im1, _ = W.Plan(cfg).calibrate(a0, n, amplitude=0.5)
    im2, _ = W.Plan(cfg).calibrate(a0, n, amplitude=0.5)
    assert torch.equal(im1, im2)
    for B in (2, 14, 100):
        im3, _ = W.Plan(dict(cfg, batch=B)).calibrate(a0, n, amplitude=0.5)
        assert torch.equal(im1, im3), B


def test_calibrate_writes_rows_with_a_leading_dimension():
    torch, W = _gpu()
    cfg, a0, n, _, _ = _case("two_ngs_dm11")
    plan = W.Plan(cfg)
    im, _ = plan.calibrate(a0, n, amplitude=0.5)
    big = torch.full((n, plan.n_slopes + 13), 7.0, device="cuda")
    im2, _ = plan.calibrate(a0, n, amplitude=0.5, im=big)
    assert torch.equal(big[:, :plan.n_slopes], im)
    assert torch.all(big[:, plan.n_slopes:] == 7.0)


def test_calibrate_full_closed_loop_system_sampled_actuators():
    """The 5,389 actuators of the three DMs (0, 4 and 12.7 km) seen by six LGS and three NGS:
    the whole matrix on the GPU, two sampled rows against the oracle."""
    torch, W = _gpu()
    from paper_1608_00386_amd import calib
    cfg, n = calib.dm_config(synth.config4(batch=1), batch=128)
    assert n == 5389
    amp = 0.5
    plan = W.Plan(cfg)
    im, ref = plan.calibrate(0, n, amplitude=amp)
    assert torch.isfinite(im).all()
    assert float(ref.abs().max()) < 1e-3  # flat: spots centred
    tol = slope_tolerance(cfg) / amp
    # actuators 12 m (0 km), 9 m (4 km) and 8.5 m (12.7 km) off axis: outside the central
    # obstruction's shadow
    for j in (20 * 40 + 8, 1600 + 21 * 42 + 30, 1600 + 1764 + 22 * 45 + 30):
        want = oracle.interaction_matrix(cfg, j, 1, amp, batch=128)[0]
        got = im[j].cpu().numpy().astype(np.float64)
        err = np.abs(got - want) / tol
        assert err.max() <= 1.0, (j, err.max())
        assert np.abs(want).max() > 1e-2


def _im_small():
    cfg, a0, n = _system()
    im = oracle.interaction_matrix(cfg, a0, n, 0.05, batch=8)
    return im


@pytest.mark.parametrize("eps,weighted", [(0.05, False), (0.05, True), (0.5, True)])
def test_tlse_matches_oracle(eps, weighted):
    """Relative error bound: FP32 Cholesky and triangular solves, condition number of the
    regularised normal matrix at most about 1 / eps times the spread of its diagonal."""
    torch, W = _gpu()
    im = _im_small().astype(np.float32)
    m = im.shape[0]
    w = np.where(np.arange(m) % 7 < 3, 1.0, 3.0).astype(np.float32) if weighted else None
    imt = torch.from_numpy(im).cuda()
    wt = torch.from_numpy(w).cuda() if weighted else None
    R = W.tlse(imt, eps=eps, weights=wt)
    want = oracle.regularised_lse(im.astype(np.float64), eps, w)
    got = R.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - want) <= 1e-4 * np.linalg.norm(want)
    # in place: the same bits
    imc = imt.clone()
    R2 = W.tlse(imc, eps=eps, weights=wt, out=imc)
    assert torch.equal(R2, R)


def test_tlse_full_rank_without_regularisation_is_the_pseudo_inverse():
    torch, W = _gpu()
    rng = np.random.default_rng(9)
    im = rng.standard_normal((300, 2000)).astype(np.float32)
    R = W.tlse(torch.from_numpy(im).cuda(), eps=0.0)
    want = np.linalg.pinv(im.astype(np.float64).T)
    got = R.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - want) <= 1e-4 * np.linalg.norm(want)


def test_tlse_rejects_a_singular_normal_matrix():
    torch, W = _gpu()
    im = torch.from_numpy(_im_small().astype(np.float32)).cuda()  # unseen actuators: zero rows
    with pytest.raises(W.WfsError, match="positive definite"):
        W.tlse(im, eps=0.0)


def test_closed_loop_with_calibrated_reconstructor_converges_on_gpu():
    """Static turbulence, integrator a <- a - g R s with R from the GPU calibration: the slopes
    fall to the part the DMs cannot fit, as in the oracle's loop."""
    torch, W = _gpu()
    from paper_1608_00386_amd import calib
    cfg, a0, n = _system(turbulence=True)
    ccfg, n2 = calib.dm_config(cfg, batch=8)
    assert n2 == n
    im, _ = W.Plan(ccfg).calibrate(0, n, amplitude=0.05)
    R = W.tlse(im, eps=0.05)
    rng = np.random.default_rng(6)
    x = np.zeros((1, cfg["layer_stride"]))
    x[0, :a0] = rng.standard_normal(a0) * 0.15
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    plan = W.Plan(cfg)
    s0, _ = plan.forward(xt)
    s0 = s0.clone()
    dm = xt[:, a0:a0 + n]
    for _ in range(25):
        s, _ = plan.forward(xt)
        W.recon_apply(R, s, dm, alpha=-0.5, beta=1.0, ldc=cfg["layer_stride"])
    s_end, _ = plan.forward(xt)
    n0 = float(s0.norm())
    ne = float(s_end.norm())
    im64 = im.cpu().double().numpy()
    R64 = oracle.regularised_lse(im64, 0.05)
    fit = np.linalg.norm(s0.cpu().double().numpy()[0] - im64.T @ (R64 @ s0.cpu().double().numpy()[0]))
    assert ne < 0.5 * n0
    assert abs(ne - fit) <= 0.05 * n0
