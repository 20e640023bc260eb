"""GPU parity, against the FP64 oracle, of a plan whose lag-domain sensors have different
subaperture sizes (one spot launch per size; Sec. 2.7 sensors of a multi-sensor system, each
with its own grid): forward slopes in every field schedule, frames in a row, the tuned
schedule and the adjoint, with and without an FFT-path sensor in the same plan."""

import numpy as np
import pytest

import oracle
import synth
from wfs_cases import CASES, layers_for, slope_tolerance

pytestmark = pytest.mark.gpu

NAMES = ["uneven_lgs_ngs", "uneven_lgs_ngs_fft"]


def _gpu():
    import torch
    import paper_1608_00386_amd as W
    return torch, W


def _flags(W, mode):
    return {"default": 0, "split": W.WFS_FLAG_SPLIT, "fused": W.WFS_FLAG_FUSED,
            "footprint": W.WFS_FLAG_FOOTPRINT}[mode]


def _check(cfg, x, s_gpu, a_gpu, step, seed=42):
    s_ref, a_ref = oracle.forward(x.astype(np.float64), cfg, step, seed, noise=True)
    tol = slope_tolerance(cfg)
    err = np.abs(s_gpu - s_ref)
    worst = float((err / tol[None, :]).max())
    assert worst <= 1.0, f"slope error {worst:.3g} x tolerance (max abs {err.max():.3g})"
    np.testing.assert_allclose(a_gpu, a_ref, rtol=2e-5, atol=1e-4 * np.abs(a_ref).max())


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("mode", ["default", "split", "fused", "footprint"])
@pytest.mark.parametrize("step", [0, 3])
def test_uneven_forward_matches_oracle(name, mode, step):
    torch, W = _gpu()
    cfg = CASES[name]()
    x = layers_for(cfg)
    plan = W.Plan(cfg, flags=_flags(W, mode), batch=cfg["batch"])
    s, a = plan.forward(torch.from_numpy(x).cuda(), step=step, seed=42)
    torch.cuda.synchronize()
    _check(cfg, x, s.cpu().numpy().astype(np.float64), a.cpu().numpy().astype(np.float64), step)


@pytest.mark.parametrize("name", NAMES)
def test_uneven_frames_in_a_row_equal_single_frames(name):
    """wfs_forward_steps in every frame schedule the plan offers: bit for bit the frames of
    one wfs_forward each."""
    torch, W = _gpu()
    cfg = CASES[name]()
    x = torch.from_numpy(layers_for(cfg)).cuda()
    for flags in (0, W.WFS_FLAG_SPLIT, W.WFS_FLAG_FOOTPRINT):
        plan = W.Plan(cfg, flags=flags)
        for frames in plan.FRAMES:
            try:
                plan.set_schedule(frames=frames)
            except W.WfsError:
                continue  # a schedule this plan cannot take
            many, _ = plan.forward_steps(x, 2, 4)
            for k in range(4):
                one, _ = plan.forward(x, step=2 + k)
                assert torch.equal(many[k], one), (flags, frames, k)


@pytest.mark.parametrize("name", NAMES)
def test_uneven_tuned_plan_matches_oracle(name):
    torch, W = _gpu()
    cfg = CASES[name]()
    x = layers_for(cfg)
    xt = torch.from_numpy(x).cuda()
    plan = W.Plan(cfg)
    plan.tune(xt, iters=2)
    s, a = plan.forward(xt, step=5, seed=42)
    _check(cfg, x, s.cpu().numpy().astype(np.float64), a.cpu().numpy().astype(np.float64), 5)


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("mode", ["split", "fused"])
def test_uneven_adjoint_matches_oracle(name, mode):
    torch, W = _gpu()
    cfg = CASES[name]()
    for s in cfg["sensors"]:
        s["photons"] = 0.0
        s["read_noise_e"] = 0.0
    x = layers_for(cfg, scale=0.5)
    g = synth.random_field((cfg["batch"], oracle.n_slopes(cfg)), seed=9)
    plan = W.Plan(cfg, flags=_flags(W, mode))
    xt, gt = torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda()
    for step in (0, 4):
        got = plan.adjoint(xt, gt, step=step).cpu().numpy().astype(np.float64)
        ref = oracle.adjoint(x.astype(np.float64), cfg, step, g.astype(np.float64))
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert rel <= 1e-4, (step, rel)
        assert np.abs(got - ref).max() <= 1e-3 * np.abs(ref).max()
