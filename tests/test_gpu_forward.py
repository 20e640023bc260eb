"""GPU parity of wfs_forward / wfs_project against the FP64 oracle (same float32 inputs)."""

import numpy as np
import pytest

import oracle
import synth
from wfs_cases import CASES, layers_for, slope_tolerance

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    import paper_1608_00386_amd as W
    return torch, W


def _flags(W, mode):
    """Plan flags of a field mode: projection kernel first, per-pixel gather in the spot
    waves, or the default (staged footprint where every lag-domain sensor allows it)."""
    return {"split": W.WFS_FLAG_SPLIT, "fused": W.WFS_FLAG_FUSED,
            "footprint": W.WFS_FLAG_FOOTPRINT, "default": 0}[mode]


def _run(cfg, x, step, seed=42, flags=0):
    torch, W = _gpu()
    plan = W.Plan(cfg, flags=flags, batch=x.shape[0])
    xt = torch.from_numpy(x).cuda()
    s, a = plan.forward(xt, step=step, seed=seed)
    torch.cuda.synchronize()
    return s.cpu().numpy().astype(np.float64), a.cpu().numpy().astype(np.float64), plan, xt


def _check(cfg, x, s_gpu, a_gpu, step, seed=42):
    s_ref, a_ref = oracle.forward(x.astype(np.float64), cfg, step, seed, noise=True)
    tol = slope_tolerance(cfg)
    err = np.abs(s_gpu - s_ref)
    worst = float((err / tol[None, :]).max())
    assert worst <= 1.0, f"slope error {worst:.3g} x tolerance (max abs {err.max():.3g})"
    np.testing.assert_allclose(a_gpu, a_ref, rtol=2e-5, atol=1e-4 * np.abs(a_ref).max())
    return worst


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("step", [0, 7])
@pytest.mark.parametrize("mode", ["split", "fused", "footprint"])
def test_forward_matches_oracle(name, step, mode):
    torch, W = _gpu()
    cfg = CASES[name]()
    x = layers_for(cfg)
    s, a, plan, _ = _run(cfg, x, step, flags=_flags(W, mode))
    want = {"split": "split", "fused": "gather", "footprint": "footprint"}[mode]
    if mode == "footprint" and 1 in plan.paths:
        want = "split"  # FFT-path sensors read the projected phase
    assert plan.schedule()["field"] == want
    assert s.shape == (cfg["batch"], oracle.n_slopes(cfg))
    _check(cfg, x, s, a, step)


@pytest.mark.parametrize("name", ["cfg0", "fft_ngs_n14_N32_b4", "ngs_n2_N4_b2"])
def test_forward_forced_fft_path(name):
    """The FFT path on sensors the lag-domain path also serves (no elongation)."""
    torch, W = _gpu()
    cfg = CASES[name]()
    x = layers_for(cfg)
    try:
        s, a, plan, _ = _run(cfg, x, 3, flags=W.WFS_FLAG_FORCE_FFT)
    except W.WfsError as e:
        assert e.code == -4 and name == "ngs_n2_N4_b2"  # N = 4 has no FFT kernel
        return
    assert all(p == 1 for p in plan.paths)
    _check(cfg, x, s, a, 3)


def test_paths_chosen_by_the_plan():
    torch, W = _gpu()
    plan = W.Plan(CASES["mixed_lgs_ngs_batch2"]())
    assert plan.paths == [0, 1]
    plan2 = W.Plan(synth.config2(batch=1))
    assert plan2.paths == [0] * 6 + [1] * 3
    assert plan2.n_slopes == 55608


def test_forward_is_bitwise_deterministic():
    cfg = CASES["lgs_n10_N32_b4_noise"]()
    x = layers_for(cfg)
    torch, W = _gpu()
    plan = W.Plan(cfg)
    xt = torch.from_numpy(x).cuda()
    s1, a1 = plan.forward(xt, step=3, seed=9)
    s1, a1 = s1.clone(), a1.clone()
    s2, a2 = plan.forward(xt, step=3, seed=9)
    assert torch.equal(s1, s2) and torch.equal(a1, a2)
    s3, _ = plan.forward(xt, step=3, seed=10)
    assert not torch.equal(s1, s3)  # the seed reaches the noise


def test_flat_screens_give_zero_slopes_on_gpu():
    for name in ("cfg0", "lgs_n10_N32_b4_noise", "ngs_n6_N12_b4_oddpix"):
        cfg = CASES[name]()
        for s in cfg["sensors"]:
            s["photons"] = 0.0
        x = np.zeros((cfg["batch"], cfg["layer_stride"]), np.float32)
        s, a, _, _ = _run(cfg, x, 0)
        assert np.abs(s).max() < 2e-6, name


def test_tuned_schedule_matches_oracle():
    """Whatever schedule the autotuner keeps (split/fused, tasks per wave, block order)
    computes the same slopes."""
    torch, W = _gpu()
    cfg = CASES["lgs_n10_N32_b4_noise"]()
    x = layers_for(cfg)
    plan = W.Plan(cfg)
    xt = torch.from_numpy(x).cuda()
    plan.tune(xt, iters=3)
    s, a = plan.forward(xt, step=5)
    _check(cfg, x, s.cpu().numpy().astype(np.float64), a.cpu().numpy().astype(np.float64), 5)


def test_device_step_counter_matches_host_step():
    torch, W = _gpu()
    cfg = CASES["lgs_n4_N8_b2"]()
    x = layers_for(cfg)
    plan = W.Plan(cfg)
    xt = torch.from_numpy(x).cuda()
    ref, _ = plan.forward(xt, step=5, seed=3)
    ref = ref.clone()
    plan.set_step(3)
    plan.advance_step(2)
    got, _ = plan.forward(xt, step=W.WFS_STEP_DEVICE, seed=3)
    assert torch.equal(ref, got)


def test_project_matches_oracle():
    torch, W = _gpu()
    cfg = CASES["dm_two_ngs_batch2"]()
    x = layers_for(cfg)
    plan = W.Plan(cfg)
    xt = torch.from_numpy(x).cuda()
    ph = plan.project(xt, step=11).cpu().numpy().astype(np.float64)
    o = 0
    for si, sensor in enumerate(cfg["sensors"]):
        geo = oracle.pupil_geometry(sensor)
        n = sensor["n_sub"]
        for bi in range(cfg["batch"]):
            psi = oracle.project(x[bi].astype(np.float64), cfg, sensor, 11)
            ref = np.stack([psi[a * n:(a + 1) * n, b * n:(b + 1) * n].ravel()
                            for a, b in geo["valid"]]).ravel()
            got = ph[bi, o:o + ref.size]
            np.testing.assert_allclose(got, ref, atol=2e-5 * max(1.0, np.abs(ref).max()))
        o += len(geo["valid"]) * n * n


@pytest.mark.parametrize("name", ["lgs_n10_N32_b4_noise", "mixed_lgs_ngs_batch2", "cfg0"])
def test_spots_of_projection_is_the_forward(name):
    """wfs_spots(wfs_project(x)) is the split forward, bit for bit (noise included)."""
    torch, W = _gpu()
    cfg = CASES[name]()
    x = layers_for(cfg)
    plan = W.Plan(cfg)
    xt = torch.from_numpy(x).cuda()
    s1, a1 = plan.forward(xt, step=5, seed=3)
    s2, a2 = plan.spots(plan.project(xt, step=5), step=5, seed=3)
    assert torch.equal(s1, s2) and torch.equal(a1, a2)


@pytest.mark.parametrize("name", sorted(CASES))
def test_footprint_field_equals_split_bitwise(name):
    """The staged-footprint field repeats the projection kernel's indices, weights and
    operation order, so its slopes equal the split schedule's bit for bit (periodic wrap,
    zero-boundary DM grid and a step far from the origin included)."""
    torch, W = _gpu()
    cfg = CASES[name]()
    x = layers_for(cfg)
    xt = torch.from_numpy(x).cuda()
    pf = W.Plan(cfg, flags=W.WFS_FLAG_FOOTPRINT, batch=x.shape[0])
    if pf.schedule()["field"] != "footprint":
        assert 1 in pf.paths
        pytest.skip("FFT-path sensors read the projected phase")
    ps = W.Plan(cfg, flags=W.WFS_FLAG_SPLIT, batch=x.shape[0])
    assert ps.schedule()["field"] == "split"
    for step in (0, 7, 100003):
        s1, a1 = pf.forward(xt, step=step, seed=9)
        s2, a2 = ps.forward(xt, step=step, seed=9)
        assert torch.equal(s1, s2) and torch.equal(a1, a2), step


@pytest.mark.parametrize("name", ["lgs_n10_N32_b4_noise", "mixed_lgs_ngs_batch2",
                                  "dm_two_ngs_batch2", "fft_ngs_n64_N128_b4"])
@pytest.mark.parametrize("mode", ["split", "fused", "footprint", "default"])
def test_forward_steps_equals_single_frames(name, mode):
    """Frames in a row (pipelined split launches, or one staged-footprint launch) give the
    single-frame results bit for bit, also from the device step counter; by default the single
    frames run split and the frames in a row as one footprint launch."""
    torch, W = _gpu()
    cfg = CASES[name]()
    x = layers_for(cfg)
    plan = W.Plan(cfg, flags=_flags(W, mode))
    xt = torch.from_numpy(x).cuda()
    n, k0 = 5, 3
    s, a = plan.forward_steps(xt, k0, n, seed=7)
    for k in range(n):
        s1, a1 = plan.forward(xt, step=k0 + k, seed=7)
        assert torch.equal(s[k], s1) and torch.equal(a[k], a1), k
    plan.set_step(k0)
    sd, ad = plan.forward_steps(xt, W.WFS_STEP_DEVICE, n, seed=7)
    assert torch.equal(sd, s) and torch.equal(ad, a)
    s_ref, _ = oracle.forward(x.astype(np.float64), cfg, k0 + n - 1, 7, noise=True)
    err = np.abs(s[n - 1].cpu().numpy().astype(np.float64) - s_ref)
    assert (err / slope_tolerance(cfg)[None, :]).max() <= 1.0


def test_forward_steps_config1_equals_single_frames():
    """Config 1, 6 frames in one staged-footprint launch: every frame's slopes equal the
    split schedule's single-frame call."""
    torch, W = _gpu()
    cfg = synth.config1()
    x = synth.make_batch(cfg, [0])
    plan = W.Plan(cfg)
    assert plan.schedule()["frames"] == "one_launch"
    split = W.Plan(cfg, flags=W.WFS_FLAG_SPLIT)
    xt = torch.from_numpy(x).cuda()
    s, _ = plan.forward_steps(xt, 40, 6)
    for k in (0, 5):
        s1, _ = split.forward(xt, step=40 + k)
        assert torch.equal(s[k], s1)


def test_forward_steps_after_tune_config2_equals_single_frames():
    """Config 2 (6 LGS + 3 NGS, 8 realisations) after the tuner has chosen between pipelined
    and one-frame-after-the-other steps: each frame equals the single-frame call."""
    torch, W = _gpu()
    cfg = synth.config2(batch=8)
    x = synth.make_batch(cfg, range(8))
    plan = W.Plan(cfg, batch=8)
    xt = torch.from_numpy(x).cuda()
    plan.tune(xt, iters=2)
    sch = plan.schedule()
    assert sch["field"] != "footprint"  # single frames: FFT-path NGS read the projected phase
    assert sch["field"] == "split" or sch["frames"] == "sequential"
    s, a = plan.forward_steps(xt, 11, 3)
    for k in range(3):
        s1, a1 = plan.forward(xt, step=11 + k)
        assert torch.equal(s[k], s1) and torch.equal(a[k], a1), (k, sch)


def test_footprint_matches_oracle_coordinates():
    """Distinct layer pixels under the bilinear stencils of the valid subapertures' pixels."""
    torch, W = _gpu()
    cfg = CASES["dm_two_ngs_batch2"]()
    plan = W.Plan(cfg)
    step = 9
    want = 0
    for L in cfg["layers"]:
        hit = np.zeros((L["ny"], L["nx"]), bool)
        for sensor in cfg["sensors"]:
            geo = oracle.pupil_geometry(sensor)
            n = sensor["n_sub"]
            u, v = oracle.wfs_oracle._layer_coords(L, sensor, geo, step, cfg["dt_s"])
            iu0, iu1, _, _, ou0, ou1 = oracle.wfs_oracle._bilinear_taps(u, L["nx"], L["boundary"])
            iv0, iv1, _, _, ov0, ov1 = oracle.wfs_oracle._bilinear_taps(v, L["ny"], L["boundary"])
            for a, b in geo["valid"]:
                rs, cs = slice(a * n, (a + 1) * n), slice(b * n, (b + 1) * n)
                for iv, ov in ((iv0, ov0), (iv1, ov1)):
                    for iu, ou in ((iu0, ou0), (iu1, ou1)):
                        m = ov[rs][:, None] & ou[cs][None, :]
                        hit[np.broadcast_to(iv[rs][:, None], m.shape)[m],
                            np.broadcast_to(iu[cs][None, :], m.shape)[m]] = True
        want += int(hit.sum())
    got, n_phase = plan.footprint(step)
    assert n_phase == plan.phase_numel
    assert abs(got - want) <= 0.002 * want, (got, want)


@pytest.mark.parametrize("step,mode", [(0, "split"), (61, "split"), (61, "fused"),
                                       (61, "footprint")])
def test_config1_full_frame_matches_oracle(step, mode):
    """E-ELT 80x80 LGS (config 1), every one of the 4,632 subapertures, noise on."""
    torch, W = _gpu()
    cfg = synth.config1()
    x = synth.make_batch(cfg, [0])
    s, a, plan, _ = _run(cfg, x, step, flags=_flags(W, mode))
    assert plan.n_slopes == 9264
    worst = _check(cfg, x, s, a, step)
    print(f"config1 step {step}: worst slope error {worst:.3g} of tolerance")


def test_config0_paper_sampling_counts():
    torch, W = _gpu()
    plan = W.Plan(synth.config0())
    assert plan.n_valid == [52] and plan.n_slopes == 104
    plan1 = W.Plan(synth.config1())
    assert plan1.n_valid == [4632]
    np.testing.assert_allclose(plan1.pix_scale[0], oracle.pixel_scale(synth.config1()["sensors"][0]))


@pytest.mark.parametrize("name", ["mixed_lgs_ngs_batch2", "config2_batch2", "cfg1",
                                  "lgs_n4_N8_b2_20layers", "ngs_n12_N24_b3"])
def test_lag_passes_give_the_same_bits(name):
    """The split field's spot waves form each lag row in 2 or 3 passes (wfs_plan_set_schedule's
    lag_passes): the same multiply-adds in the same order, so single frames, pipelined and
    overlapped frames give the same bits either way; other values are refused."""
    torch, W = _gpu()
    if name == "config2_batch2":
        cfg, B = synth.config2(batch=2), 2
        x = synth.make_batch(cfg, range(B))
    elif name == "cfg1":
        cfg, B = synth.config1(), 1
        x = synth.make_batch(cfg, [0])
    else:
        cfg = CASES[name]()
        x = layers_for(cfg)
        B = x.shape[0]
    xt = torch.from_numpy(x).cuda()
    plan = W.Plan(cfg, batch=B)
    plan.set_schedule(field="split", frames="sequential", lag_passes=2)
    ref, aref = plan.forward(xt, step=4, seed=6)
    ref, aref = ref.clone(), aref.clone()
    steps2, _ = plan.forward_steps(xt, 4, 3, seed=6)
    for frames in ("sequential", "pipelined", "overlapped"):
        plan.set_schedule(field="split", frames=frames, lag_passes=3)
        assert plan.schedule()["lag_passes"] == 3
        s, a = plan.forward(xt, step=4, seed=6)
        assert torch.equal(s, ref) and torch.equal(a, aref), frames
        s3, _ = plan.forward_steps(xt, 4, 3, seed=6)
        assert torch.equal(s3, steps2), frames
    for bad in (1, 4):
        with pytest.raises(W.WfsError) as e:
            plan.set_schedule(lag_passes=bad)
        assert e.value.code == -1


@pytest.mark.parametrize("name", ["mixed_lgs_ngs_batch2", "config2_batch2"])
def test_overlapped_frames_match_single_frames_and_replay(name):
    """Overlapped frames (frame k + 1 projected on the plan's projection stream while frame
    k's spots run): every frame equals the single-frame call bit for bit, eagerly and in a
    captured graph replayed several times with eager work in between."""
    torch, W = _gpu()
    if name == "config2_batch2":
        cfg, B = synth.config2(batch=2), 2
        x = synth.make_batch(cfg, range(B))
    else:
        cfg = CASES[name]()
        x = layers_for(cfg)
        B = x.shape[0]
    plan = W.Plan(cfg, batch=B)
    xt = torch.from_numpy(x).cuda()
    n, k0 = 5, 7
    plan.set_schedule(field="split", frames="overlapped")
    assert plan.schedule()["frames"] == "overlapped"
    ref = torch.stack([plan.forward(xt, step=k0 + k, seed=2)[0].clone() for k in range(n)])
    s, _ = plan.forward_steps(xt, k0, n, seed=2)
    assert torch.equal(s, ref)
    out = torch.empty_like(ref)
    aux = torch.empty(n, B, plan.n_valid_total, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.forward_steps(xt, k0, n, seed=2, slopes=out, aux=aux)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.forward_steps(xt, k0, n, seed=2, slopes=out, aux=aux)
    for rep in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep
        plan.forward_steps(xt, 1, 2, seed=9)  # eager work between the replays
        torch.cuda.synchronize()


def test_side_stream_graph_replays_match_eager():
    """A plan with FFT-path and lag-domain sensors runs the FFT-path blocks on a side stream
    (fork and join events); a captured graph of single frames and of frames in a row replays
    to the eager results every time, with eager work in between."""
    torch, W = _gpu()
    cfg = CASES["mixed_lgs_ngs_batch2"]()
    x = layers_for(cfg)
    plan = W.Plan(cfg, batch=x.shape[0])
    assert 1 in plan.paths and 0 in plan.paths
    xt = torch.from_numpy(x).cuda()
    n = 3
    ref = torch.stack([plan.forward(xt, step=4 + k, seed=5)[0].clone() for k in range(n)])
    ref_steps, _ = plan.forward_steps(xt, 4, n, seed=5)
    assert torch.equal(ref_steps, ref)
    out = torch.empty_like(ref)
    aux = torch.empty(n, x.shape[0], plan.n_valid_total, device="cuda")
    out2 = torch.empty_like(ref)
    aux2 = torch.empty_like(aux)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.forward(xt, step=0, seed=5, slopes=out[0], aux=aux[0])
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for k in range(n):
            plan.forward(xt, step=4 + k, seed=5, slopes=out[k], aux=aux[k])
        plan.forward_steps(xt, 4, n, seed=5, slopes=out2, aux=aux2)
    for rep in range(3):
        out.zero_()
        out2.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref) and torch.equal(out2, ref), rep
        plan.forward(xt, step=11, seed=1)  # eager work between the replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("flags", ["footprint", "default"])
def test_mixed_plan_frames_in_one_footprint_launch_equal_single_frames(flags):
    """Config 2 with WFS_FLAG_FOOTPRINT: the lag-domain LGS frames run as one staged-footprint
    launch while the FFT-path NGS run frame by frame on the side stream; every frame equals
    the single-frame call bit for bit.  Without the flag such a plan keeps split frames."""
    torch, W = _gpu()
    cfg = synth.config2(batch=2)
    x = synth.make_batch(cfg, range(2))
    plan = W.Plan(cfg, batch=2, flags=W.WFS_FLAG_FOOTPRINT if flags == "footprint" else 0)
    sch = plan.schedule()
    assert sch["field"] == "split"
    assert sch["frames"] == ("one_launch" if flags == "footprint" else "pipelined")
    xt = torch.from_numpy(x).cuda()
    s, a = plan.forward_steps(xt, 5, 4)
    for k in range(4):
        s1, a1 = plan.forward(xt, step=5 + k)
        assert torch.equal(s[k], s1) and torch.equal(a[k], a1), k


@pytest.mark.parametrize("name", ["mixed_lgs_ngs_batch2", "config2_batch2"])
def test_pinned_schedules_give_the_same_bits(name):
    """wfs_plan_set_schedule: the FFT-path blocks on the side stream or in the same launch as
    the lag-domain blocks (and, pipelined, the next step's projection: one launch per step),
    frames one after the other or pipelined, either block order: the slopes are bit for bit
    those of the split single frame; impossible schedules are refused."""
    torch, W = _gpu()
    if name == "config2_batch2":
        cfg, B = synth.config2(batch=2), 2
        x = synth.make_batch(cfg, range(B))
    else:
        cfg = CASES[name]()
        x = layers_for(cfg)
        B = x.shape[0]
    xt = torch.from_numpy(x).cuda()
    plan = W.Plan(cfg, batch=B)
    plan.set_schedule(field="split", frames="sequential", xcd_remap=1, fft_launch="side_stream")
    n, k0 = 3, 6
    ref = [plan.forward(xt, step=k0 + k, seed=4) for k in range(n)]
    ref = [(s.clone(), a.clone()) for s, a in ref]
    for fft_launch in ("side_stream", "same_launch"):
        for frames in ("sequential", "pipelined", "overlapped"):
            for remap in (0, 1):
                plan.set_schedule(field="split", frames=frames, xcd_remap=remap,
                                  fft_launch=fft_launch)
                sch = plan.schedule()
                assert (sch["frames"], sch["fft_launch"]) == (frames, fft_launch)
                s, a = plan.forward_steps(xt, k0, n, seed=4)
                for k in range(n):
                    assert torch.equal(s[k], ref[k][0]) and torch.equal(a[k], ref[k][1]), \
                        (fft_launch, frames, remap, k)
                s1, a1 = plan.forward(xt, step=k0, seed=4)
                assert torch.equal(s1, ref[0][0]) and torch.equal(a1, ref[0][1])
    with pytest.raises(W.WfsError) as e:
        plan.set_schedule(field="footprint")  # FFT-path sensors read the projected phase
    assert e.value.code == -4
    with pytest.raises(W.WfsError) as e:
        plan.set_schedule(field="gather", frames="pipelined")
    assert e.value.code == -4


@pytest.mark.parametrize("name", ["mixed_lgs_ngs_batch2", "config2_batch2", "cfg1"])
def test_projection_tile_heights_give_the_same_bits(name):
    """The projection kernel's tile height (wfs_plan_set_schedule's proj_rows: 8, 16 or 32
    pupil rows per block) moves pixels between blocks, not their arithmetic: the projected
    phase and the slopes (single split frames, pipelined frames) are bit for bit the same at
    every height the plan offers; a height it does not offer is refused."""
    torch, W = _gpu()
    if name == "config2_batch2":
        cfg, B = synth.config2(batch=2), 2
        x = synth.make_batch(cfg, range(B))
    elif name == "cfg1":
        cfg, B = synth.config1(), 1
        x = synth.make_batch(cfg, [0])
    else:
        cfg = CASES[name]()
        x = layers_for(cfg)
        B = x.shape[0]
    xt = torch.from_numpy(x).cuda()
    plan = W.Plan(cfg, batch=B)
    offered = []
    for rows in (8, 16, 32):
        try:
            plan.set_schedule(field="split", frames="sequential", proj_rows=rows)
        except W.WfsError as e:
            assert e.code == -4
            continue
        assert plan.schedule()["proj_rows"] == rows
        offered.append((rows, plan.project(xt, step=5).clone(),
                        plan.forward(xt, step=5, seed=3)[0].clone()))
        plan.set_schedule(frames="pipelined")
        offered[-1] += (plan.forward_steps(xt, 5, 3, seed=3)[0].clone(),)
    assert offered and offered[0][0] == 8
    for rows, ph, s1, s3 in offered[1:]:
        assert torch.equal(ph, offered[0][1]), rows
        assert torch.equal(s1, offered[0][2]), rows
        assert torch.equal(s3, offered[0][3]), rows
    assert torch.equal(offered[0][3][0], offered[0][2])
    for bad in (12, 64):
        with pytest.raises(W.WfsError) as e:
            plan.set_schedule(proj_rows=bad)
        assert e.value.code == -4
