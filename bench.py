#!/usr/bin/env python3
"""Benchmark of the Shack-Hartmann wavefront-sensor path on one MI355X.

Headline (`value`): E-ELT 80x80 LGS frames per second (config 1: 39 m pupil, 4,632 valid
10x10-pixel subapertures, 32-point FFT-equivalent spots, 8x8 binned pixels, 10 frozen-flow
layers of 1024^2, cone compression, 10 km sodium elongation, photon + read noise), one
frame = the whole sensor at one time step, inputs resident in HBM; the K timed frames are one
wfs_forward_steps call (the projection of step k+1 runs inside the spot launch of step k),
captured in a HIP graph and replayed.  The one-wfs_forward-per-frame rate is reported too.

Also reported (same JSON line): the batched multi-sensor step (config 2), the adjoint
(config 3) and the reconstructor (config 4 shape), each against the plain forward, the
roofline fraction of the dominant kernel and the FP64 oracle's rate on the host CPU.

    python bench.py [--gpus 1] [--steps 200] [--warmup 20] [--quick]
"""

import argparse
import copy
import glob
import json
import math
import os
import sys
import time

# the oracle baseline is timed on one core; keep BLAS/FFT helpers single-threaded
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import numpy as np  # noqa: E402

import synth  # noqa: E402

METRIC = ("WFS frames/s (subaperture spots/s) at 80×80 LGS; batched+adjoint vs plain "
          "forward")
PEAK_FP32_VALU = 157.3e12  # MI355X published FP32 vector peak
PEAK_HBM = 8.0e12
PEAK_FP32_MFMA = 157.3e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------------------------------------
# algorithmic work (what the method must compute; FFT counted as 5 N log2 N per transform)
# ------------------------------------------------------------------------------------------

def flops_per_subap(n_sub, N, b, elong):
    lg = np.log2(N)
    n_pix = N // b
    f = 4 * n_sub ** 2                                  # field: scale, ramp, sin, cos
    f += 5 * N * lg * (n_sub + N)                       # zero-padded 2-D FFT, pruned rows
    f += 3 * N * N + N * N                              # |F|^2 and normalisation
    if elong:
        f += 2 * 2.5 * N * N * np.log2(N * N) + 10 * N * (N // 2 + 1)  # R2C, x K, C2R
    f += N * N                                          # binning
    f += 4 * n_pix ** 2 + 4                             # centre of gravity
    return float(f)


def proj_flops(cfg, plan, batch=1):
    """Algorithmic FLOP of the projection (Sec. 2.2) of one frame: per valid pixel and layer a
    bilinear stencil (two row blends of 3, their weighted sum 4) and the wavelength scaling."""
    nl = len(cfg["layers"])
    return float(batch * sum(nv * s["n_sub"] ** 2 * (10 * nl + 1)
                             for s, nv in zip(cfg["sensors"], plan.n_valid)))


def plan_flops(cfg, plan, batch=1):
    """Algorithmic FLOP of one wfs_forward over the plan (valid counts from the library)."""
    tot = 0.0
    for s, nv in zip(cfg["sensors"], plan.n_valid):
        el = s["na_fwhm_m"] > 0 and np.isfinite(s["src_alt_m"])
        tot += nv * flops_per_subap(s["n_sub"], s["n_fft"], s["bin"], el)
    return tot * batch


# ------------------------------------------------------------------------------------------
# timing helpers
# ------------------------------------------------------------------------------------------

def graph_of(torch, fn, n):
    """Capture n calls fn(i) into one HIP graph."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for i in range(min(n, 3)):  # warm the allocator / code objects on the side stream
            fn(i)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    # captured on the warm stream: recon_apply's workspace belongs to the stream it runs on
    with torch.cuda.graph(g, stream=s):
        for i in range(n):
            fn(i)
    torch.cuda.synchronize()
    return g


def timed_replay(torch, g, n_calls):
    """Replay graph g once between events on the current stream; returns (wall s, gpu ms)."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return t1 - t0, e0.elapsed_time(e1) / n_calls


def eager_kernel_ms(torch, fn, n):
    """Mean duration of fn's launch, event pair per call (stream-ordered, eager), after one
    untimed call (first-use allocations and table builds stay outside the mean)."""
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(n)]
    fn(0)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(evs):
        a.record()
        fn(i)
        b.record()
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in evs]))


# ------------------------------------------------------------------------------------------
# workloads
# ------------------------------------------------------------------------------------------

def bench_config1(torch, W, steps, warmup, k0=0, tune=True, flags=0):
    cfg = synth.config1()
    x = torch.from_numpy(synth.make_batch(cfg, [0])).cuda()
    plan = W.Plan(cfg, flags=flags)
    tuned_us = plan.tune(x, iters=10) if tune else None
    slopes, aux = plan.forward(x, step=0)

    def frame(i):
        plan.forward(x, step=k0 + i, seed=42, slopes=slopes, aux=aux)

    for i in range(warmup):
        frame(i)
    kernel_ms_eager = eager_kernel_ms(torch, frame, min(steps, 50))
    g = graph_of(torch, frame, steps)
    g.replay()  # warm replay
    wall1, gpu_ms1 = timed_replay(torch, g, steps)
    del g
    # pipelined frames: one wfs_forward_steps call over the K steps (projection of step k+1
    # inside the spot launch of step k), captured once and replayed
    sK = torch.empty(steps, 1, plan.n_slopes, device="cuda")
    aK = torch.empty(steps, 1, plan.n_valid_total, device="cuda")
    plan.forward_steps(x, k0, min(steps, warmup + 2), slopes=sK[:min(steps, warmup + 2)],
                       aux=aK[:min(steps, warmup + 2)])
    gK = graph_of(torch, lambda i: plan.forward_steps(x, k0, steps, slopes=sK, aux=aK), 1)
    gK.replay()
    wallK, gpu_msK = timed_replay(torch, gK, steps)
    del gK
    out = dict(cfg=cfg, plan=plan, wall=wallK, gpu_ms_per_frame=gpu_msK,
               single_wall=wall1, single_gpu_ms_per_frame=gpu_ms1,
               kernel_ms_eager=kernel_ms_eager, tuned_us=tuned_us, x=x,
               schedule=plan.schedule(), pipelined=plan.schedule()["frames"] != "sequential")
    out.update(kernel_split_ms(torch, plan, x, slopes, aux, k0, min(steps, 100)))
    return out


def kernel_split_ms(torch, plan, x, slopes, aux, k0, n):
    """Per-launch duration of the projection kernel and of the spot kernel of a split frame,
    each from a graph of n back-to-back launches of that kernel alone, HIP events around the
    replay on the launch stream."""
    phase = plan.project(x, step=k0)
    gp = graph_of(torch, lambda i: plan.project(x, step=k0 + i, out=phase), n)
    gp.replay()
    _, proj_ms = timed_replay(torch, gp, n)
    del gp
    gs = graph_of(torch, lambda i: plan.spots(phase, step=k0 + i, seed=42, slopes=slopes,
                                              aux=aux), n)
    gs.replay()
    _, spots_ms = timed_replay(torch, gs, n)
    del gs
    return dict(project_ms=proj_ms, spots_ms=spots_ms)


def bench_batched(torch, W, steps=20, batch=8):
    """Config 2: 6 LGS + 3 NGS x 8 realisations.  The steps are one wfs_forward_steps call
    captured in a HIP graph, pipelined (the projection of step k+1 inside the spot launch of
    step k) if the tuner found that faster; one wfs_forward per step is reported beside it."""
    cfg = synth.config2(batch=batch)
    x = torch.from_numpy(synth.make_batch(cfg, range(batch))).cuda()
    plan = W.Plan(cfg, batch=batch)
    plan.tune(x, iters=20)  # 20 frames a candidate: the steady state of frames in a row
    slopes, aux = plan.forward(x, step=0)

    def step(i):
        plan.forward(x, step=i, seed=42, slopes=slopes, aux=aux)

    g = graph_of(torch, step, steps)
    g.replay()
    _, single_ms = timed_replay(torch, g, steps)
    del g
    sK = torch.empty(steps, batch, plan.n_slopes, device="cuda")
    aK = torch.empty(steps, batch, plan.n_valid_total, device="cuda")
    gK = graph_of(torch, lambda i: plan.forward_steps(x, 0, steps, slopes=sK, aux=aK), 1)
    gK.replay()
    wall, gpu_ms = timed_replay(torch, gK, steps)
    del gK
    n_lgs = sum(1 for s in cfg["sensors"] if np.isfinite(s["src_alt_m"]))
    lgs_subaps = sum(nv for s, nv in zip(cfg["sensors"], plan.n_valid) if np.isfinite(s["src_alt_m"]))
    flops = plan_flops(cfg, plan, batch)
    # the projection of every sensor and realisation on its own: a graph of wfs_project
    # launches; algorithmic bytes = the compulsory union over sensors of the layer pixels the
    # stencils touch (per realisation) + the phase written
    phase = plan.project(x, step=0)
    gp = graph_of(torch, lambda i: plan.project(x, step=i, out=phase), 20)
    gp.replay()
    _, proj_ms = timed_replay(torch, gp, 20)
    del gp, phase
    foot, n_phase = plan.footprint(0)
    proj_bytes = 4.0 * (foot + n_phase) * batch
    return dict(workload="config2: 6 LGS 80x80 + 3 NGS 2x2 (64 px, N=128), 8 realisations, "
                         "10 layers 1024^2, noise on, %d steps in one wfs_forward_steps graph "
                         "(frame schedule as tuned)" % steps,
                ms_per_step=gpu_ms, steps=steps,
                single_step_ms=single_ms,
                lgs_frames_per_s=n_lgs * batch / (gpu_ms * 1e-3),
                subap_spots_per_s=(sum(plan.n_valid) * batch) / (gpu_ms * 1e-3),
                lgs_subaps_per_step=lgs_subaps * batch,
                achieved_tflops=flops / (gpu_ms * 1e-3) / 1e12,
                frac_fp32_valu=flops / (gpu_ms * 1e-3) / PEAK_FP32_VALU,
                projection={"kernel": "wfs_project_kernel", "kernel_ms": proj_ms,
                            "algorithmic_bytes_per_step": proj_bytes,
                            "achieved": proj_bytes / (proj_ms * 1e-3) / 1e9,
                            "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                            "frac": proj_bytes / (proj_ms * 1e-3) / PEAK_HBM},
                schedule=plan.schedule(), paths=plan.paths)


def bench_closed_loop(torch, W, steps=20, batch=8, gain=0.4):
    """Config 4: config-2 sensors with three DM grids as weight -1 layers, reconstructor
    5400 x 55608 applied as a GEMM over the 8 realisations straight into the DM actuators
    (a += g R s), the loop steps captured in one HIP graph."""
    cfg = synth.config4(batch=batch)
    x = torch.from_numpy(synth.make_batch(cfg, range(batch))).cuda()
    plan = W.Plan(cfg, batch=batch)
    plan.tune(x, iters=20)
    R = torch.from_numpy(synth.make_reconstructor(cfg["n_act_rows"], plan.n_slopes)).cuda()
    slopes, aux = plan.forward(x, step=0)
    dm = x.view(batch, -1)[:, cfg["dm_offset"]:]
    ldc = cfg["layer_stride"]

    def step(i):
        plan.forward(x, step=i, seed=42, slopes=slopes, aux=aux)
        W.recon_apply(R, slopes, dm, alpha=gain, beta=1.0, ldc=ldc)

    step(0)
    g = graph_of(torch, step, steps)
    g.replay()
    wall, gpu_ms = timed_replay(torch, g, steps)
    return dict(workload="config4: config2 sensors + 3 DMs (40^2, 42^2, 45^2 @ 0/4/12.7 km), "
                         "R 5400 x 55608 FP32, integrator g=0.4, graph of %d steps" % steps,
                ms_per_step=gpu_ms, steps_per_s=1e3 / gpu_ms, n_slopes=plan.n_slopes)


def bench_calibration(torch, W, batch=128, amp=0.5, eps=0.05, loop_steps=60, gain=0.4):
    """Interaction matrix of the 5,389 config-4 DM actuators by push-pull through the batched
    forward (a DM-only plan, noise off, batch / 2 actuators per call), the regularised
    least-squares control matrix from it, and the config-4 loop closed with that matrix:
    slope norms against the open loop over the same frozen-flow steps (noise on)."""
    cfg4 = synth.config4(batch=8)
    ccfg, n = W.calib.dm_config(cfg4, batch=batch)
    plan = W.Plan(ccfg)
    im, ref = plan.calibrate(0, n, amplitude=amp)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    plan.calibrate(0, n, amplitude=amp, im=im, ref=ref)
    e1.record()
    torch.cuda.synchronize()
    cal_ms = e0.elapsed_time(e1)
    W.tlse(im, eps=eps)  # warm the library handles
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    R = W.tlse(im, eps=eps)
    tlse_ms = (time.perf_counter() - t0) * 1e3
    m_act, n_s = im.shape
    del im
    # library FLOPs of the solve: syrk m^2 n_s, Cholesky m^3 / 3, two triangular solves of
    # m^2 n_s each (FP32, priced against the FP32 matrix-core peak)
    tlse_flops = 3.0 * m_act * m_act * n_s + m_act ** 3 / 3.0
    # closed loop against open loop, same layers and steps, with and without noise
    B = cfg4["batch"]
    x0 = torch.from_numpy(synth.make_batch(cfg4, range(B))).cuda()
    o, ldc = cfg4["dm_offset"], cfg4["layer_stride"]
    x0[:, o:] = 0.0
    tail = max(1, loop_steps // 3)

    def loop(cfg):
        lp = W.Plan(cfg)
        xc = x0.clone()
        dm = xc[:, o:o + n]
        s = torch.empty(B, lp.n_slopes, device="cuda")
        a = torch.empty(B, lp.n_valid_total, device="cuda")
        open_n, closed_n = [], []
        for k in range(loop_steps):
            lp.forward(x0, step=k, slopes=s, aux=a)
            open_n.append(float(s.norm()))
            lp.forward(xc, step=k, slopes=s, aux=a)
            closed_n.append(float(s.norm()))
            W.recon_apply(R, s, dm, alpha=-gain, beta=1.0, ldc=ldc)
        return float(np.mean(closed_n[-tail:]) / np.mean(open_n[-tail:]))

    ratio = loop(cfg4)
    n_lgs = sum(1 for sd in cfg4["sensors"] if np.isfinite(sd["src_alt_m"]))
    real_flops = plan_flops(ccfg, plan)  # one realisation, all nine sensors, FFT convention
    quiet = copy.deepcopy(cfg4)
    for sd in quiet["sensors"]:
        sd["photons"] = 0.0
        sd["read_noise_e"] = 0.0
    ratio_nf = loop(quiet)
    return dict(workload="config4 DMs (5,389 actuators at 0/4/12.7 km) seen by 6 LGS + 3 NGS "
                         "(55,608 slopes); push-pull amplitude %.2f rad, %d realisations per "
                         "call; R = (D^T D + %.2g mean diag I)^-1 D^T" % (amp, batch, eps),
                calibration_ms=cal_ms, actuators_per_s=n / (cal_ms * 1e-3),
                sensor_frames_per_s=2 * n / (cal_ms * 1e-3),
                lgs_frames_per_s=n_lgs * 2 * n / (cal_ms * 1e-3),
                effective_tflops=2 * n * real_flops / (cal_ms * 1e-3) / 1e12,
                tlse_ms=tlse_ms,
                tlse_roofline=dict(bound="mfma", flops=tlse_flops,
                                   achieved=tlse_flops / (tlse_ms * 1e-3) / 1e12, peak=157.3,
                                   unit="TFLOP/s",
                                   frac=tlse_flops / (tlse_ms * 1e-3) / 1e12 / 157.3,
                                   note="rocBLAS ssyrk + rocSOLVER spotrf + 2 rocBLAS strsm, "
                                        "host-timed call including its synchronisation"),
                closed_loop_steps=loop_steps,
                closed_over_open_slope_norm=ratio,
                closed_over_open_slope_norm_noise_free=ratio_nf,
                note="slope norms over the last %d steps, integrator a <- a - %.1f R s"
                     % (tail, gain))


def bench_psf(torch, W, frames=20, lam=2.2e-6, N=2048):
    """Long-exposure K-band PSFs of a 3 x 3 grid of test stars (30 arcsec spacing) through the
    config-4 layers and DMs: 800 x 800 pupil padded to 2048 x 2048, one psf_accumulate per
    frame (row-FFT and column-FFT passes per star), frames captured in one HIP graph."""
    from synth.configs import ARCSEC
    cfg = synth.config4(batch=1)
    x = torch.from_numpy(synth.make_batch(cfg, [0])[0]).cuda()
    stars = [(a * 30 * ARCSEC, b * 30 * ARCSEC) for b in (-1, 0, 1) for a in (-1, 0, 1)]
    n_pup = 800
    plan = W.PsfPlan(cfg, stars, 39.0, 11.0, n_pup, [lam], [N])
    psf, var = plan.buffers()
    g = graph_of(torch, lambda i: plan.accumulate(x, i, psf, var), frames)
    g.replay()
    wall, gpu_ms = timed_replay(torch, g, frames)
    ns = len(stars)
    # HBM bytes a two-pass transform cannot avoid: the row transforms written and read back
    # (n_pup x N complex per star) and the long-exposure image read and written (N^2 floats)
    byts = ns * (2 * n_pup * N * 8 + 2 * N * N * 4)
    # FLOPs, FFT convention: 5 N log2 N per N-point transform (n_pup rows, N columns), and
    # |F|^2, scale and accumulation (4 per image pixel)
    flops = ns * ((n_pup + N) * 5 * N * math.log2(N) + 4 * N * N)
    return dict(workload="config4 layers + DMs, 9 test stars, 800^2 pupil padded to %d^2, "
                         "lambda %.2f um (pixel %.1f mas), graph of %d frames"
                         % (N, lam * 1e6, lam / (N * 39.0 / n_pup) / ARCSEC * 1e3, frames),
                ms_per_frame=gpu_ms, psf_frames_per_s=1e3 / gpu_ms,
                star_psfs_per_s=ns * 1e3 / gpu_ms,
                roofline={"bound": "hbm", "algorithmic_bytes_per_frame": byts,
                          "achieved": byts / (gpu_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                          "unit": "GB/s", "frac": byts / (gpu_ms * 1e-3) / PEAK_HBM},
                alu={"algorithmic_flop_per_frame": flops,
                     "achieved": flops / (gpu_ms * 1e-3) / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": flops / (gpu_ms * 1e-3) / PEAK_FP32_VALU})


def bench_screens(torch, W, reps=5):
    """The ten 1024^2 von Karman layers of config 1 (0.04875 m pitch, r0 per layer, L0 25 m)
    generated on the GPU straight into a layer buffer: one atmosphere = ten screen_generate
    calls, captured in a HIP graph."""
    cfg = synth.config1()
    x = torch.zeros(cfg["layer_stride"], device="cuda")
    turb = [(l, L) for l, L in enumerate(cfg["layers"]) if L["weight"] > 0]
    views = [x[L["offset"]:L["offset"] + L["nx"] * L["ny"]].view(L["ny"], L["nx"])
             for _, L in turb]

    def atmosphere(i):
        for (l, L), v in zip(turb, views):
            W.screen_generate(L["nx"], L["pitch_m"], L["r0_m"], L["L0_m"], 1608 + i, l, out=v)

    g = graph_of(torch, atmosphere, reps)
    g.replay()
    wall, gpu_ms = timed_replay(torch, g, reps)
    n = turb[0][1]["nx"]
    byts = len(turb) * (2 * n * n * 8 + n * n * 4)
    flops = len(turb) * (2 * n * 5 * n * math.log2(n) + 10 * n * n)  # transforms + filter
    return dict(workload="config1 atmosphere: %d von Karman screens %d^2, graph of %d "
                         "atmospheres" % (len(turb), n, reps),
                ms_per_atmosphere=gpu_ms, screens_per_s=len(turb) * 1e3 / gpu_ms,
                roofline={"bound": "hbm", "algorithmic_bytes_per_atmosphere": byts,
                          "achieved": byts / (gpu_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
                          "unit": "GB/s", "frac": byts / (gpu_ms * 1e-3) / PEAK_HBM},
                alu={"algorithmic_flop_per_atmosphere": flops,
                     "achieved": flops / (gpu_ms * 1e-3) / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": flops / (gpu_ms * 1e-3) / PEAK_FP32_VALU})


def bench_adjoint(torch, W, reps=20):
    cfg = synth.config3()
    x = torch.from_numpy(synth.make_batch(cfg, [cfg["guess_realisation"]])).cuda()
    plan = W.Plan(cfg)
    g = torch.from_numpy(synth.random_field((1, plan.n_slopes), seed=7)).cuda()
    s, a = plan.forward(x, step=0)
    out = torch.empty_like(x)
    fwd_ms = eager_kernel_ms(torch, lambda i: plan.forward(x, step=0, slopes=s, aux=a), reps)
    adj_ms = eager_kernel_ms(torch, lambda i: plan.adjoint(x, g, step=0, fwd_slopes=s,
                                                          fwd_aux=a, out=out), reps)
    adj_re_ms = eager_kernel_ms(torch, lambda i: plan.adjoint(x, g, step=0, out=out), reps)
    frames = len(cfg["sensors"])
    return dict(workload="config3: 6 LGS 80x80, 10 layers 1024^2, one realisation, noise off",
                forward_ms=fwd_ms, adjoint_ms=adj_ms, adjoint_recompute_ms=adj_re_ms,
                adjoint_frames_per_s=frames / (adj_ms * 1e-3),
                adjoint_vs_forward=fwd_ms / adj_ms)


def bench_recon(torch, W, reps=10):
    """The config-4 reconstructor on its three kernels: B = 1 (GEMV), B = 8 (the small-batch
    vector-ALU kernel of the loop) and B = 16 (the MFMA kernel)."""
    M, N = synth.configs.N_ACT_ROWS, 55608
    R = torch.from_numpy(synth.make_reconstructor(M, N)).cuda()
    S = torch.from_numpy(synth.random_field((16, N), seed=11)).cuda()
    out = {}
    byts = M * N * 4
    for B in (8, 1, 16):
        Sb = S[:B].contiguous()
        C = torch.zeros(B, M, device="cuda")
        W.recon_apply(R, Sb, C)
        ms = eager_kernel_ms(torch, lambda i: W.recon_apply(R, Sb, C), reps)
        out[f"ms_b{B}"] = ms
        out[f"hbm_gbps_b{B}"] = byts / (ms * 1e-3) / 1e9
        out[f"hbm_frac_b{B}"] = byts / (ms * 1e-3) / PEAK_HBM
    return dict(workload="config4 reconstructor 5400 x 55608 FP32: B=8 (vector-ALU batch "
                         "kernel), B=1 (GEMV), B=16 (MFMA)", **out)


def cpu_baseline(frames=40):
    """The FP64 oracle on whole config-1 frames, one thread."""
    import oracle
    cfg = synth.config1()
    x = synth.make_batch(cfg, [0]).astype(np.float64)
    oracle.forward(x, cfg, 0)  # warm
    t0 = time.perf_counter()
    for k in range(frames):
        oracle.forward(x, cfg, k)
    dt = time.perf_counter() - t0
    return {"value": frames / dt, "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"{frames} full config-1 frames (4,632 subapertures each), numpy FP64, "
                      f"1 thread, {dt:.1f} s"}


def cpu_baseline_configs():
    """The FP64 oracle on the other workloads, one thread (numpy's FFT is single-threaded):
    config 2 as one (realisation, step) of its 6 LGS + 3 NGS with noise, extrapolated to a
    step of 8 realisations and to the 100-step run; the config-3 loss and its gradient (6 LGS,
    ten 1024^2 layers); the config-4 reconstructor as a numpy FP64 matmul of 8 slope vectors
    (BLAS thread count stated)."""
    import oracle
    out = {}
    cfg2 = synth.config2(batch=1)
    x2 = synth.make_batch(cfg2, [0]).astype(np.float64)
    t0 = time.perf_counter()
    oracle.forward(x2, cfg2, 0, realisations=[0])
    dt = time.perf_counter() - t0
    out["config2"] = {"value": 1.0 / (dt * 8), "unit": "steps/s", "cores": 1, "kind": "oracle",
                      "extrapolated": True,
                      "sample": f"one (realisation, step) of 6 LGS + 3 NGS in {dt:.2f} s; a step of "
                                f"8 realisations = 8x, the 100-step run = {800 * dt:.0f} s "
                                "(extrapolated)"}
    cfg3 = synth.config3()
    x3 = synth.make_batch(cfg3, [cfg3["guess_realisation"]]).astype(np.float64)
    target = synth.random_field((1, oracle.n_slopes(cfg3)), seed=7).astype(np.float64)
    t0 = time.perf_counter()
    s3, _ = oracle.forward(x3, cfg3, 0, noise=False)
    oracle.adjoint(x3, cfg3, 0, 2.0 * (s3 - target))
    dt = time.perf_counter() - t0
    out["config3"] = {"value": 1.0 / dt, "unit": "loss+gradient evaluations/s", "cores": 1,
                      "kind": "oracle",
                      "sample": f"one loss + gradient over 6 LGS and ten 1024^2 layers, {dt:.2f} s"}
    try:
        from threadpoolctl import threadpool_info
        blas = [i.get("num_threads") for i in threadpool_info() if i.get("user_api") == "blas"]
        blas_threads = blas[0] if blas else None
    except Exception:
        blas_threads = None
    M, N = synth.configs.N_ACT_ROWS, 55608
    R = synth.make_reconstructor(M, N).astype(np.float64)
    S = synth.random_field((8, N), seed=11).astype(np.float64)
    oracle.recon(R[:64], S)  # warm BLAS
    t0 = time.perf_counter()
    oracle.recon(R, S)
    dt = time.perf_counter() - t0
    del R
    out["config4_recon"] = {"value": 1.0 / dt, "unit": "recon_apply/s", "cores": blas_threads,
                            "kind": "oracle",
                            "sample": f"C = S R^T, R 5400 x 55608 FP64, 8 slope vectors, numpy "
                                      f"matmul with {blas_threads} BLAS threads, {dt * 1e3:.0f} ms"}
    return out


_POOL_X = None


def _oracle_frames(args):
    import oracle
    k0, n = args
    cfg = synth.config1()
    for k in range(k0, k0 + n):
        oracle.forward(_POOL_X, cfg, k)
    return n


def cpu_baseline_pool(frames_per_core=4):
    """The same oracle frames spread over every core of this process's affinity set, one
    single-threaded worker per core (forked before anything touches the GPU)."""
    import multiprocessing as mp
    global _POOL_X
    cores = len(os.sched_getaffinity(0))
    _POOL_X = synth.make_batch(synth.config1(), [0]).astype(np.float64)
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_frames, [(0, 1)] * cores)  # warm every worker
        t0 = time.perf_counter()
        done = sum(pool.map(_oracle_frames, [(c * frames_per_core, frames_per_core)
                                             for c in range(cores)]))
        dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "frames/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} full config-1 frames over {cores} single-threaded worker "
                      f"processes, numpy FP64, {dt:.1f} s"}


def profile_run(torch, W, n, flags=0):
    """Short run for a profiler: the headline's n frames through wfs_forward_steps (with the
    default schedule, one staged-footprint launch for all n frames), one split frame
    (projection kernel, then the spot kernel) for the projection's counters, and n plain
    copies of 256 MiB, the HBM counter calibration.  The plans keep their default schedules:
    timings taken under counter collection would mislead the tuner."""
    cfg = synth.config1()
    x = torch.from_numpy(synth.make_batch(cfg, [0])).cuda()
    plan = W.Plan(cfg, flags=flags)
    sK = torch.empty(n, 1, plan.n_slopes, device="cuda")
    aK = torch.empty(n, 1, plan.n_valid_total, device="cuda")
    src = torch.empty(64 << 20, device="cuda")  # 256 MiB
    dst = torch.empty_like(src)
    split = W.Plan(cfg, flags=flags | W.WFS_FLAG_SPLIT)
    torch.cuda.synchronize()
    plan.forward_steps(x, 0, n, slopes=sK, aux=aK)
    split.forward(x, step=0, slopes=sK[0], aux=aK[0])
    for i in range(n):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"profile_frames": n, "schedule": plan.schedule(),
                      "copy_bytes": 2 * src.numel() * 4}), flush=True)


def kernel_source_digest():
    """SHA-256 of the kernel and ABI sources (the counters in profiles/ name the digest they
    were taken with; a different digest means they no longer describe these kernels)."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(root, "paper_1608_00386_amd", "csrc", "*")))
    files.append(os.path.join(root, "include", "wfs.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None when
    there is none or the kernel sources changed since it was taken."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        "hbm_traffic_config1.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != kernel_source_digest():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if k is None:
        return None
    # per frame: a dispatch of the one-launch schedule covers several frames
    return (k["fetch_bytes"] + k["write_bytes"]) / k.get("frames_per_dispatch", 1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--quick", action="store_true", help="headline only (no extras, no CPU)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=40)
    ap.add_argument("--no-tune", action="store_true", help="keep the plan's default schedule")
    ap.add_argument("--fused", action="store_true", help="projection fused into the spot kernel")
    ap.add_argument("--profile-frames", type=int, default=0,
                    help="short run for a profiler: N pipelined config-1 frames (default "
                         "schedule) and N plain copies of 256 MiB (the HBM counter "
                         "calibration), then exit")
    ap.add_argument("--only", choices=["psf", "calibration", "adjoint", "recon", "batched",
                                       "closed_loop", "screens"],
                    help="run one of the extra workloads alone and print its JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (got --gpus {args.gpus}); the "
              "multi-GPU sharding is a design note, not a launched path.", file=sys.stderr)
        sys.exit(2)

    cpu = cpu_pool = cpu_cfgs = None
    if not args.quick and not args.no_cpu and args.profile_frames == 0:
        # the oracle baselines run first: the pool forks before anything touches the GPU
        log("[bench] cpu baseline (oracle, 1 thread) ...")
        cpu = cpu_baseline(args.cpu_frames)
        log("[bench] cpu baseline (oracle, all cores) ...")
        try:
            cpu_pool = cpu_baseline_pool()
        except Exception as e:  # report, do not hide
            cpu_pool = {"error": repr(e)}
        log("[bench] cpu baseline (oracle) of configs 2-4 ...")
        try:
            cpu_cfgs = cpu_baseline_configs()
        except Exception as e:
            cpu_cfgs = {"error": repr(e)}

    import torch
    import paper_1608_00386_amd as W
    W.lib()  # fails loudly when the HIP library is missing
    torch.cuda.set_device(0)

    if args.profile_frames > 0:
        profile_run(torch, W, args.profile_frames, flags=W.WFS_FLAG_FUSED if args.fused else 0)
        return
    if args.only:  # one extra on its own (a short run for a profiler)
        fn = {"psf": bench_psf, "calibration": bench_calibration, "adjoint": bench_adjoint,
              "screens": bench_screens,
              "recon": bench_recon, "batched": bench_batched,
              "closed_loop": bench_closed_loop}[args.only]
        print(json.dumps({args.only: fn(torch, W)}), flush=True)
        return

    log("[bench] config1 forward ...")
    r1 = bench_config1(torch, W, args.steps, args.warmup, tune=not args.no_tune,
                       flags=W.WFS_FLAG_FUSED if args.fused else 0)
    cfg1 = r1["cfg"]
    subaps = r1["plan"].n_valid[0]
    frames_per_s = args.steps / r1["wall"]
    spot_flops = plan_flops(cfg1, r1["plan"])
    flops = spot_flops
    # dominant kernel: the spot launch, charged with the spot stage's algorithmic FLOPs only
    # (96,020 per LGS subaperture); when its waves also project their own pixels (staged
    # footprint) that work is reported beside it (projection_flop_per_frame), not added; a
    # separate projection kernel's bytes are reported under "projection".
    #   one launch (staged footprint): the K frames are one dispatch; per frame, the replayed
    #     graph's time divided by K;
    #   pipelined (split): one launch per frame that forms the spots of step k and projects
    #     step k+1; the graph's time per frame less the one leading projection;
    #   sequential split / gather: the spot launch of each frame.
    frames = r1["schedule"]["frames"]
    field = r1["schedule"]["field"]
    lp = r1["schedule"].get("lag_passes", 2)  # last template argument of the spot kernels
    if frames == "one_launch":
        kern_ms = r1["gpu_ms_per_frame"]
        kern_name = ("wfs_forward_kernel<10, footprint> (the K frames of one call in launches "
                     "of up to 256 frames, each after the small launch that fills its frames' "
                     "stencil entries; each wave projects its subaperture from a footprint "
                     "staged in LDS)")
        traffic_key = "wfs_forward_kernel<10, 2, false, false, 2>"
    elif frames == "pipelined":
        kern_ms = (r1["gpu_ms_per_frame"] * args.steps - r1["project_ms"]) / args.steps
        kern_name = "wfs_forward_kernel<10, split> (spots of step k + projection of step k+1)"
        traffic_key = "wfs_forward_kernel<10, 1, false, true, %d>" % lp
    elif frames == "overlapped":  # projections run beside the spots: the spot launch alone
        kern_ms = r1["spots_ms"]
        kern_name = "wfs_forward_kernel<10, split> (spots; projections on a second stream)"
        traffic_key = "wfs_forward_kernel<10, 1, false, false, %d>" % lp
    elif field == "split":
        kern_ms = r1["gpu_ms_per_frame"] - r1["project_ms"]
        kern_name = "wfs_forward_kernel<10, split> (spots)"
        traffic_key = "wfs_forward_kernel<10, 1, false, false, %d>" % lp
    elif field == "footprint":
        kern_ms = r1["gpu_ms_per_frame"]
        kern_name = "wfs_forward_kernel<10, footprint> (one frame per launch)"
        traffic_key = "wfs_forward_kernel<10, 2, false, false, 2>"
    else:
        kern_ms = r1["gpu_ms_per_frame"]
        kern_name = "wfs_forward_kernel<10, gather> (per-pixel gather)"
        traffic_key = "wfs_forward_kernel<10, 0, false, false, 2>"
    in_wave_proj = field == "footprint" or frames == "one_launch"
    achieved = flops / (kern_ms * 1e-3)
    foot, n_phase = r1["plan"].footprint(0)
    proj_bytes = 4.0 * (foot + n_phase)  # each layer pixel read once, each phase pixel written
    out = {
        "metric": METRIC,
        "value": frames_per_s,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r1["wall"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded von Karman screens, config-1 geometry)",
        "config": {"workload": "config1: E-ELT 80x80 LGS, 39 m/11 m pupil, 4632 subaps of 10x10 "
                               "px, N=32, 8x8 px, 10 layers 1024^2 0-16 km, H=90 km, Na 10 km, "
                               "noise on", "frames_per_step": 1, "subaps": subaps,
                   "graph_replay": True, "frames_schedule": r1["schedule"]["frames"]},
        "spots_per_s": frames_per_s * subaps,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32_VALU / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VALU,
                     "traffic": recorded_traffic(traffic_key),
                     "kernel": kern_name,
                     "kernel_ms": kern_ms,
                     "algorithmic_flop_per_frame": flops,
                     "projection_flop_per_frame": proj_flops(cfg1, r1["plan"]),
                     "projection_in_launch": in_wave_proj,
                     "frames_per_call": args.steps if frames == "one_launch" else 1,
                     "spots_only_kernel_ms": r1["spots_ms"],
                     "spots_only_frac": spot_flops / (r1["spots_ms"] * 1e-3) / PEAK_FP32_VALU,
                     "schedule": r1["schedule"]},
        "single_frame": {"frames_per_s": args.steps / r1["single_wall"],
                         "gpu_ms_per_frame": r1["single_gpu_ms_per_frame"],
                         "eager_ms_per_frame": r1["kernel_ms_eager"],
                         "note": "one wfs_forward per frame (projection, then spots), graph "
                                 "of K frames"},
        "projection": {"bound": "hbm", "kernel": "wfs_project_kernel", "kernel_ms":
                       r1["project_ms"], "algorithmic_bytes_per_launch": proj_bytes,
                       "achieved": proj_bytes / (r1["project_ms"] * 1e-3) / 1e9,
                       "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                       "frac": proj_bytes / (r1["project_ms"] * 1e-3) / PEAK_HBM,
                       "traffic": recorded_traffic("wfs_project_kernel")},
    }
    if not args.quick:
        try:
            log("[bench] config3 adjoint ...")
            adj = bench_adjoint(torch, W)
            adj["plain_forward_frames_per_s"] = frames_per_s
            out["adjoint"] = adj
        except Exception as e:  # report, do not hide
            out["adjoint"] = {"error": repr(e)}
        try:
            log("[bench] config4 reconstructor ...")
            out["recon"] = bench_recon(torch, W)
        except Exception as e:
            out["recon"] = {"error": repr(e)}
        try:
            log("[bench] config2 batched ...")
            bt = bench_batched(torch, W)
            bt["lgs_frames_vs_plain_forward"] = bt["lgs_frames_per_s"] / frames_per_s
            out["batched"] = bt
        except Exception as e:
            out["batched"] = {"error": repr(e)}
        try:
            log("[bench] config4 closed loop ...")
            out["closed_loop"] = bench_closed_loop(torch, W)
        except Exception as e:
            out["closed_loop"] = {"error": repr(e)}
        try:
            log("[bench] config4 calibration and calibrated loop ...")
            out["calibration"] = bench_calibration(torch, W)
        except Exception as e:
            out["calibration"] = {"error": repr(e)}
        try:
            log("[bench] screens ...")
            out["screens"] = bench_screens(torch, W)
        except Exception as e:
            out["screens"] = {"error": repr(e)}
        try:
            log("[bench] PSF module ...")
            out["psf"] = bench_psf(torch, W)
        except Exception as e:
            out["psf"] = {"error": repr(e)}
        if cpu is not None:
            out["cpu_baseline"] = cpu
            out["cpu_baseline_all_cores"] = cpu_pool
            out["cpu_baseline_other_configs"] = cpu_cfgs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
