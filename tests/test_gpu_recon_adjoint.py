"""GPU parity of recon_apply and wfs_adjoint against the FP64 oracle."""

import numpy as np
import pytest

import oracle
import synth
from wfs_cases import CASES, layers_for

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    import paper_1608_00386_amd as W
    return torch, W


def _recon_check(R, S, C0, alpha, beta, got, rows=None, rel=2e-5):
    rows = np.arange(R.shape[0]) if rows is None else rows
    R64 = R[rows].astype(np.float64)
    S64 = S.astype(np.float64)
    ref = alpha * (S64 @ R64.T) + beta * C0[:, rows].astype(np.float64)
    scale = np.abs(alpha) * (np.abs(S64) @ np.abs(R64).T) + np.abs(beta * C0[:, rows]) + 1e-30
    err = np.abs(got[:, rows] - ref) / scale
    assert err.max() <= rel, f"recon error {err.max():.3g} of sum |R s|"


@pytest.mark.parametrize("M,N,B", [(37, 101, 1), (37, 101, 3), (70, 256, 1), (70, 256, 2),
                                   (70, 256, 8), (45, 1000, 17), (300, 4096, 8)])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (0.4, 1.0)])
def test_recon_small(M, N, B, alpha, beta):
    torch, W = _gpu()
    rng = np.random.default_rng(M * 1000 + N + B)
    R = rng.standard_normal((M, N)).astype(np.float32)
    S = rng.standard_normal((B, N)).astype(np.float32)
    ldc = M + 5
    C0 = rng.standard_normal((B, ldc)).astype(np.float32)
    Ct = torch.from_numpy(C0.copy()).cuda()
    W.recon_apply(torch.from_numpy(R).cuda(), torch.from_numpy(S).cuda(), Ct, alpha=alpha,
                  beta=beta, ldc=ldc)
    got = Ct.cpu().numpy().astype(np.float64)
    _recon_check(R, S, C0[:, :M], alpha, beta, got[:, :M])
    np.testing.assert_array_equal(got[:, M:], C0[:, M:])  # padding untouched


def test_recon_integer_exact():
    torch, W = _gpu()
    rng = np.random.default_rng(3)
    R = rng.integers(-3, 4, size=(50, 400)).astype(np.float32)
    S = rng.integers(-3, 4, size=(4, 400)).astype(np.float32)
    C = W.recon_apply(torch.from_numpy(R).cuda(), torch.from_numpy(S).cuda())
    np.testing.assert_array_equal(C.cpu().numpy(), (S.astype(np.int64) @ R.T.astype(np.int64)))


@pytest.mark.parametrize("B", [1, 8])
def test_recon_full_size_sampled_rows(B):
    """5,400 x 55,608 reconstructor (entries N(0,1)/sqrt(N)), sampled rows against FP64."""
    torch, W = _gpu()
    M, N = 5400, 55608
    R = synth.make_reconstructor(M, N)
    S = synth.random_field((B, N), seed=11)
    Rt = torch.from_numpy(R).cuda()
    St = torch.from_numpy(S).cuda()
    C = W.recon_apply(Rt, St)
    C2 = W.recon_apply(Rt, St)
    assert torch.equal(C, C2)  # deterministic
    rows = np.random.default_rng(0).choice(M, 64, replace=False)
    rows = np.concatenate([rows, [0, M - 1]])
    got = C.cpu().numpy().astype(np.float64)
    _recon_check(R, S, np.zeros((B, M), np.float32), 1.0, 0.0, got, rows=rows, rel=1e-4)


def test_recon_streams_and_graphs_keep_their_own_workspace():
    """Calls on two streams at once use separate partial-sum buffers (each result equals the
    call made alone); a graph captured on a stream still replays correctly after a larger
    problem on that stream has outgrown its buffer (the old buffer stays alive); and a capture
    that would need a new buffer is refused with an error instead of allocating."""
    torch, W = _gpu()
    rng = np.random.default_rng(5)
    M, N = 700, 20000
    Ra = torch.from_numpy(rng.standard_normal((M, N)).astype(np.float32)).cuda()
    Rb = torch.from_numpy(rng.standard_normal((M, N)).astype(np.float32)).cuda()
    Sa = torch.from_numpy(rng.standard_normal((8, N)).astype(np.float32)).cuda()
    Sb = torch.from_numpy(rng.standard_normal((8, N)).astype(np.float32)).cuda()
    ref_a = W.recon_apply(Ra, Sa)
    ref_b = W.recon_apply(Rb, Sb)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for s in (s1, s2):
        s.wait_stream(torch.cuda.current_stream())
    for _ in range(3):
        with torch.cuda.stream(s1):
            ca = W.recon_apply(Ra, Sa, stream=s1)
        with torch.cuda.stream(s2):
            cb = W.recon_apply(Rb, Sb, stream=s2)
        torch.cuda.synchronize()
        assert torch.equal(ca, ref_a) and torch.equal(cb, ref_b)
    # a graph on s1, then a larger problem on s1 (new buffer), then replays
    out = torch.zeros(8, M, device="cuda")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s1):
        W.recon_apply(Ra, Sa, out, stream=s1)
    Mb = 5000
    Rbig = torch.from_numpy(rng.standard_normal((Mb, N)).astype(np.float32)).cuda()
    with torch.cuda.stream(s1):
        big = W.recon_apply(Rbig, Sa, stream=s1)
    torch.cuda.synchronize()
    for rep in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref_a), rep
    _recon_check(Rbig.cpu().numpy(), Sa.cpu().numpy(), np.zeros((8, Mb), np.float32), 1.0, 0.0,
                 big.cpu().numpy().astype(np.float64), rows=np.arange(0, Mb, 97))
    # capture on a stream whose buffer is too small: refused before any launch
    s3 = torch.cuda.Stream()
    g2 = torch.cuda.CUDAGraph()
    with pytest.raises(RuntimeError, match="capturing"):
        with torch.cuda.graph(g2, stream=s3):
            W.recon_apply(Ra, Sa, stream=s3)
    torch.cuda.synchronize()


def _adjoint_case(name, seed=1):
    cfg = CASES[name]()
    for s in cfg["sensors"]:
        s["photons"] = 0.0
        s["read_noise_e"] = 0.0
    x = layers_for(cfg, scale=0.5)
    g = synth.random_field((cfg["batch"], oracle.n_slopes(cfg)), seed=seed)
    return cfg, x, g


@pytest.mark.parametrize("name", ["lgs_n4_N8_b2", "lgs_n10_N32_b4_noise",
                                  "lgs_n5_N10_b2_2sens_batch3", "dm_two_ngs_batch2", "cfg0",
                                  "ngs_n6_N12_b4_oddpix"])
@pytest.mark.parametrize("saved", [False, True])
@pytest.mark.parametrize("mode", ["split", "fused", "split_atomic", "footprint"])
def test_adjoint_matches_oracle(name, saved, mode):
    torch, W = _gpu()
    cfg, x, g = _adjoint_case(name)
    step = 4
    flags = {"split": W.WFS_FLAG_SPLIT, "fused": W.WFS_FLAG_FUSED,
             "split_atomic": W.WFS_FLAG_SPLIT | W.WFS_FLAG_ADJOINT_ATOMIC,
             "footprint": W.WFS_FLAG_FOOTPRINT}[mode]
    plan = W.Plan(cfg, flags=flags)
    xt = torch.from_numpy(x).cuda()
    gt = torch.from_numpy(g).cuda()
    if saved:
        s, a = plan.forward(xt, step=step)
        out = plan.adjoint(xt, gt, step=step, fwd_slopes=s, fwd_aux=a)
    else:
        out = plan.adjoint(xt, gt, step=step)
    got = out.cpu().numpy().astype(np.float64)
    ref = oracle.adjoint(x.astype(np.float64), cfg, step, g.astype(np.float64))
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel <= 1e-4, rel
    assert np.abs(got - ref).max() <= 1e-3 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["fft_ngs_n14_N32_b4", "fft_ngs_n20_N64_b2",
                                  "fft_ngs_n64_N128_b4", "fft_ngs_n40_N128_b4",
                                  "mixed_lgs_ngs_batch2"])
@pytest.mark.parametrize("saved", [False, True])
@pytest.mark.parametrize("mode", ["split", "fused"])
def test_adjoint_fft_path_matches_oracle(name, saved, mode):
    """Sensors on the FFT path (one wave per spectrum chunk: one chunk at N = 32, four at 64,
    sixteen at 128), alone and beside a lag-domain LGS, against the FP64 oracle gradient."""
    torch, W = _gpu()
    cfg, x, g = _adjoint_case(name)
    step = 5
    plan = W.Plan(cfg, flags=W.WFS_FLAG_SPLIT if mode == "split" else W.WFS_FLAG_FUSED)
    assert 1 in plan.paths
    xt = torch.from_numpy(x).cuda()
    gt = torch.from_numpy(g).cuda()
    if saved:
        s, a = plan.forward(xt, step=step)
        out = plan.adjoint(xt, gt, step=step, fwd_slopes=s, fwd_aux=a)
    else:
        out = plan.adjoint(xt, gt, step=step)
    got = out.cpu().numpy().astype(np.float64)
    ref = oracle.adjoint(x.astype(np.float64), cfg, step, g.astype(np.float64))
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel <= 1e-4, rel
    assert np.abs(got - ref).max() <= 1e-3 * np.abs(ref).max()
    o2 = plan.adjoint(xt, gt, step=step)
    assert torch.equal(o2, plan.adjoint(xt, gt, step=step))  # bitwise deterministic


def test_adjoint_fft_path_refuses_the_atomic_scatter():
    torch, W = _gpu()
    cfg, x, g = _adjoint_case("fft_ngs_n14_N32_b4")
    plan = W.Plan(cfg, flags=W.WFS_FLAG_ADJOINT_ATOMIC)
    with pytest.raises(W.WfsError) as e:
        plan.adjoint(torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda(), step=1)
    assert e.value.code == -4


@pytest.mark.parametrize("name", ["lgs_n10_N32_b4_noise", "dm_two_ngs_batch2"])
def test_adjoint_gather_is_bitwise_deterministic(name):
    torch, W = _gpu()
    cfg, x, g = _adjoint_case(name)
    plan = W.Plan(cfg)
    xt = torch.from_numpy(x).cuda()
    gt = torch.from_numpy(g).cuda()
    o1 = plan.adjoint(xt, gt, step=3).clone()
    o2 = plan.adjoint(xt, gt, step=3)
    assert torch.equal(o1, o2)


def test_adjoint_small_periodic_grid_wraps():
    """A screen smaller than the pupil footprint (several periodic images per pixel)."""
    torch, W = _gpu()
    from wfs_cases import ngs_case
    cfg = ngs_case(6, 4, 8, 2, D=6.0, layers=1, n=16, pitch=0.25)
    for s in cfg["sensors"]:
        s["photons"] = 0.0
    x = layers_for(cfg, scale=0.5)
    g = synth.random_field((1, oracle.n_slopes(cfg)), seed=4)
    plan = W.Plan(cfg)
    out = plan.adjoint(torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda(), step=5)
    ref = oracle.adjoint(x.astype(np.float64), cfg, 5, g.astype(np.float64))
    got = out.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-4


@pytest.mark.parametrize("n,D", [(128, 12.5), (64, 6.0)])
def test_adjoint_coarse_pupil_two_periodic_images(n, D):
    """A pupil 2.5 times as coarse as the layer (2.5 layer pixels per pupil pixel) whose
    footprint wraps about twice around a small periodic screen: most layer pixels take taps
    from two periodic images, which the gather finds by searching each tile's candidates."""
    torch, W = _gpu()
    from wfs_cases import ngs_case
    cfg = ngs_case(10 if n == 128 else 8, 10 if n == 128 else 6, 20 if n == 128 else 12, 2,
                   D=D, layers=2, n=n, pitch=0.05)
    for s in cfg["sensors"]:
        s["photons"] = 0.0
    x = layers_for(cfg, scale=0.5)
    g = synth.random_field((1, oracle.n_slopes(cfg)), seed=8)
    plan = W.Plan(cfg)
    out = plan.adjoint(torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda(), step=3)
    ref = oracle.adjoint(x.astype(np.float64), cfg, 3, g.astype(np.float64))
    got = out.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-4
    assert np.abs(got - ref).max() <= 1e-3 * np.abs(ref).max()
    o2 = plan.adjoint(torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda(), step=3)
    assert torch.equal(out, o2)


def test_autograd_function_uses_the_adjoint():
    torch, W = _gpu()
    cfg, x, _ = _adjoint_case("lgs_n5_N10_b2_2sens_batch3")
    plan = W.Plan(cfg)
    target = torch.zeros(cfg["batch"], plan.n_slopes, device="cuda")
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    s = W.wfs_slopes(xt, plan, step=2)
    loss = ((s - target) ** 2).sum()
    loss.backward()
    s_ref = oracle.forward(x.astype(np.float64), cfg, 2, noise=False)[0]
    ref = oracle.adjoint(x.astype(np.float64), cfg, 2, 2.0 * s_ref)
    got = xt.grad.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-4


def test_autograd_function_on_a_noisy_plan_uses_the_noise_free_adjoint():
    """With photon and read noise on, WFSFunction's backward does not reuse the noisy forward
    outputs: it runs the adjoint of the noise-free model (fields and spot sums recomputed), so
    the layer gradient of sum(s^2) is J^T (2 s) with J the noise-free Jacobian and s the noisy
    slopes the forward returned."""
    import copy
    torch, W = _gpu()
    cfg = CASES["lgs_n10_N32_b4_noise"]()
    assert any(sd["photons"] > 0 for sd in cfg["sensors"])
    x = layers_for(cfg, scale=0.5)
    plan = W.Plan(cfg)
    xt = torch.from_numpy(x).cuda().requires_grad_(True)
    s = W.wfs_slopes(xt, plan, step=3, seed=11)
    (s ** 2).sum().backward()
    g = 2.0 * s.detach().cpu().numpy().astype(np.float64)
    quiet = copy.deepcopy(cfg)
    for sd in quiet["sensors"]:
        sd["photons"] = 0.0
        sd["read_noise_e"] = 0.0
    s_quiet = oracle.forward(x.astype(np.float64), quiet, 3, noise=False)[0]
    assert np.abs(g / 2.0 - s_quiet).max() > 1e-3  # the forward really was noisy
    ref = oracle.adjoint(x.astype(np.float64), quiet, 3, g)
    got = xt.grad.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-4


def test_adjoint_dot_product_with_gpu_forward():
    """<J v, g> from a central difference of the GPU forward equals <v, J^T g> from the GPU
    adjoint (to the accuracy of an FP32 difference quotient)."""
    torch, W = _gpu()
    cfg, x, g = _adjoint_case("lgs_n10_N32_b4_noise")
    plan = W.Plan(cfg)
    xt = torch.from_numpy(x).cuda()
    gt = torch.from_numpy(g).cuda()
    adj = plan.adjoint(xt, gt, step=1).double()
    v = torch.from_numpy(synth.random_field(x.shape, seed=5)).cuda()
    h = 1e-2
    sp, _ = plan.forward(xt + h * v, step=1)
    sp = sp.double().clone()
    sm, _ = plan.forward(xt - h * v, step=1)
    jv = (sp - sm.double()) / (2 * h)
    lhs = float((jv * gt.double()).sum())
    rhs = float((adj * v.double()).sum())
    assert abs(lhs - rhs) <= 2e-3 * max(abs(lhs), abs(rhs)), (lhs, rhs)
