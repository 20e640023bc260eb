"""Python front end of libwfs: plans, the forward sensor model, its adjoint (autograd) and the
reconstructor.  Argument marshalling only: every step runs in the HIP kernels of libwfs.so.

PyTorch provides device memory and streams.  Tensors must be float32, contiguous and on the
plan's GPU.
"""

import ctypes

import torch

from . import _lib as L


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need(t, name, shape=None, numel=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32 (got {t.dtype})")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


class Plan:
    """A set of Shack-Hartmann sensors looking through a set of layers (``wfs_plan``).

    ``cfg`` is a dict with ``layers`` and ``sensors`` (the fields of wfs_layer_desc and
    wfs_sensor_desc), ``layer_stride``, ``batch``, ``lambda_ref_m`` and ``dt_s``; an optional
    ``na_profile`` (sodium-profile time series) goes to ``wfs_plan_na_profile``.
    """

    def __init__(self, cfg, flags=0, batch=None):
        self._lib = L.lib()
        self.cfg = cfg
        self.batch = int(batch if batch is not None else cfg.get("batch", 1))
        self.layer_stride = int(cfg["layer_stride"])
        nl, ns = len(cfg["layers"]), len(cfg["sensors"])
        self._ld = (L.LayerDesc * nl)(*[L.layer_desc(x) for x in cfg["layers"]])
        self._sd = (L.SensorDesc * ns)(*[L.sensor_desc(x) for x in cfg["sensors"]])
        h = ctypes.c_void_p()
        L.check(self._lib.wfs_plan(self._ld, nl, self.layer_stride, self._sd, ns, self.batch,
                                   float(cfg["lambda_ref_m"]), float(cfg["dt_s"]), int(flags),
                                   ctypes.byref(h)), "wfs_plan")
        self._h = h
        n_slopes, n_valid_total = ctypes.c_int32(), ctypes.c_int32()
        nv = (ctypes.c_int32 * ns)()
        ps = (ctypes.c_double * ns)()
        L.check(self._lib.wfs_plan_info(h, ctypes.byref(n_slopes), ctypes.byref(n_valid_total),
                                        nv, ps), "wfs_plan_info")
        self.n_slopes = n_slopes.value
        self.n_valid_total = n_valid_total.value
        self.n_valid = list(nv)
        self.pix_scale = list(ps)
        paths = (ctypes.c_int32 * ns)()
        L.check(self._lib.wfs_plan_path(h, paths), "wfs_plan_path")
        self.paths = list(paths)
        self.device = torch.cuda.current_device()
        if cfg.get("na_profile"):
            self.set_na_profile(cfg["na_profile"])

    def set_na_profile(self, profile):
        """Time-varying multi-peak sodium profile: a list of entries (frame k uses entry
        k mod len), each a list of (dh_m, fwhm_m, weight) peaks; None or [] restores the
        sensors' single Gaussians (``wfs_plan_na_profile``; synchronises the device)."""
        if not profile:
            L.check(self._lib.wfs_plan_na_profile(self._h, 0, 0, None), "wfs_plan_na_profile")
            return
        n_e, n_p, tab = L.na_profile_table(profile)
        L.check(self._lib.wfs_plan_na_profile(self._h, n_e, n_p, tab), "wfs_plan_na_profile")

    # -- lifetime -------------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.check(self._lib.wfs_plan_destroy(self._h), "wfs_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- calls ----------------------------------------------------------------------------
    def _layers(self, layers):
        _need(layers, "layers", numel=self.batch * self.layer_stride)

    def forward(self, layers, step=0, seed=42, slopes=None, aux=None, stream=None):
        """Slopes [B][n_slopes] (and per-subaperture flux [B][n_valid_total])."""
        self._layers(layers)
        if slopes is None:
            slopes = torch.empty(self.batch, self.n_slopes, device=layers.device)
        if aux is None:
            aux = torch.empty(self.batch, self.n_valid_total, device=layers.device)
        _need(slopes, "slopes", numel=self.batch * self.n_slopes)
        _need(aux, "aux", numel=self.batch * self.n_valid_total)
        L.check(self._lib.wfs_forward(self._h, _ptr(layers), int(step), int(seed), _ptr(slopes),
                                      _ptr(aux), _stream(stream)), "wfs_forward")
        return slopes, aux

    def forward_steps(self, layers, step0, n_steps, seed=42, slopes=None, aux=None,
                      stream=None):
        """Slopes [n_steps][B][n_slopes] of steps step0 .. step0+n_steps-1 (pipelined)."""
        self._layers(layers)
        n = int(n_steps)
        if slopes is None:
            slopes = torch.empty(n, self.batch, self.n_slopes, device=layers.device)
        if aux is None:
            aux = torch.empty(n, self.batch, self.n_valid_total, device=layers.device)
        _need(slopes, "slopes", numel=n * self.batch * self.n_slopes)
        _need(aux, "aux", numel=n * self.batch * self.n_valid_total)
        L.check(self._lib.wfs_forward_steps(self._h, _ptr(layers), int(step0), n, int(seed),
                                            _ptr(slopes), _ptr(aux), _stream(stream)),
                "wfs_forward_steps")
        return slopes, aux

    @property
    def phase_numel(self):
        return sum(nv * s["n_sub"] ** 2 for nv, s in zip(self.n_valid, self.cfg["sensors"]))

    def spots(self, phase, step=0, seed=42, slopes=None, aux=None, stream=None):
        """Slopes from a phase buffer laid out as ``project`` returns it (``wfs_spots``)."""
        _need(phase, "phase", numel=self.batch * self.phase_numel)
        if slopes is None:
            slopes = torch.empty(self.batch, self.n_slopes, device=phase.device)
        if aux is None:
            aux = torch.empty(self.batch, self.n_valid_total, device=phase.device)
        _need(slopes, "slopes", numel=self.batch * self.n_slopes)
        _need(aux, "aux", numel=self.batch * self.n_valid_total)
        L.check(self._lib.wfs_spots(self._h, _ptr(phase), int(step), int(seed), _ptr(slopes),
                                    _ptr(aux), _stream(stream)), "wfs_spots")
        return slopes, aux

    FIELDS = ("gather", "split", "footprint")
    FRAMES = ("sequential", "pipelined", "one_launch", "overlapped")
    FFT_LAUNCH = ("side_stream", "same_launch")

    def schedule(self):
        """dict(field, frames, xcd_remap, fft_launch, proj_rows) of the current launch
        schedule: field is where a frame's spot waves get the phase ("gather", "split",
        "footprint"), frames how ``forward_steps`` runs ("sequential", "pipelined",
        "one_launch", "overlapped": the next frame projected on a second stream), fft_launch where FFT-path blocks run ("side_stream" or "same_launch"),
        proj_rows the projection kernel's pupil rows per block, lag_passes the split field's
        passes over each lag row (2 or 3)."""
        v = [ctypes.c_int32() for _ in range(6)]
        L.check(self._lib.wfs_plan_schedule(self._h, *[ctypes.byref(x) for x in v]),
                "wfs_plan_schedule")
        return dict(field=self.FIELDS[v[0].value], frames=self.FRAMES[v[1].value],
                    xcd_remap=v[2].value, fft_launch=self.FFT_LAUNCH[v[3].value],
                    proj_rows=v[4].value, lag_passes=v[5].value)

    def set_schedule(self, field=None, frames=None, xcd_remap=None, fft_launch=None,
                     proj_rows=None, lag_passes=None):
        """Pin a launch schedule (names as ``schedule`` reports them; None keeps a choice)."""
        def code(names, v):
            return -1 if v is None else (names.index(v) if isinstance(v, str) else int(v))
        L.check(self._lib.wfs_plan_set_schedule(
            self._h, code(self.FIELDS, field), code(self.FRAMES, frames),
            -1 if xcd_remap is None else int(xcd_remap), code(self.FFT_LAUNCH, fft_launch),
            -1 if proj_rows is None else int(proj_rows),
            -1 if lag_passes is None else int(lag_passes)), "wfs_plan_set_schedule")

    def footprint(self, step=0):
        """(distinct layer pixels read, projected pixels) per realisation at ``step``."""
        d, n = ctypes.c_int64(), ctypes.c_int64()
        L.check(self._lib.wfs_plan_footprint(self._h, int(step), ctypes.byref(d),
                                             ctypes.byref(n)), "wfs_plan_footprint")
        return d.value, n.value

    def project(self, layers, step=0, out=None, stream=None):
        self._layers(layers)
        n = self.phase_numel
        if out is None:
            out = torch.empty(self.batch, n, device=layers.device)
        _need(out, "phase", numel=self.batch * n)
        L.check(self._lib.wfs_project(self._h, _ptr(layers), int(step), _ptr(out),
                                      _stream(stream)), "wfs_project")
        return out

    def adjoint(self, layers, grad_slopes, step=0, fwd_slopes=None, fwd_aux=None, out=None,
                stream=None):
        self._layers(layers)
        _need(grad_slopes, "grad_slopes", numel=self.batch * self.n_slopes)
        if (fwd_slopes is None) != (fwd_aux is None):
            raise ValueError("give both fwd_slopes and fwd_aux, or neither")
        if fwd_slopes is not None:
            _need(fwd_slopes, "fwd_slopes", numel=self.batch * self.n_slopes)
            _need(fwd_aux, "fwd_aux", numel=self.batch * self.n_valid_total)
        if out is None:
            out = torch.empty_like(layers)
        _need(out, "grad_layers", numel=self.batch * self.layer_stride)
        L.check(self._lib.wfs_adjoint(self._h, _ptr(layers), _ptr(grad_slopes),
                                      _ptr(fwd_slopes), _ptr(fwd_aux), int(step), _ptr(out),
                                      _stream(stream)), "wfs_adjoint")
        return out

    def set_step(self, step, stream=None):
        L.check(self._lib.wfs_set_step(self._h, int(step), _stream(stream)), "wfs_set_step")

    def advance_step(self, delta=1, stream=None):
        L.check(self._lib.wfs_advance_step(self._h, int(delta), _stream(stream)),
                "wfs_advance_step")

    def calibrate(self, act_offset, n_act, amplitude=0.1, step=0, seed=42, base=None,
                  im=None, ref=None, stream=None):
        """Push-pull interaction matrix of actuators act_offset .. act_offset + n_act - 1 of a
        realisation's buffer (``wfs_calibrate``): returns (im [n_act][n_slopes], ref
        [n_slopes]); row j is d slopes / d actuator j.  The plan's batch (even) sets the
        actuators per forward call (batch / 2)."""
        n_act = int(n_act)
        dev = torch.device("cuda", self.device)
        if base is not None:
            _need(base, "base", numel=self.layer_stride)
        if im is None:
            im = torch.empty(n_act, self.n_slopes, device=dev)
        if ref is None:
            ref = torch.empty(self.n_slopes, device=dev)
        _need(im, "im")
        _need(ref, "ref", numel=self.n_slopes)
        if im.dim() != 2 or im.shape[0] != n_act or im.shape[1] < self.n_slopes:
            raise ValueError(f"im {tuple(im.shape)} must be [{n_act}][>= {self.n_slopes}]")
        nw = ctypes.c_int64()
        L.check(self._lib.wfs_calibrate_work(self._h, ctypes.byref(nw)), "wfs_calibrate_work")
        work = torch.empty(nw.value, device=dev)
        L.check(self._lib.wfs_calibrate(self._h, _ptr(base), int(act_offset), n_act,
                                        float(amplitude), int(step), int(seed), _ptr(im),
                                        int(im.stride(0)), _ptr(ref), _ptr(work), nw.value,
                                        _stream(stream)), "wfs_calibrate")
        return im, ref

    def tune(self, layers, iters=20, stream=None):
        """Time the launch schedules on ``layers`` and keep the fastest; returns its us/call."""
        self._layers(layers)
        best = ctypes.c_double()
        L.check(self._lib.wfs_plan_tune(self._h, _ptr(layers), int(iters), ctypes.byref(best),
                                        _stream(stream)), "wfs_plan_tune")
        return best.value


def recon_apply(R, S, C=None, alpha=1.0, beta=0.0, ldc=None, stream=None, noalloc=False):
    """C[b] = alpha R S[b] + beta C[b]; R [M][N], S [B][N]; C [B][ldc] (default ldc = M).
    ``noalloc``: call ``recon_apply_noalloc`` (partial sums in the library's fixed array; the
    caller then passes C, since allocating it here would defeat the purpose)."""
    _need(R, "R")
    _need(S, "S")
    if R.dim() != 2 or S.dim() != 2 or S.shape[1] != R.shape[1]:
        raise ValueError(f"R {tuple(R.shape)} and S {tuple(S.shape)} do not match")
    M, N = R.shape
    B = S.shape[0]
    if C is None:
        if noalloc:
            raise ValueError("recon_apply(noalloc=True) needs the output C")
        C = torch.zeros(B, M, device=R.device)
        ldc = M
    if not isinstance(C, torch.Tensor) or C.dtype != torch.float32 or not C.is_cuda:
        raise TypeError("C must be a float32 GPU tensor")
    if C.dim() != 2 or C.shape[0] != B or C.shape[1] < M or C.stride(1) != 1:
        raise ValueError(f"C {tuple(C.shape)} must be [B][>= M] with unit column stride")
    if ldc is None:
        ldc = C.stride(0)
    if C.stride(0) != ldc or ldc < M:
        raise ValueError(f"C row stride {C.stride(0)} must equal ldc={ldc} >= M={M}")
    fn = "recon_apply_noalloc" if noalloc else "recon_apply"
    L.check(getattr(L.lib(), fn)(_ptr(R), int(M), int(N), _ptr(S), int(B), _ptr(C), int(ldc),
                                 float(alpha), float(beta), _stream(stream)), fn)
    return C


def tlse(im, eps=1e-3, weights=None, out=None, stream=None):
    """Control matrix R [m][n_s] = (D^T D + eps mean(diag D^T D) diag(w))^-1 D^T of the
    interaction matrix im [m][n_s] (row j = slopes of actuator j), ``wfs_tlse``.  ``out`` may
    be ``im`` itself (computed in place).  Synchronises the stream."""
    _need(im, "im")
    if im.dim() != 2:
        raise ValueError(f"im must be [m][n_s] (got {tuple(im.shape)})")
    m, n_s = im.shape
    if weights is not None:
        _need(weights, "weights", numel=m)
    if out is None:
        out = torch.empty(m, n_s, device=im.device)
    _need(out, "out", shape=(m, n_s))
    work = torch.empty(m * m + 64, device=im.device)
    L.check(L.lib_tlse().wfs_tlse(_ptr(im), int(m), int(n_s), int(n_s), float(eps),
                                  _ptr(weights), _ptr(out), int(n_s), _ptr(work), work.numel(),
                                  _stream(stream)), "wfs_tlse")
    return out


class WFSFunction(torch.autograd.Function):
    """slopes = WFS(layers); backward runs wfs_adjoint (the noise-free model's adjoint, with the
    subaperture fields recomputed from the layers)."""

    @staticmethod
    def forward(ctx, layers, plan, step, seed):
        slopes, aux = plan.forward(layers, step=step, seed=seed)
        ctx.plan = plan
        ctx.step = step
        noisy = any(s["photons"] > 0 for s in plan.cfg["sensors"])
        ctx.save_for_backward(layers, slopes, aux)
        ctx.noisy = noisy
        return slopes

    @staticmethod
    def backward(ctx, grad_slopes):
        layers, slopes, aux = ctx.saved_tensors
        g = grad_slopes.contiguous()
        if ctx.noisy:  # the forward outputs carry noise: recompute the noise-free ones
            out = ctx.plan.adjoint(layers, g, step=ctx.step)
        else:
            out = ctx.plan.adjoint(layers, g, step=ctx.step, fwd_slopes=slopes, fwd_aux=aux)
        return out, None, None, None


def wfs_slopes(layers, plan, step=0, seed=42):
    """Differentiable slopes of ``plan`` for ``layers`` ([B][layer_stride] float32)."""
    return WFSFunction.apply(layers, plan, step, seed)
