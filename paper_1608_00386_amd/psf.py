"""Python front end of the PSF / Strehl module and the phase-screen generator of libwfs
(``psf_*``, ``screen_generate`` in include/wfs.h).  Argument marshalling only: the
projection, fields, noise, filters, FFTs and sums run in the HIP kernels."""

import ctypes

import torch

from . import _lib as L
from .wfs import _need, _ptr, _stream


class PsfPlan:
    """Long-exposure PSFs of test stars (Sec. 2.8).  ``cfg`` supplies ``layers``,
    ``layer_stride``, ``lambda_ref_m`` and ``dt_s`` (as for ``Plan``); ``stars`` is a list of
    (theta_x, theta_y) in radians; ``lambdas`` the wavelengths (m) and ``n_fft`` the padded
    transform size per wavelength (PSF pixel = lambda / (n_fft * pupil_d / n_pup))."""

    def __init__(self, cfg, stars, pupil_d_m, obs_d_m, n_pup, lambdas, n_fft):
        self._lib = L.lib()
        self.cfg = cfg
        self.stars = [(float(a), float(b)) for a, b in stars]
        self.lambdas = [float(x) for x in lambdas]
        self.n_fft = [int(x) for x in n_fft]
        if len(self.lambdas) != len(self.n_fft):
            raise ValueError("one n_fft per wavelength")
        self.layer_stride = int(cfg["layer_stride"])
        nl, ns, nw = len(cfg["layers"]), len(self.stars), len(self.lambdas)
        self._ld = (L.LayerDesc * nl)(*[L.layer_desc(x) for x in cfg["layers"]])
        th = (ctypes.c_double * (2 * ns))(*[v for st in self.stars for v in st])
        lam = (ctypes.c_double * nw)(*self.lambdas)
        nf = (ctypes.c_int32 * nw)(*self.n_fft)
        h = ctypes.c_void_p()
        L.check(self._lib.psf_plan(self._ld, nl, self.layer_stride, th, ns, float(pupil_d_m),
                                   float(obs_d_m), int(n_pup), lam, nf, nw,
                                   float(cfg["lambda_ref_m"]), float(cfg["dt_s"]),
                                   ctypes.byref(h)), "psf_plan")
        self._h = h
        fl, lit = ctypes.c_int64(), ctypes.c_int64()
        offs = (ctypes.c_int64 * nw)()
        L.check(self._lib.psf_plan_info(h, ctypes.byref(fl), offs, ctypes.byref(lit)),
                "psf_plan_info")
        self.psf_floats = fl.value
        self.offsets = list(offs)
        self.n_lit = lit.value
        self.n_pup = int(n_pup)
        self.device = torch.cuda.current_device()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.check(self._lib.psf_plan_destroy(self._h), "psf_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def buffers(self):
        """Zeroed long-exposure buffers: (psf [psf_floats] float32, phase_var [n_lambda *
        n_stars] float64)."""
        dev = torch.device("cuda", self.device)
        return (torch.zeros(self.psf_floats, device=dev),
                torch.zeros(len(self.lambdas) * len(self.stars), dtype=torch.float64,
                            device=dev))

    def image(self, psf, lam_index, star):
        """View of one long-exposure image [n_fft][n_fft] inside the PSF buffer."""
        N = self.n_fft[lam_index]
        o = self.offsets[lam_index] + star * N * N
        return psf[o:o + N * N].view(N, N)

    def accumulate(self, layers, step, psf, phase_var=None, stream=None):
        """Add one frame of every (wavelength, star) to ``psf`` (and ``phase_var``)."""
        _need(layers, "layers", numel=self.layer_stride)
        _need(psf, "psf", numel=self.psf_floats)
        if phase_var is not None:
            if (phase_var.dtype != torch.float64 or not phase_var.is_cuda or
                    phase_var.numel() != len(self.lambdas) * len(self.stars)):
                raise ValueError("phase_var must be a float64 GPU tensor [n_lambda * n_stars]")
        L.check(self._lib.psf_accumulate(self._h, _ptr(layers), int(step), _ptr(psf),
                                         _ptr(phase_var), _stream(stream)), "psf_accumulate")
        return psf, phase_var

    def strehl(self, psf, phase_var, n_frames, stream=None):
        """(sr_psf, sr_marechal), each [n_lambda][n_stars] float32 on the GPU."""
        nw, ns = len(self.lambdas), len(self.stars)
        dev = torch.device("cuda", self.device)
        a = torch.empty(nw, ns, device=dev)
        b = torch.empty(nw, ns, device=dev)
        L.check(self._lib.psf_strehl(self._h, _ptr(psf), _ptr(phase_var), int(n_frames),
                                     _ptr(a) if psf is not None else None,
                                     _ptr(b) if phase_var is not None else None,
                                     _stream(stream)), "psf_strehl")
        return a, b


def screen_generate(n, pitch_m, r0_m, L0_m, seed, stream_id=0, out=None, stream=None):
    """One periodic n x n von Karman phase screen on the GPU (``screen_generate``); returns a
    float32 [n][n] tensor (radians at the wavelength r0 refers to)."""
    n = int(n)
    dev = torch.device("cuda", torch.cuda.current_device())
    if out is None:
        out = torch.empty(n, n, device=dev)
    _need(out, "out", numel=n * n)
    work = torch.empty(2 * n * n, device=dev)
    L.check(L.lib().screen_generate(n, float(pitch_m), float(r0_m), float(L0_m), int(seed),
                                    int(stream_id), _ptr(out), _ptr(work), work.numel(),
                                    _stream(stream)), "screen_generate")
    return out
