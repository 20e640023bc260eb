"""Host-side checks of the C ABI that need no GPU: the library loads, exports every function
declared in include/wfs.h, and rejects bad arguments before touching the device."""

import ctypes
import math
import os
import re

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wfs.h")
TLSE_HEADER = os.path.join(ROOT, "include", "wfs_tlse.h")


def _declared_functions(header=HEADER):
    txt = open(header).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_path_entry_points():
    names = _declared_functions()
    for n in ("wfs_plan", "wfs_forward", "wfs_adjoint", "recon_apply", "wfs_plan_destroy",
              "wfs_plan_info", "wfs_last_error", "wfs_project", "wfs_spots"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1608_00386_amd import _lib
    L = _lib.lib()
    for n in _declared_functions():
        assert hasattr(L, n), n
    # the ctypes prototypes cover the whole header
    assert set(_declared_functions()) == set(_lib._PROTOS)
    T = _lib.lib_tlse()
    assert _declared_functions(TLSE_HEADER) == ["wfs_tlse"]
    for n in _declared_functions(TLSE_HEADER):
        assert hasattr(T, n), n
    assert set(_declared_functions(TLSE_HEADER)) == set(_lib._TLSE_PROTOS)


def test_hot_path_library_needs_no_dense_algebra_library():
    """libwfs.so (the per-frame path) does not link rocBLAS or rocSOLVER; only the control-matrix
    library does, and it finds libwfs.so beside itself."""
    import shutil
    import subprocess
    from paper_1608_00386_amd import _lib
    readelf = shutil.which("readelf")
    if readelf is None:
        pytest.skip("no readelf")

    def needed(path):
        out = subprocess.run([readelf, "-d", path], capture_output=True, text=True,
                             check=True).stdout
        return re.findall(r"\(NEEDED\)\s+Shared library: \[([^\]]+)\]", out), out
    libs, _ = needed(_lib.LIB_PATH)
    assert libs and not any("rocblas" in n or "rocsolver" in n for n in libs), libs
    libs, out = needed(_lib.TLSE_LIB_PATH)
    assert "libwfs.so" in libs and any("rocblas" in n for n in libs), libs
    assert "$ORIGIN" in out


def test_struct_layouts_match_header_sizes(tmp_path):
    """The ctypes descriptors have the C compiler's size and field offsets for include/wfs.h."""
    import shutil
    import subprocess
    from paper_1608_00386_amd import _lib
    # int64 + 2*int32 + 4*double + float + int32 = 56 bytes
    assert ctypes.sizeof(_lib.LayerDesc) == 56
    # 6 doubles + 4 int32 + 8 doubles = 128 bytes
    assert ctypes.sizeof(_lib.SensorDesc) == 128
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = []
    for ct, cname in ((_lib.LayerDesc, "wfs_layer_desc"), (_lib.SensorDesc, "wfs_sensor_desc")):
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in ct._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"wfs.h\"\n"
                   "int main(void) {\n" + "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                   text=True).stdout.splitlines())
    for ct, cname in ((_lib.LayerDesc, "wfs_layer_desc"), (_lib.SensorDesc, "wfs_sensor_desc")):
        assert int(got[cname]) == ctypes.sizeof(ct), cname
        for f, _ in ct._fields_:
            assert int(got[f"{cname}.{f}"]) == getattr(ct, f).offset, (cname, f)


def _plan_rc(cfg, batch=1, flags=0, mutate=None):
    from paper_1608_00386_amd import _lib
    L = _lib.lib()
    layers = [dict(x) for x in cfg["layers"]]
    sensors = [dict(x) for x in cfg["sensors"]]
    stride = cfg["layer_stride"]
    lam = cfg["lambda_ref_m"]
    if mutate:
        stride, lam = mutate(layers, sensors, stride, lam)
    ld = (_lib.LayerDesc * len(layers))(*[_lib.layer_desc(x) for x in layers])
    sd = (_lib.SensorDesc * len(sensors))(*[_lib.sensor_desc(x) for x in sensors])
    h = ctypes.c_void_p()
    rc = L.wfs_plan(ld, len(layers), stride, sd, len(sensors), batch, lam, cfg["dt_s"], flags,
                    ctypes.byref(h))
    return rc, L.wfs_last_error().decode()


def _set(which, key, value):
    def m(layers, sensors, stride, lam):
        (layers if which == "layer" else sensors)[0][key] = value
        return stride, lam
    return m


@pytest.mark.parametrize("mutate,needle", [
    (_set("sensor", "n_fft", 30), "multiple of bin"),
    (_set("sensor", "n_fft", 16), "2*n_sub"),
    (_set("sensor", "n_fft", 33), "even"),
    (_set("sensor", "bin", 0), "bin=0"),
    (_set("sensor", "obs_d_m", 40.0), "obstruction"),
    (_set("sensor", "valid_frac", 0.0), "valid_frac"),
    (_set("sensor", "src_alt_m", 10e3), "LGS altitude"),
    (_set("sensor", "tilt_y_rad", math.inf), "tip-tilt"),
    (_set("layer", "boundary", 3), "boundary"),
    (_set("layer", "pitch_m", 0.0), "geometry"),
    (_set("layer", "nx", 1), "grid"),
    (lambda l, s, st, lam: (l[0].update(nx=1 << 15, ny=1 << 15) or 1 << 31, lam), "2^29"),
    (lambda l, s, st, lam: (100, lam), "outside the stride"),
    (lambda l, s, st, lam: (st, -1.0), "lambda_ref"),
])
def test_plan_rejects_bad_descriptors_on_the_host(mutate, needle):
    rc, msg = _plan_rc(synth.config1(), mutate=mutate)
    assert rc == -1, msg
    assert needle in msg


def test_plan_rejects_conflicting_flags_and_bad_batch():
    from paper_1608_00386_amd import _lib
    rc, msg = _plan_rc(synth.config0(), flags=_lib.WFS_FLAG_FORCE_FFT | _lib.WFS_FLAG_FORCE_OTF)
    assert rc == -1 and "FORCE" in msg
    rc, msg = _plan_rc(synth.config0(), batch=0)
    assert rc == -1 and "batch" in msg


def test_calls_reject_null_handles_without_a_device():
    from paper_1608_00386_amd import _lib
    L = _lib.lib()
    assert L.wfs_forward(None, None, 0, 0, None, None, None) == -1
    assert L.wfs_adjoint(None, None, None, None, None, 0, None, None) == -1
    assert L.wfs_plan_destroy(None) == -1
    assert L.wfs_spots(None, None, 0, 0, None, None, None) == -1
    assert L.wfs_plan_schedule(None, None, None, None, None, None, None) == -1
    assert L.wfs_plan_set_schedule(None, -1, -1, -1, -1, -1, -1) == -1
    assert L.wfs_plan_footprint(None, 0, None, None) == -1
    assert L.recon_apply(None, 1, 1, None, 1, None, 1, 1.0, 0.0, None) == -1
    assert "null" in L.wfs_last_error().decode()
    assert L.wfs_plan_na_profile(None, 1, 1, None) == -1
    assert "null plan" in L.wfs_last_error().decode()


def test_na_profile_table_pads_entries_with_zero_weight_peaks():
    from paper_1608_00386_amd import _lib
    n_e, n_p, tab = _lib.na_profile_table([[(100.0, 2e3, 1.0)], [(0.0, 1e3, 2.0), (5e3, 0.0, 1.0)]])
    assert (n_e, n_p) == (2, 2)
    assert list(tab) == [100.0, 2e3, 1.0, 0.0, 0.0, 0.0, 0.0, 1e3, 2.0, 5e3, 0.0, 1.0]


def test_recon_rejects_bad_shapes_without_a_device():
    from paper_1608_00386_amd import _lib
    L = _lib.lib()
    fake = ctypes.c_void_p(4096)  # never dereferenced: validation fails first
    assert L.recon_apply(fake, 0, 4, fake, 1, fake, 4, 1.0, 0.0, None) == -1
    assert L.recon_apply(fake, 8, 4, fake, 1, fake, 4, 1.0, 0.0, None) == -1
    assert "ldc" in L.wfs_last_error().decode()
    assert L.recon_apply(fake, 8, 4, fake, 1, fake, 8, math.nan, 0.0, None) == -1


def test_calibration_calls_reject_bad_arguments_without_a_device():
    from paper_1608_00386_amd import _lib
    L = _lib.lib()
    fake = ctypes.c_void_p(4096)  # never dereferenced: validation fails first
    n = ctypes.c_int64()
    assert L.wfs_calibrate_work(None, ctypes.byref(n)) == -1
    assert L.wfs_calibrate(None, None, 0, 1, 0.1, 0, 42, fake, 8, None, fake, 1 << 20,
                           None) == -1
    assert "null plan" in L.wfs_last_error().decode()
    # wfs_tlse: shapes, leading dimensions, eps, workspace, in-place stride
    T = _lib.lib_tlse()
    assert T.wfs_tlse(None, 4, 8, 8, 0.1, None, fake, 8, fake, 100, None) == -1
    assert T.wfs_tlse(fake, 0, 8, 8, 0.1, None, fake, 8, fake, 100, None) == -1
    assert T.wfs_tlse(fake, 4, 8, 7, 0.1, None, fake, 8, fake, 100, None) == -1
    assert "ld_im" in L.wfs_last_error().decode()
    assert T.wfs_tlse(fake, 4, 8, 8, -1.0, None, fake, 8, fake, 100, None) == -1
    assert T.wfs_tlse(fake, 4, 8, 8, math.nan, None, fake, 8, fake, 100, None) == -1
    assert T.wfs_tlse(fake, 4, 8, 8, 0.1, None, fake, 8, fake, 79, None) == -1
    assert "work" in L.wfs_last_error().decode()
    assert T.wfs_tlse(fake, 4, 8, 8, 0.1, None, ctypes.c_void_p(4096), 9, fake, 100,
                      None) == -1
    assert "in place" in L.wfs_last_error().decode()


def test_dm_calibration_config_keeps_actuator_order():
    from paper_1608_00386_amd import calib
    cfg = synth.config4(batch=1)
    ccfg, n_act = calib.dm_config(cfg, batch=64)
    assert n_act == 40 * 40 + 42 * 42 + 45 * 45 == 5389
    assert [L["offset"] for L in ccfg["layers"]] == [0, 1600, 1600 + 1764]
    assert all(L["weight"] < 0 and L["boundary"] == 1 for L in ccfg["layers"])
    assert ccfg["layer_stride"] % 64 == 0 and ccfg["layer_stride"] >= n_act
    assert all(s["photons"] == 0 and s["read_noise_e"] == 0 for s in ccfg["sensors"])
    assert any(s["photons"] > 0 for s in cfg["sensors"])  # the original is left alone
    with pytest.raises(ValueError):
        calib.dm_config(cfg, batch=3)


def test_psf_and_screen_calls_reject_bad_arguments_without_a_device():
    from paper_1608_00386_amd import _lib
    L = _lib.lib()
    c = ctypes
    fake = c.c_void_p(4096)
    ld = (_lib.LayerDesc * 1)(_lib.layer_desc(dict(offset=0, nx=64, ny=64, pitch_m=0.25,
                                                   alt_m=0.0, vx_mps=0.0, vy_mps=0.0,
                                                   weight=1.0, boundary=0)))
    th = (c.c_double * 2)(0.0, 0.0)
    lam = (c.c_double * 1)(1e-6)
    h = c.c_void_p()

    def plan(n_pup=32, nfft=64, stride=4096, D=8.0, obs=1.0, n_stars=1):
        nf = (c.c_int32 * 1)(nfft)
        return L.psf_plan(ld, 1, stride, th, n_stars, D, obs, n_pup, lam, nf, 1, 0.5e-6, 0.002,
                          c.byref(h))

    assert plan(nfft=48) == -1           # not a power of two
    assert "power of two" in L.wfs_last_error().decode()
    assert plan(nfft=16, n_pup=32) == -1  # smaller than the pupil
    assert plan(nfft=8192) == -1
    assert plan(stride=100) == -1         # layer outside the stride
    assert plan(obs=9.0) == -1            # obstruction wider than the pupil
    assert plan(n_stars=0) == -1
    assert L.psf_accumulate(None, fake, 0, fake, None, None) == -1
    assert L.psf_strehl(None, fake, None, 1, fake, None, None) == -1
    assert L.psf_plan_destroy(None) == -1
    W = 2 * 64 * 64
    assert L.screen_generate(48, 0.1, 0.1, 25.0, 1, 0, fake, fake, W, None) == -1
    assert L.screen_generate(64, 0.1, 0.1, 25.0, 1, 0, fake, fake, W - 1, None) == -1
    assert "work" in L.wfs_last_error().decode()
    assert L.screen_generate(64, -0.1, 0.1, 25.0, 1, 0, fake, fake, W, None) == -1
    assert L.screen_generate(64, 0.1, 0.1, 25.0, 1, 0, None, fake, W, None) == -1
