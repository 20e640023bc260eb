"""Build libwfs.so (the HIP kernels and the C ABI) in-tree for gfx950.

    python -m paper_1608_00386_amd.build          # or __graft_entry__.build()
"""

import concurrent.futures
import glob
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwfs.so")
# the control-matrix solve (rocBLAS / rocSOLVER) is a library of its own, beside libwfs.so
TLSE_SRC = "tlse.hip"
TLSE_LIB = os.path.join(HERE, "libwfs_tlse.so")
ARCH = os.environ.get("WFS_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 (v_pk_*_f32) stays off: the compiler emits plain VALU FP32 instead
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # floating-point atomics as hardware atomics (the adjoint's layer scatter)
    "-munsafe-fp-atomics",
    "-Wall",
    "-Wno-unused-result",
]


def hipcc():
    for c in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libwfs.so)")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = r.stdout + r.stderr
    # the host pass does not know the device target feature: drop that one harmless warning
    lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l or "error" in l]
    return r.returncode, lines


def build(verbose=False, extra=()):
    """Compile every csrc/*.hip unit to an object (in parallel), then link libwfs.so (all but
    tlse.hip) and libwfs_tlse.so (tlse.hip, rocBLAS, rocSOLVER and libwfs.so)."""
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with tempfile.TemporaryDirectory(prefix="wfs_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(s)[:-4] + ".o") for s in srcs]
        cmds = [[hipcc()] + FLAGS + list(extra) + ["-c", s, "-o", o] for s, o in zip(srcs, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(_run, cmds))
        msgs = [l for _, lines in results for l in lines]
        if any(rc != 0 for rc, _ in results):
            raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
        tlse_obj = [o for s, o in zip(srcs, objs) if os.path.basename(s) == TLSE_SRC]
        wfs_objs = [o for o in objs if o not in tlse_obj]
        tmp = LIB + ".tmp"
        link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC"] + wfs_objs + ["-o", tmp]
        rc, lines = _run(link)
        if rc != 0:
            raise RuntimeError("link failed:\n" + "\n".join(lines))
        os.replace(tmp, LIB)
        # rocBLAS / rocSOLVER: the one-off dense algebra of the control matrix (wfs_tlse);
        # libwfs.so found beside it at load time
        rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
        tmp2 = TLSE_LIB + ".tmp"
        link2 = ([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC"] + tlse_obj +
                 [f"-L{HERE}", "-lwfs", "-Wl,-rpath,$ORIGIN", f"-L{rocm_lib}", "-lrocsolver",
                  "-lrocblas", "-o", tmp2])
        rc, lines2 = _run(link2)
        if rc != 0:
            raise RuntimeError("link failed:\n" + "\n".join(lines2))
        os.replace(tmp2, TLSE_LIB)
        if verbose and msgs + lines + lines2:
            print("\n".join(msgs + lines + lines2))
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
