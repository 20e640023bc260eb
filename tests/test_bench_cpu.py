"""Host-side checks of bench.py: the multi-GPU refusal and the algorithmic FLOP and byte
counts its roofline lines use."""

import math
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_flops_per_lgs_subaperture_follow_the_fft_convention():
    """n = 10 pixels, N = 32, b = 4, with elongation: field 4n^2, zero-padded 2-D FFT
    5 N log2 N (n + N), |F|^2 3 N^2, scale N^2, elongation 2 x 2.5 N^2 log2 N^2 + 10 N (N/2 + 1),
    binning N^2, centroid 4 n_pix^2 + 4 = 96,020."""
    import bench
    n, N, b = 10, 32, 4
    want = (4 * n * n + 5 * N * math.log2(N) * (n + N) + 3 * N * N + N * N
            + 2 * 2.5 * N * N * math.log2(N * N) + 10 * N * (N // 2 + 1) + N * N
            + 4 * (N // b) ** 2 + 4)
    assert want == 96020
    assert bench.flops_per_subap(n, N, b, True) == want
