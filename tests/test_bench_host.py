"""Host-side checks of the benchmark's contract and of its roofline
accounting (CPU only: no kernel runs).

The algorithmic bytes that the roofline divides by are pinned here by an
independent tally of the buffers each pass of the paper-scale step must move
(N = 65536, 256 signals in 128 pairs, L = 131072, rank 32, rows of 4096 so
L1 = 32 and 256 column blocks of 16 columns): FP32 signals 4 B per sample,
the pair-packed complex64 intermediate 8 B per point, U once (FP32), the
kernel spectrum once (FP32, L values), the coefficient partials and d (.) C.
"""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

N, B, L, R, L1 = 65536, 256, 131072, 32, 32
PAIRS = B // 2
X = N * B * 4                 # signals in (or out), FP32
Z = PAIRS * L * 8             # the pair intermediate, complex64
U = N * R * 4                 # transition vectors, FP32
SPEC = L * 4                  # kernel spectrum, FP32
BLOCKS = (L // L1) // 16      # column blocks of pass A (one partial each)
PART = BLOCKS * R * B * 4     # coefficient partials
DC = R * B * 4                # d (.) C


def test_paper_scale_pass_bytes():
    assert bench.kernel_bytes("col_fwd_corr_bf16x3", N, B, L, R, PAIRS, 5) == X + Z + U + PART
    assert bench.kernel_bytes("row_conv", N, B, L, R, PAIRS, 5) == 2 * Z + SPEC
    assert bench.kernel_bytes("col_inv_corr_bf16x3", N, B, L, R, PAIRS, 5) == Z + X + U + DC
    # the plain passes move the same signal and intermediate bytes without U
    assert bench.kernel_bytes("col_fwd", N, B, L, R, PAIRS) == X + Z
    assert bench.kernel_bytes("col_inv", N, B, L, R, PAIRS) == Z + X
    # the separate correction kernels: x (or y twice) and U once
    assert bench.kernel_bytes("corr_partial_bf16x3", N, B, L, R, PAIRS) == X + U
    assert bench.kernel_bytes("corr_apply", N, B, L, R, PAIRS) == 2 * X + U


def test_step_bytes_against_compulsory():
    """The three passes move about 5.2 times the compulsory bytes (x in, y out)."""
    step = sum(bench.kernel_bytes(k, N, B, L, R, PAIRS, 5)
               for k in ("col_fwd_corr_bf16x3", "row_conv", "col_inv_corr_bf16x3"))
    assert 5.1 < step / (2 * X) < 5.3


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
    assert r.stdout == ""
