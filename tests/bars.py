"""Image bars of the GPU ADMM parity tests that cannot use the 1e-4 NRMSE bar,
each derived from the oracle's own sensitivity.

tests/golden/make_tolerances.py runs the FP64 oracle's ADMM with every F and
F^H output perturbed by a relative L2 error eps (fresh complex Gaussian
direction per call, several seeds) or rounded to complex64, and stores how far
the image moves (tolerances.json).  The shift grows linearly with eps, so a
GPU form whose operators carry error eps is expected to land that far from the
oracle through rounding order alone; its bar is twice the largest shift
measured at its operator-error level.  For the three large problems whose
oracle reconstructions are stored beside the tolerances (the 256x256
benchmark at 30 x 5, slice 0 of the 32 x 384^2 batch at 2 x 2, the 1024x512
Table I problem at 1 x 2) the stored reconstruction is the exact image and
only the BF16x3 operator error is measured.  test_tolerances.py re-derives
some of the stored shifts on the CPU.
"""
import json
import os

_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tolerances.json")
with open(_PATH) as _f:
    SENSITIVITY = json.load(_f)

MARGIN = 2.0


def _max_shift(case, eps_keys):
    c = SENSITIVITY[case]
    vals = [c["c64"]] + [v for k in eps_keys for v in c["noise"][k]]
    return max(vals)


# The 32x32 / 4-coil / 16x64 workload at 10 ADMM x 3 CG in BF16x3, whose
# operators carry ~4e-6 relative error (16-bit split operands).
BF16X3_ADMM32 = MARGIN * _max_shift("admm32", ["4e-06"])
# The 128x64 / 12-coil / 13x128 Table I problem (lambda 1e-7, up to 5 ADMM x
# 20 CG) in the forms whose operators carry 1e-7 .. 1e-6 relative error (FP32,
# FP16x3): the almost unregularised least-squares solve moves by several 1e-3.
TABLE1_128x64 = MARGIN * _max_shift("table1_128x64", ["1e-07", "1e-06"])


def _stored_max(case):
    """Largest shift of a case measured against a stored oracle reconstruction."""
    return max(v for vals in SENSITIVITY[case]["noise"].values() for v in vals)


# BF16x3 (operator error ~4e-6) on the large problems: the benchmark solve
# (150 CG steps amplify the error most), slice 0 of the 384^2 batch and the
# 1024x512 Table I problem, the last two at the reduced counts of their stored
# oracle reconstructions.
BF16X3_ADMM256 = MARGIN * _stored_max("admm256_bf16x3")
BF16X3_SLICES384 = MARGIN * _stored_max("slices384_bf16x3")
BF16X3_TABLE1_LARGE = MARGIN * _stored_max("table1_large_bf16x3")
