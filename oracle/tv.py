"""Finite-difference sparsifying transform and soft threshold, FP64 (test oracle only).

Theta is the finite-difference operator the paper uses as sparsifying
transform (Sec. III-A) and implements as 1-D convolutions (Sec. IV-B).  The
paper does not state direction, boundary or stacking; the reading taken here
is forward differences with periodic wrap, stacked x-difference first:

    Theta(v)[0, i, j] = v[i, (j+1) mod nx] - v[i, j]
    Theta(v)[1, i, j] = v[(i+1) mod ny, j] - v[i, j]

and Theta^H is its exact conjugate transpose.

The soft threshold of eq. (10) is written for real arguments; on complex
values it shrinks the magnitude (complex-magnitude shrinkage), which reduces
to eq. (10) on real inputs.  The printed lambda_1 is read as lambda.
"""
import numpy as np


def tv_forward(image):
    """Theta(image): [ny, nx] -> [2, ny, nx] (x-difference, y-difference)."""
    v = np.asarray(image, dtype=np.complex128)
    dx = np.roll(v, -1, axis=1) - v
    dy = np.roll(v, -1, axis=0) - v
    return np.stack([dx, dy])


def tv_adjoint(grad):
    """Theta^H(grad): [2, ny, nx] -> [ny, nx]."""
    g = np.asarray(grad, dtype=np.complex128)
    return (np.roll(g[0], 1, axis=1) - g[0]) + (np.roll(g[1], 1, axis=0) - g[1])


def soft_threshold(z, thr):
    """Element-wise S_thr(z), eq. (10): 0 where |z| <= thr, else z (1 - thr/|z|)."""
    z = np.asarray(z, dtype=np.complex128)
    mag = np.abs(z)
    keep = mag > thr
    scale = np.zeros_like(mag)
    scale[keep] = 1.0 - thr / mag[keep]
    return z * scale
