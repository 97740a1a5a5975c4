"""Multi-coil non-uniform DFT and its adjoint, FP64 (test oracle only).

Forward model, eq. (1)-(2): d[g, k] = sum_n s[g, n] rho[n] exp(-i 2 pi k_k . r_n).

Readings of the paper used here:
  * the trajectory is given as omega = 2 pi k in radians per pixel, and r_n
    are integer pixel offsets, so the phase is omega . r (the paper does not
    state units);
  * the image grid is centred: r = index - n//2 on each axis;
  * column 0 of the trajectory pairs with x (the fast image axis), column 1
    with y, as the first image coordinate pairs with the first k column in
    Alg. 1;
  * F carries no normalisation and no density compensation;
  * the paper's "inverse DFT" inside the CG operator (Alg. 3) is the adjoint
    F^H, conjugate coil combine included, since the normal matrix of eq. (12)
    needs F^H F.

The phase matrix is built per axis and combined by an outer product, as Alg. 1
builds its DFT operator: exp(-i(wx x + wy y)) = exp(-i wx x) exp(-i wy y).
"""
import numpy as np


def grid_coords(n):
    """Centred integer pixel offsets 0 - n//2 ... n-1 - n//2, float64."""
    return np.arange(n, dtype=np.float64) - (n // 2)


def phase_matrix(omega, n):
    """exp(-i omega_k r_j) for every sample k and pixel offset j: [nk, n].

    Alg. 1: map_to_unit_circle applied to the product of k and r on one axis.
    """
    omega = np.asarray(omega, dtype=np.float64)
    return np.exp(-1j * np.outer(omega, grid_coords(n)))


def forward(image, smaps, traj):
    """y = F(image), eq. (1): image [ny, nx], smaps [nc, ny, nx], traj [nk, 2]
    -> data [nc, nk], complex128.

    d[g, k] = sum_{i, j} Ey[k, i] Ex[k, j] s[g, i, j] image[i, j]
    with Ex = phase_matrix(traj[:, 0], nx), Ey = phase_matrix(traj[:, 1], ny).
    """
    image = np.asarray(image, dtype=np.complex128)
    smaps = np.asarray(smaps, dtype=np.complex128)
    traj = np.asarray(traj, dtype=np.float64)
    nc, ny, nx = smaps.shape
    ex = phase_matrix(traj[:, 0], nx)
    ey = phase_matrix(traj[:, 1], ny)
    out = np.empty((nc, traj.shape[0]), dtype=np.complex128)
    for g in range(nc):
        weighted = smaps[g] * image                 # s_g (.) rho
        t = ex @ weighted.T                         # [nk, ny]: sum over x
        out[g] = np.sum(t * ey, axis=1)             # sum over y
    return out


def adjoint(data, smaps, traj):
    """x = F^H(data): data [nc, nk] -> image [ny, nx], complex128.

    x[i, j] = sum_g conj(s[g, i, j]) sum_k conj(Ey[k, i] Ex[k, j]) data[g, k].
    """
    data = np.asarray(data, dtype=np.complex128)
    smaps = np.asarray(smaps, dtype=np.complex128)
    traj = np.asarray(traj, dtype=np.float64)
    nc, ny, nx = smaps.shape
    ex = phase_matrix(traj[:, 0], nx)
    ey = phase_matrix(traj[:, 1], ny)
    out = np.zeros((ny, nx), dtype=np.complex128)
    for g in range(nc):
        w = np.conj(ey) * data[g][:, None]          # [nk, ny]
        xg = w.T @ np.conj(ex)                      # [ny, nx]: sum over k
        out += np.conj(smaps[g]) * xg
    return out


def forward_samples(image, smaps, traj, coils, samples):
    """F(image)[coils[t], samples[t]] for a list of (coil, sample) pairs.

    Each value is the full pixel sum of eq. (1) for one output, so sampled
    outputs of a large problem can be checked one by one.
    """
    image = np.asarray(image, dtype=np.complex128)
    smaps = np.asarray(smaps, dtype=np.complex128)
    traj = np.asarray(traj, dtype=np.float64)
    _, ny, nx = smaps.shape
    out = np.empty(len(samples), dtype=np.complex128)
    for t, (g, k) in enumerate(zip(coils, samples)):
        ex = np.exp(-1j * traj[k, 0] * grid_coords(nx))
        ey = np.exp(-1j * traj[k, 1] * grid_coords(ny))
        out[t] = ey @ (smaps[g] * image) @ ex
    return out


def adjoint_pixels(data, smaps, traj, rows, cols):
    """F^H(data)[rows[t], cols[t]] for a list of pixels (full sample sums)."""
    data = np.asarray(data, dtype=np.complex128)
    smaps = np.asarray(smaps, dtype=np.complex128)
    traj = np.asarray(traj, dtype=np.float64)
    _, ny, nx = smaps.shape
    yc = grid_coords(ny)
    xc = grid_coords(nx)
    out = np.empty(len(rows), dtype=np.complex128)
    for t, (i, j) in enumerate(zip(rows, cols)):
        ph = np.exp(1j * (traj[:, 0] * xc[j] + traj[:, 1] * yc[i]))   # conj of the forward phase
        out[t] = np.sum(np.conj(smaps[:, i, j]) * (data @ ph))
    return out
