"""Conjugate gradient and ADMM for the CS-MRI problem, FP64 (test oracle only).

Problem, eq. (3):   min_rho ||F(rho) - d||_2^2 + lam ||Theta(rho)||_1.
ADMM in scaled form, updates in the paper's order mu -> rho -> eta:
    eq. (9):  mu'   = S_{lam/beta}(Theta rho + eta)
    eq. (11): A rho' = b with, eq. (12), A = F^H F + (beta/2) Theta^H Theta
                      and, eq. (13), b = F^H d + (beta/2) Theta^H (mu' - eta)
    eq. (8):  eta'  = eta + Theta rho' - mu'
The rho-update is solved by conjugate gradient (Alg. 2); Alg. 4 drives the
loop and stops on an iteration cap or on the relative image change.

Readings where the paper is silent or inconsistent (the GPU path takes the
same ones):
  * CG starts from r = b - A x0 (Alg. 2 forms the residual without b);
  * CG rebinds r, d, x, tau each step and stops when tau <= atol^2 or after
    max_iterations steps; it also stops when d^H A d <= 0 (breakdown guard);
    tau = r^H r is real, alpha = tau / Re(d^H A d);
  * the dual update uses the new image rho^{m+1}, as eq. (8) states
    (Alg. 4 passes the old one);
  * CG is warm-started from the current image rho^m (flag ``warm``); with
    warm=False it restarts from the initial image every ADMM iteration, the
    literal reading of Alg. 4;
  * initial image = x0 or zeros, eta = 0, F^H d computed once;
  * alpha = ||rho^{m+1} - rho^m||^2 / ||rho^m||^2, checked after the dual
    update; with ||rho^m|| = 0 it is 1 if the image changed and 0 otherwise;
    ADMM continues while iterations remain and alpha > rtol^2.
"""
import dataclasses

import numpy as np

from . import nudft, tv


def normal_op(v, smaps, traj, beta):
    """A v = F^H F v + (beta/2) Theta^H Theta v, eq. (12)."""
    fhf = nudft.adjoint(nudft.forward(v, smaps, traj), smaps, traj)
    return fhf + 0.5 * beta * tv.tv_adjoint(tv.tv_forward(v))


def _dot(a, b):
    """a^H b over all elements, complex128."""
    return np.vdot(np.asarray(a).ravel(), np.asarray(b).ravel())


def conjugate_gradient(apply_a, b, x0, max_iterations, atol):
    """Alg. 2: solve A x = b from x0; returns (x, steps_taken, final tau)."""
    x = np.array(x0, dtype=np.complex128, copy=True)
    r = np.asarray(b, dtype=np.complex128) - apply_a(x)
    d = r.copy()
    tau = _dot(r, r).real
    steps = 0
    while steps < max_iterations and tau > atol * atol:
        a_d = apply_a(d)
        curv = _dot(d, a_d).real
        if not curv > 0.0:
            break
        alpha = tau / curv
        x = x + alpha * d
        r = r - alpha * a_d
        tau_next = _dot(r, r).real
        d = r + (tau_next / tau) * d
        tau = tau_next
        steps += 1
    return x, steps, tau


@dataclasses.dataclass
class AdmmResult:
    image: np.ndarray
    admm_iters: int
    cg_steps: int
    alpha: float
    tau: float
    history: list   # image after every ADMM iteration


def admm(data, smaps, traj, lam, beta, admm_iters, cg_iters, rtol=0.0, atol=0.0,
         x0=None, warm=True, apply_a=None, adjoint=None):
    """Alg. 4 with the readings in the module docstring.

    ``apply_a`` / ``adjoint`` default to the NUDFT normal operator and F^H of
    this package; the tests substitute dense matrices on tiny problems.
    """
    smaps = np.asarray(smaps)
    ny, nx = smaps.shape[1:]
    if apply_a is None:
        def apply_a(v):
            return normal_op(v, smaps, traj, beta)
    if adjoint is None:
        def adjoint(u):
            return nudft.adjoint(u, smaps, traj)
    fhd = adjoint(data)                                    # F^H d, once
    rho0 = np.zeros((ny, nx), np.complex128) if x0 is None else np.asarray(x0, np.complex128)
    rho = rho0.copy()
    eta = np.zeros((2, ny, nx), np.complex128)
    alpha = 1.0
    tau = 0.0
    m = 0
    cg_total = 0
    history = []
    while m < admm_iters and alpha > rtol * rtol:
        mu = tv.soft_threshold(tv.tv_forward(rho) + eta, lam / beta)        # eq. (9)
        b = fhd + 0.5 * beta * tv.tv_adjoint(mu - eta)                      # eq. (13)
        start = rho if warm else rho0
        rho_next, steps, tau = conjugate_gradient(apply_a, b, start, cg_iters, atol)
        cg_total += steps
        num = np.sum(np.abs(rho_next - rho) ** 2)
        den = np.sum(np.abs(rho) ** 2)
        if den > 0.0:
            alpha = num / den
        else:
            alpha = 1.0 if num > 0.0 else 0.0
        eta = eta + tv.tv_forward(rho_next) - mu                              # eq. (8)
        rho = rho_next
        history.append(rho.copy())
        m += 1
    return AdmmResult(rho, m, cg_total, float(alpha), float(tau), history)


def objective(image, data, smaps, traj, lam):
    """Eq. (3): ||F(image) - d||^2 + lam * sum |Theta(image)|."""
    resid = nudft.forward(image, smaps, traj) - np.asarray(data, np.complex128)
    return float(np.sum(np.abs(resid) ** 2) + lam * np.sum(np.abs(tv.tv_forward(image))))
