"""FP64 reference solvers (test infrastructure only).

Plain NumPy versions of the reconstruction routines of Sec. IV: the
objective of eq. "exp_tikh",

    F(u) = 1/2 |s W u - p|^2 + lambda/2 |u|^2,

minimised by conjugate gradients on the normal equations (CGLS) and by
Nesterov's accelerated gradient, and the spectral norm of W by power
iteration (the paper normalises W by it, Sec. IV).  W is any object with
``@`` and ``.T`` (the oracle's scipy CSR matrix); vectors are flat float64
arrays, one problem at a time.  Each function performs the textbook steps in
order, so that a reader can check it line by line against the definitions;
nothing here is shared with the HIP library.
"""
from __future__ import annotations

import numpy as np


def power_norm(W, v0, iters: int) -> float:
    """Power iteration on W^T W from v0: the Rayleigh quotient |W v|^2 of the
    last normalised iterate v is an estimate of ||W||_2^2 from below."""
    v = np.asarray(v0, dtype=np.float64).ravel()
    v = v / np.linalg.norm(v)
    sigma2 = 0.0
    for _ in range(iters):
        u = W @ v
        sigma2 = float(u @ u)
        w = W.T @ u
        v = w / np.linalg.norm(w)
    return float(np.sqrt(sigma2))


def cgls(W, p, x0, iters: int, lam: float = 0.0, s: float = 1.0):
    """Conjugate gradients on (s^2 W^T W + lam I) u = s W^T p.

    Returns the iterate after `iters` steps and the squared norms of the
    normal-equation residual (the gradient of F) before every step and after
    the last one."""
    p = np.asarray(p, dtype=np.float64).ravel()
    x = np.asarray(x0, dtype=np.float64).ravel().copy()
    r = p - s * (W @ x)                 # data residual
    g = s * (W.T @ r) - lam * x         # minus the gradient of F
    d = g.copy()                        # search direction
    gamma = float(g @ g)
    hist = [gamma]
    for _ in range(iters):
        q = s * (W @ d)
        delta = float(q @ q) + lam * float(d @ d)
        alpha = gamma / delta if delta > 0 else 0.0
        x = x + alpha * d
        r = r - alpha * q
        g = s * (W.T @ r) - lam * x
        gamma_new = float(g @ g)
        hist.append(gamma_new)
        beta = gamma_new / gamma if gamma > 0 else 0.0
        gamma = gamma_new
        d = g + beta * d
    return x, np.array(hist)


def nag(W, p, x0, iters: int, norm: float, lam: float = 0.0, s: float = 1.0):
    """Nesterov's accelerated gradient with the FISTA momentum sequence
    t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2 and the fixed step 1/L,
    L = s^2 norm^2 + lam (the Lipschitz constant of grad F).

    Returns u_iters and |grad F(z_k)|^2 at every extrapolated point z_k."""
    p = np.asarray(p, dtype=np.float64).ravel()
    x = np.asarray(x0, dtype=np.float64).ravel().copy()
    L = s * s * norm * norm + lam
    z = x.copy()
    x_prev = x.copy()
    t = 1.0
    hist = []
    for _ in range(iters):
        grad = s * (W.T @ (s * (W @ z) - p)) + lam * z
        hist.append(float(grad @ grad))
        x = z - grad / L
        t_next = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
        z = x + ((t - 1.0) / t_next) * (x - x_prev)
        x_prev = x
        t = t_next
    return x, np.array(hist)


def objective(W, p, u, lam: float = 0.0, s: float = 1.0) -> float:
    r = s * (W @ u) - p
    return 0.5 * float(r @ r) + 0.5 * lam * float(u @ u)
