"""Total variation (Eq. 2) and its prox with non-negativity (Eq. 17).

Finite differences (the paper's Fig. 1 is missing; reading): forward
differences, horizontal h_j^T x = x[iy, ix+1] - x[iy, ix] and vertical
v_j^T x = x[iy+1, ix] - x[iy, ix], each zero on the last column / row.
The divergence is the negative adjoint of that gradient.

The prox (Sec. 2.2: Chambolle's projection algorithm modified for x >= 0) is
computed on the dual: with ``psi(x) = max_{|p_j| <= 1} -<grad x, p>`` the
minimiser of ``lam psi(x) + 1/2 ||x - z||^2`` over x >= 0 is
``x = max(0, z - lam div p)`` for the dual optimum p, and p is found by
projected gradient steps of size tau_c/lam (tau_c = 1/8 is the step 1/L for
the dual's Lipschitz constant 8 lam^2):

    x~ = max(0, z - lam div p)
    p  <- (p - (tau_c/lam) grad x~) / max(1, |p - (tau_c/lam) grad x~|)   pointwise

repeated n_tv times from a warm-started p, then x = max(0, z - lam div p).
"""
import numpy as np


def grad(x):
    """(h, v) forward differences, zero on the last column / row."""
    g1 = np.zeros_like(x)
    g2 = np.zeros_like(x)
    g1[:, :-1] = x[:, 1:] - x[:, :-1]
    g2[:-1, :] = x[1:, :] - x[:-1, :]
    return g1, g2


def div(p1, p2):
    """Negative adjoint of ``grad``: <grad x, p> = -<x, div p>.

    The last column of p1 and the last row of p2 pair with differences that are
    identically zero and so never enter; with that, (div p)[i, j] =
    p1[i, j] - p1[i, j-1] + p2[i, j] - p2[i-1, j] with out-of-range terms zero.
    """
    q1 = p1.copy()
    q1[:, -1] = 0.0
    q2 = p2.copy()
    q2[-1, :] = 0.0
    d = q1 + q2
    d[:, 1:] -= q1[:, :-1]
    d[1:, :] -= q2[:-1, :]
    return d


def tv_norm(x):
    """psi(x) of Eq. 2: sum over pixels of the Euclidean norm of (h_j^T x, v_j^T x)."""
    g1, g2 = grad(np.asarray(x, dtype=np.float64))
    return float(np.sqrt(g1 * g1 + g2 * g2).sum())


def tv_dual_step(z, lam, p1, p2, tau_c=0.125):
    """One projected-gradient step on the dual of the constrained ROF problem."""
    xt = np.maximum(0.0, z - lam * div(p1, p2))
    g1, g2 = grad(xt)
    q1 = p1 - (tau_c / lam) * g1
    q2 = p2 - (tau_c / lam) * g2
    scale = np.maximum(1.0, np.sqrt(q1 * q1 + q2 * q2))
    return q1 / scale, q2 / scale


def tv_prox(z, lam, p1=None, p2=None, n_iter=10, tau_c=0.125):
    """Approximate argmin_{x >= 0} lam psi(x) + 1/2 ||x - z||^2 (Eq. 17).

    Returns (x, p1, p2); p is the warm start for the next call.  lam == 0
    gives the projection max(0, z) (Algorithm 1').
    """
    z = np.asarray(z, dtype=np.float64)
    if p1 is None:
        p1 = np.zeros_like(z)
        p2 = np.zeros_like(z)
    if lam == 0.0:
        return np.maximum(0.0, z), p1, p2
    for _ in range(n_iter):
        p1, p2 = tv_dual_step(z, lam, p1, p2, tau_c)
    return np.maximum(0.0, z - lam * div(p1, p2)), p1, p2


def prox_duality_gap(z, lam, p1, p2):
    """Primal minus dual value of the constrained ROF problem at the dual point p.

    primal: lam psi(x) + 1/2 ||x - z||^2 at x = max(0, z - lam div p)
    dual:   1/2 ||z||^2 - 1/2 ||max(0, z - lam div p)||^2   (|p_j| <= 1)
    """
    x = np.maximum(0.0, z - lam * div(p1, p2))
    primal = lam * tv_norm(x) + 0.5 * float(((x - z) ** 2).sum())
    dual = 0.5 * float((z * z).sum()) - 0.5 * float((x * x).sum())
    return primal - dual
