"""The two unpreconditioned comparators the paper runs against Algorithms 1
and 2 (Sec. 4; Table 1 places them in the same first-order primal-dual
family), in float64.

The paper's bibliography is not part of the text, so both are written from
the original publications:

* GIST (Loris and Verhoeven, "On a generalization of the iterative
  soft-thresholding algorithm for the case of non-separable penalty",
  Inverse Problems 27, 2011): a gradient step on the differentiable data
  term, a proximal (projection) step on the dual of the non-separable
  penalty.  Eq. 1 also carries the constraint x >= 0; it enters as the
  projection P+ in the primal-dual fixed-point form of Chen, Huang and Zhang
  ("A primal-dual fixed point algorithm for minimization of the sum of three
  convex separable functions", Fixed Point Theory Appl. 2016), which reduces
  to the Loris-Verhoeven iteration without the constraint.  For
  f(x) = 1/2 ||Ax - b||_W^2, penalty beta ||grad x||_{2,1}:

      u       = x^k - gamma A^T W (A x^k - b)
      y       = P+(u + lam div v^k)
      v^{k+1} = projection of (v^k + grad y) onto {|v_j| <= gamma beta / lam}
      x^{k+1} = P+(u + lam div v^{k+1})

  with 0 < gamma < 2 / lambda_max(A^T W A) and 0 < lam <= 1/8 (the bound
  ||grad||^2 <= 8).  Here gamma = rho * 2 / lambda_max(A^T W A), lam = 1/8.

* Chambolle-Pock (Chambolle and Pock, "A first-order primal-dual algorithm
  for convex problems with applications to imaging", J. Math. Imaging Vis.
  40, 2011, Algorithm 1 with theta = 1) for the few-view problem
  min ||grad x||_{2,1} s.t. Ax = b, x >= 0, with K = [A; grad]:

      y1 <- y1 + s (A xbar - b)
      y2 <- projection of (y2 + s grad xbar) onto {|y2_j| <= 1}
      x  <- P+(x - t (A^T y1 - div y2))
      xbar = 2 x^{new} - x^{old}

  with s = t = rho / L, L^2 = lambda_max(A^T A) + 8 >= ||K||^2.

Both start from zero in every variable.
"""
from dataclasses import dataclass

import numpy as np

from .app import lambda_max
from .projector import back_project, forward_project
from .tv import div, grad

GIST_LAM = 0.125


def lambda_atwa(w, n):
    """lambda_max(A^T W A), the Lipschitz constant of the gradient of 1/2 ||Ax - b||_W^2."""
    w = np.asarray(w, dtype=np.float64)
    m, nb = w.shape
    op = lambda v: back_project(w * forward_project(v.reshape(n, n), m, nb), n).ravel()
    return lambda_max(op, n * n)


def lambda_ata(n, m, nb):
    """lambda_max(A^T A)."""
    op = lambda v: back_project(forward_project(v.reshape(n, n), m, nb), n).ravel()
    return lambda_max(op, n * n)


@dataclass
class CompSteps:
    primal: float      # gamma (GIST) or t (CP)
    dual: float        # lam (GIST) or s (CP)
    norm: float        # lambda_max(A^T W A) (GIST) or lambda_max(A^T A) (CP)


def gist_steps(w, n, rho=0.95):
    la = lambda_atwa(w, n)
    return CompSteps(primal=rho * 2.0 / la, dual=GIST_LAM, norm=la)


def cp_steps(n, m, nb, rho=0.95):
    la = lambda_ata(n, m, nb)
    s = rho / np.sqrt(la + 8.0)
    return CompSteps(primal=s, dual=s, norm=la)


def _ball(q1, q2, radius):
    sc = np.maximum(1.0, np.hypot(q1, q2) / radius)
    return q1 / sc, q2 / sc


def gist_lowdose(b, w, beta, n, iters, gamma, lam=GIST_LAM, monitor=None):
    """GIST / primal-dual fixed-point iterations for Eq. 1.  Returns (x, (v1, v2), history)."""
    b = np.asarray(b, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    m, nb = b.shape
    x = np.zeros((n, n))
    v1 = np.zeros((n, n))
    v2 = np.zeros((n, n))
    radius = gamma * beta / lam
    hist = []
    for _ in range(iters):
        u = x - gamma * back_project(w * (forward_project(x, m, nb) - b), n)
        y = np.maximum(0.0, u + lam * div(v1, v2))
        g1, g2 = grad(y)
        if radius > 0:
            v1, v2 = _ball(v1 + g1, v2 + g2, radius)
        else:
            v1, v2 = np.zeros((n, n)), np.zeros((n, n))
        x = np.maximum(0.0, u + lam * div(v1, v2))
        if monitor is not None:
            hist.append(monitor(x))
    return x, (v1, v2), hist


def cp_fewview(b, n, iters, s, t, monitor=None):
    """Chambolle-Pock iterations for min TV s.t. Ax = b, x >= 0.  Returns (x, (y1, q1, q2), history)."""
    b = np.asarray(b, dtype=np.float64)
    m, nb = b.shape
    x = np.zeros((n, n))
    xb = np.zeros((n, n))
    y1 = np.zeros((m, nb))
    q1 = np.zeros((n, n))
    q2 = np.zeros((n, n))
    hist = []
    for _ in range(iters):
        y1 = y1 + s * (forward_project(xb, m, nb) - b)
        g1, g2 = grad(xb)
        q1, q2 = _ball(q1 + s * g1, q2 + s * g2, 1.0)
        xo = x
        x = np.maximum(0.0, x - t * (back_project(y1, n) - div(q1, q2)))
        xb = 2.0 * x - xo
        if monitor is not None:
            hist.append(monitor(x))
    return x, (y1, q1, q2), hist


def _shrink(u, t):
    """u max(0, 1 - t / ||u||): the prox of t ||.|| (Euclidean norm of the whole array)."""
    r = float(np.sqrt((u * u).sum()))
    return np.zeros_like(u) if r <= t else u * (1.0 - t / r)


def cp_fewview_eps(b, n, eps, iters, s, t, monitor=None):
    """Chambolle-Pock for min TV s.t. ||Ax - b|| <= eps, x >= 0: the same
    iteration as ``cp_fewview`` with the data block's dual prox for the ball
    indicator, prox of s (y^T b + eps ||y||) = shrink(v - s b, s eps); eps = 0
    gives ``cp_fewview``.  Returns (x, (y1, q1, q2), history)."""
    b = np.asarray(b, dtype=np.float64)
    m, nb = b.shape
    x = np.zeros((n, n))
    xb = np.zeros((n, n))
    y1 = np.zeros((m, nb))
    q1 = np.zeros((n, n))
    q2 = np.zeros((n, n))
    hist = []
    for _ in range(iters):
        y1 = _shrink(y1 + s * (forward_project(xb, m, nb) - b), s * eps)
        g1, g2 = grad(xb)
        q1, q2 = _ball(q1 + s * g1, q2 + s * g2, 1.0)
        xo = x
        x = np.maximum(0.0, x - t * (back_project(y1, n) - div(q1, q2)))
        xb = 2.0 * x - xo
        if monitor is not None:
            hist.append(monitor(x))
    return x, (y1, q1, q2), hist
