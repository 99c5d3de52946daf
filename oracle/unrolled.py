"""The unrolled Algorithm 1 as a function of its data and parameters, and its
gradient by central finite differences in float64 -- the reference the GPU's
hand-written reverse pass is checked against.

``unrolled_lowdose(b, w, beta, tau, sigma, n, iters)`` runs exactly ``iters``
iterations of Eqs. 18-20 from zero with the given step sizes (no operator
norms: tau and sigma are inputs), with D = D(tau) the smoothed ramp of Eq. 24
at kappa = mean(1/w) -- so the result depends on tau through the step, the
TV weight tau*beta and the filter.
"""
import numpy as np

from .app import app_solve
from .filters import smoothed_ramp_taps


def unrolled_lowdose(b, w, beta, tau, sigma, n, iters, n_tv=10, tau_c=0.125):
    b = np.asarray(b, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    m, nb = b.shape
    winv = 1.0 / w
    kappa = float(winv.mean())
    h = smoothed_ramp_taps(nb, m, tau, kappa)
    return app_solve(b, n, iters, tau, sigma, h, beta=beta, winv=winv, n_tv=n_tv, tau_c=tau_c).x


def sq_loss(x, x_true):
    d = np.asarray(x, dtype=np.float64) - np.asarray(x_true, dtype=np.float64)
    return float((d * d).sum())


def central_difference(f, x0, h=1e-6):
    """(f(x0 + h) - f(x0 - h)) / 2h for a scalar function of a scalar."""
    return (f(x0 + h) - f(x0 - h)) / (2.0 * h)


def fd_gradients(b, w, beta, tau, sigma, n, iters, x_true, directions=(), h=1e-6, rel_h=True, **kw):
    """Central differences of ||x_iters - x_true||^2 with respect to beta, tau,
    sigma (steps relative to the value when ``rel_h``) and along each given
    direction v in sinogram space (the directional derivative <dL/db, v>)."""
    b = np.asarray(b, dtype=np.float64)
    L = lambda **a: sq_loss(unrolled_lowdose(a.get("b", b), w, a.get("beta", beta), a.get("tau", tau),
                                             a.get("sigma", sigma), n, iters, **kw), x_true)
    out = {}
    for name, val in (("beta", beta), ("tau", tau), ("sigma", sigma)):
        if rel_h and val == 0.0:   # no relative step at zero (and beta = 0 is a kink of the prox)
            out[name] = None
            continue
        hh = h * val if rel_h else h
        out[name] = central_difference(lambda v: L(**{name: v}), val, hh)
    out["b_dir"] = [central_difference(lambda t: L(b=b + t * v), 0.0, h) for v in directions]
    return out
