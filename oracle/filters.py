"""The preconditioner D as a per-view 1-D filter along the detector (Eqs. 24, 32).

The paper writes D = F^{-1} H(omega) F with
  few-view  (Eq. 32): H(omega) = |omega| / (2 m tau)
  low-dose  (Eq. 24): H(omega) = |omega| / (2 m tau + kappa |omega|)
where kappa is the mean of the diagonal of W^{-1}.

Readings: omega is in radians per detector bin, band-limited to [-pi, pi];
D acts on each view as the linear (non-circular) convolution of the nb bins
with the inverse DTFT of H, i.e. a symmetric Toeplitz matrix
T[i, j] = h[i - j].  The taps are

  h[n] = (1/pi) * integral_0^pi H(omega) cos(n omega) d omega.

Pure ramp: h[0] = pi/2, h[n] = -2/(pi n^2) for odd n, 0 for even n != 0,
all divided by 2 m tau.

Smoothed ramp: the defining integral is evaluated by QUADPACK's
Fourier-weighted rule (scipy ``quad`` with ``weight='cos'``).  A closed form
exists: with a = 2 m tau / kappa, omega/(2 m tau + kappa omega)
= (1 - a/(a + omega))/kappa, and integrating cos(n omega)/(a + omega) with the
sine and cosine integrals Si, Ci gives

  h[0] = (pi - a ln(1 + pi/a)) / (pi kappa)
  h[n] = -(a/(pi kappa)) [cos(n a)(Ci(n(a+pi)) - Ci(n a)) + sin(n a)(Si(n(a+pi)) - Si(n a))]

but it cancels catastrophically once a is large (small kappa), so it only
serves as an independent check at moderate a.
"""
import warnings

import numpy as np
from scipy.integrate import IntegrationWarning, quad
from scipy.linalg import toeplitz
from scipy.special import sici


def ramp_taps(nb, m, tau):
    """Taps h[n], n = -(nb-1)..nb-1 (index n + nb - 1), of Eq. 32."""
    n = np.arange(-(nb - 1), nb, dtype=np.float64)
    h = np.zeros_like(n)
    h[n == 0] = np.pi / 2.0
    odd = (np.abs(n) % 2) == 1
    h[odd] = -2.0 / (np.pi * n[odd] ** 2)
    return h / (2.0 * m * tau)


def smoothed_ramp_taps(nb, m, tau, kappa):
    """Taps of Eq. 24 by quadrature of the defining integral; kappa == 0 gives Eq. 32."""
    if kappa == 0.0:
        return ramp_taps(nb, m, tau)
    c0 = 2.0 * m * tau
    g = lambda w: w / (c0 + kappa * w)
    pos = np.empty(nb)
    pos[0] = quad(g, 0.0, np.pi, epsabs=0.0, epsrel=1e-13, limit=200)[0] / np.pi
    tol = 1e-14 * pos[0] * np.pi
    with warnings.catch_warnings():
        # QUADPACK flags roundoff near its (very tight) tolerance; the taps are
        # pinned to independent quadrature and the Si/Ci form by the tests.
        warnings.simplefilter("ignore", IntegrationWarning)
        for n in range(1, nb):
            pos[n] = quad(g, 0.0, np.pi, weight="cos", wvar=n, epsabs=tol, epsrel=1e-12,
                          limit=200)[0] / np.pi
    return np.concatenate([pos[:0:-1], pos])


def smoothed_ramp_taps_sici(nb, m, tau, kappa):
    """Closed form of the Eq. 24 taps via Si/Ci (accurate only for moderate 2 m tau / kappa)."""
    a = 2.0 * m * tau / kappa
    n = np.arange(1, nb, dtype=np.float64)
    si1, ci1 = sici(n * (a + np.pi))
    si0, ci0 = sici(n * a)
    pos = -(a / (np.pi * kappa)) * (np.cos(n * a) * (ci1 - ci0) + np.sin(n * a) * (si1 - si0))
    h0 = (np.pi - a * np.log1p(np.pi / a)) / (np.pi * kappa)
    return np.concatenate([pos[::-1], [h0], pos])


def toeplitz_matrix(h):
    """Symmetric Toeplitz T[i, j] = h[i - j] from taps indexed n + nb - 1."""
    nb = (h.size + 1) // 2
    return toeplitz(h[nb - 1:])


def apply_filter(s, h):
    """(D s)[v, i] = sum_j h[i - j] s[v, j] for every view v."""
    s = np.asarray(s, dtype=np.float64)
    return s @ toeplitz_matrix(h)
