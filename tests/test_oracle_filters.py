"""Pins for the preconditioner D (Eq. 24 smoothed ramp, Eq. 32 ramp).

The taps are pinned to an independent quadrature of the defining integral,
to the Si/Ci closed form, to their own DTFT (which must reproduce H(omega)),
to the kappa -> 0 limit, and to the FBP normalisation that Eq. 24's 2m
factor implies (a uniform disk reconstructs to its density).
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import filters as F
from oracle import projector as P
from paper_1609_06041_amd import synth as S


def _h_quad(n, m, tau, kappa):
    # (1/pi) * integral_0^pi H(w) cos(n w) dw, plain adaptive quadrature.
    f = lambda w: w / (2 * m * tau + kappa * w) * math.cos(n * w)
    return quad(f, 0.0, math.pi, limit=800, epsabs=1e-14, epsrel=1e-12)[0] / math.pi


@pytest.mark.parametrize("m,tau", [(90, 1.0), (32, 0.37)])
def test_ramp_taps_match_quadrature(m, tau):
    nb = 40
    h = F.ramp_taps(nb, m, tau)
    for n in (0, 1, 2, 3, 10, 17, 39):
        ref = _h_quad(n, m, tau, 0.0)
        assert abs(h[nb - 1 + n] - ref) <= 1e-12 * abs(h[nb - 1]), n
        assert h[nb - 1 - n] == h[nb - 1 + n]


@pytest.mark.parametrize("m,tau,kappa", [(90, 2.8e-6, 1.6e-4), (720, 1e-5, 2e-5), (32, 0.5, 3.0)])
def test_smoothed_taps_match_quadrature(m, tau, kappa):
    nb = 64
    h = F.smoothed_ramp_taps(nb, m, tau, kappa)
    for n in (0, 1, 2, 5, 31, 63):
        ref = _h_quad(n, m, tau, kappa)
        assert abs(h[nb - 1 + n] - ref) <= 1e-11 * abs(h[nb - 1]), n


def test_smoothed_taps_match_sici_closed_form():
    nb, m, tau, kappa = 96, 90, 0.01, 1.0      # a = 2 m tau / kappa = 1.8
    h = F.smoothed_ramp_taps(nb, m, tau, kappa)
    c = F.smoothed_ramp_taps_sici(nb, m, tau, kappa)
    assert np.abs(h - c).max() <= 1e-13 * abs(h[nb - 1])


def test_kappa_to_zero_gives_ramp():
    nb, m, tau = 64, 90, 1.0
    r = F.ramp_taps(nb, m, tau)
    s = F.smoothed_ramp_taps(nb, m, tau, 1e-9)
    assert np.abs(s - r).max() <= 1e-8 * abs(r[nb - 1])
    assert np.array_equal(F.smoothed_ramp_taps(nb, m, tau, 0.0), r)


@pytest.mark.parametrize("kappa", [0.0, 0.02])
def test_taps_reproduce_frequency_response(kappa):
    # sum_n h[n] cos(n w) is the truncated DTFT; the tail is O(1/L).
    nb, m, tau = 2048, 90, 0.3
    h = F.smoothed_ramp_taps(nb, m, tau, kappa)
    n = np.arange(-(nb - 1), nb)
    for w in (0.3, 1.0, 2.0, 2.9):
        dtft = float(np.dot(h, np.cos(n * w)))
        hw = w / (2 * m * tau + kappa * w)
        assert abs(dtft - hw) <= 2e-3 * (math.pi / (2 * m * tau)), (w, dtft, hw)


@pytest.mark.parametrize("kappa", [0.0, 0.05])
def test_toeplitz_is_symmetric_positive_definite(kappa):
    nb, m, tau = 96, 90, 0.2
    t = F.toeplitz_matrix(F.smoothed_ramp_taps(nb, m, tau, kappa))
    assert np.array_equal(t, t.T)
    ev = np.linalg.eigvalsh(t)
    assert ev[0] > 0 and ev[-1] <= math.pi / (2 * m * tau) * (1 + 1e-12)


def test_filter_equals_linear_convolution():
    rng = np.random.default_rng(0)
    nb, m = 37, 5
    h = F.smoothed_ramp_taps(nb, m, 0.4, 0.1)
    s = rng.standard_normal((m, nb))
    got = F.apply_filter(s, h)
    ref = np.stack([np.convolve(s[v], h)[nb - 1:2 * nb - 1] for v in range(m)])
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


def test_fbp_normalisation_recovers_disk_density():
    # (1/2m) A^T ramp b reconstructs a uniform disk: this fixes omega in
    # radians per bin and the 2m of Eqs. 24 and 32.
    n, m, nb = 64, 90, 96
    disk = [S.Ellipse(0.0, 0.0, 20.0, 20.0, 0.0, 1.0)]
    b = S.line_integrals(disk, n, m, nb) * n          # density 1 per pixel
    rec = P.back_project(F.apply_filter(b, F.ramp_taps(nb, m, 1.0)), n)
    c = np.arange(n) - (n - 1) / 2.0
    inner = np.hypot(c[None, :], c[:, None]) < 15
    assert abs(rec[inner].mean() - 1.0) < 5e-3
    assert rec[inner].std() < 0.02
    outer = np.hypot(c[None, :], c[:, None]) > 25
    assert np.abs(rec[outer]).mean() < 0.02
