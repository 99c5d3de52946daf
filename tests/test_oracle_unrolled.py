"""Pins for the finite-difference reference gradient of the unrolled solve.

* One iteration with beta = 0 has the closed form x^1 = max(0, sigma tau A^T D b)
  (the TV prox reduces to the clamp), so dL/dsigma and the directional
  derivative along v follow by hand; the central differences must reproduce
  them.
* The unrolled function equals the oracle's Algorithm 1 at the same steps.
"""
import numpy as np
import pytest

from oracle import app as AP
from oracle import filters as F
from oracle import projector as P
from oracle import unrolled as U


def _problem(seed, n=12, m=10, nb=18):
    rng = np.random.default_rng(seed)
    xt = np.zeros((n, n))
    xt[3:9, 4:8] = 1.0
    b = P.forward_project(xt, m, nb) + 0.05 * rng.standard_normal((m, nb))
    w = rng.uniform(0.5, 2.0, (m, nb))
    return xt, b, w


def test_one_iteration_closed_form_gradients():
    n, m, nb = 12, 10, 18
    xt, b, w = _problem(1, n, m, nb)
    tau, sigma = 0.3, 0.7
    kappa = float((1.0 / w).mean())
    h = F.smoothed_ramp_taps(nb, m, tau, kappa)
    u = tau * P.back_project(F.apply_filter(b, h), n)          # x^1 = max(0, sigma u)
    x1 = np.maximum(0.0, sigma * u)
    np.testing.assert_allclose(U.unrolled_lowdose(b, w, 0.0, tau, sigma, n, 1), x1, atol=1e-13)
    mask = (sigma * u > 0).astype(float)
    r = 2.0 * (x1 - xt) * mask
    d_sigma = float((r * u).sum())
    v = np.random.default_rng(2).standard_normal((m, nb))
    d_v = float((r * sigma * tau * P.back_project(F.apply_filter(v, h), n)).sum())
    g = U.fd_gradients(b, w, 0.0, tau, sigma, n, 1, xt, directions=[v], rel_h=False)
    assert g["sigma"] == pytest.approx(d_sigma, rel=1e-7)
    assert g["b_dir"][0] == pytest.approx(d_v, rel=1e-7)


def test_unrolled_equals_algorithm1_at_the_same_steps():
    n, m, nb = 12, 10, 18
    _, b, w = _problem(3, n, m, nb)
    res, st = AP.lowdose_solve(b, w, 0.02, n, 4, tau=0.2, sigma=0.5)
    np.testing.assert_array_equal(U.unrolled_lowdose(b, w, 0.02, 0.2, 0.5, n, 4), res.x)
