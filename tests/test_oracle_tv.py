"""Pins for the TV norm (Eq. 2) and the TV prox with x >= 0 (Eq. 17).

Closed-form TV of rectangles and border pixels; the adjoint relation of
grad and div; the ROF duality gap (weak duality certifies optimality
independently of the algorithm); and a 1-D reduction whose exact solution
comes from a bounded least-squares solve (scipy ``lsq_linear``).
"""
import math

import numpy as np
import pytest
from scipy.optimize import lsq_linear

from oracle import tv as T


@pytest.mark.parametrize("nr,nc,c", [(1, 1, 1.0), (3, 5, 2.5), (7, 2, -0.75)])
def test_tv_of_rectangle(nr, nc, c):
    x = np.zeros((16, 16))
    x[4:4 + nr, 6:6 + nc] = c
    assert T.tv_norm(x) == pytest.approx(abs(c) * (2 * nr + 2 * nc - 2 + math.sqrt(2)), rel=1e-14)


def test_tv_of_constant_and_border_pixel():
    assert T.tv_norm(np.full((9, 9), 3.0)) == 0.0
    x = np.zeros((8, 8))
    x[7, 7] = 2.0          # bottom-right: no difference leaves the image there
    assert T.tv_norm(x) == pytest.approx(4.0, rel=1e-15)
    x = np.zeros((8, 8))
    x[0, 0] = 2.0          # top-left: only the pixel itself sees (-2, -2)
    assert T.tv_norm(x) == pytest.approx(2.0 * math.sqrt(2), rel=1e-15)


def test_div_is_negative_adjoint_of_grad():
    rng = np.random.default_rng(0)
    for shape in ((7, 7), (12, 12), (2, 2), (1, 1)):
        x = rng.standard_normal(shape)
        p1, p2 = rng.standard_normal(shape), rng.standard_normal(shape)
        g1, g2 = T.grad(x)
        lhs = float((g1 * p1).sum() + (g2 * p2).sum())
        rhs = -float((x * T.div(p1, p2)).sum())
        assert abs(lhs - rhs) <= 1e-13 * (1 + abs(lhs))


def test_div_matches_chambolle_boundary_rule():
    # Chambolle (2004): (div p)_ij = p1_ij - p1_i,j-1 inside, p1_ij on the first
    # column, -p1_i,j-1 on the last; likewise for p2 down the rows.
    rng = np.random.default_rng(6)
    n = 6
    p1, p2 = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    d = T.div(p1, p2)
    for i in range(n):
        for j in range(n):
            a = p1[i, j] if j == 0 else (-p1[i, j - 1] if j == n - 1 else p1[i, j] - p1[i, j - 1])
            b = p2[i, j] if i == 0 else (-p2[i - 1, j] if i == n - 1 else p2[i, j] - p2[i - 1, j])
            assert d[i, j] == pytest.approx(a + b, abs=1e-15)


def test_prox_with_zero_weight_is_clamp():
    rng = np.random.default_rng(1)
    z = rng.standard_normal((10, 10))
    x, _, _ = T.tv_prox(z, 0.0)
    assert np.array_equal(x, np.maximum(0.0, z))


def test_prox_duality_gap_closes():
    rng = np.random.default_rng(2)
    z = np.zeros((16, 16))
    z[3:11, 4:12] = 1.0
    z += 0.3 * rng.standard_normal(z.shape)
    lam = 0.2
    p1 = p2 = None
    gaps = []
    for i in range(6):             # 31500 projected-gradient steps in total
        x, p1, p2 = T.tv_prox(z, lam, p1, p2, n_iter=500 * 2 ** i)
        gaps.append(T.prox_duality_gap(z, lam, p1, p2))
    assert all(g >= -1e-12 for g in gaps)
    assert gaps[-1] < 1e-2 * gaps[0] and gaps[-1] < 5e-6
    assert np.all(x >= 0)


def test_prox_is_positively_homogeneous():
    rng = np.random.default_rng(3)
    z = rng.standard_normal((12, 12))
    x1, _, _ = T.tv_prox(z, 0.3, n_iter=2000)
    x2, _, _ = T.tv_prox(4.0 * z, 1.2, n_iter=2000)
    np.testing.assert_allclose(x2, 4.0 * x1, atol=1e-10)


def test_prox_reduces_to_1d_tv_denoising():
    # z constant down the columns: the minimiser is too, and every row solves
    # min_{x>=0} lam * sum |x[i+1]-x[i]| + 1/2 ||x - s||^2.  In 1-D that is the
    # clamp of the unconstrained TV prox, whose dual is a box-constrained
    # least-squares problem: u = argmin_{|u|<=lam} ||D^T u - s||, x = s - D^T u.
    rng = np.random.default_rng(4)
    n = 16
    s = np.repeat([0.8, -0.2, 1.5, 0.3], 4) + 0.2 * rng.standard_normal(n)
    lam = 0.35
    d = np.diff(np.eye(n), axis=0)             # (n-1) x n forward difference
    u = lsq_linear(d.T, s, bounds=(-lam, lam), method="bvls", tol=1e-15).x
    ref = np.maximum(0.0, s - d.T @ u)
    z = np.tile(s, (n, 1))
    x, p1, p2 = T.tv_prox(z, lam, n_iter=20000)
    np.testing.assert_allclose(x, np.tile(ref, (n, 1)), atol=1e-8)


def test_clamp_inside_the_loop_matters():
    # For 2-D isotropic TV, clamping an unconstrained prox is not the
    # constrained prox; the oracle must return the constrained one, which has
    # a smaller objective value.
    rng = np.random.default_rng(5)
    z = 0.5 * rng.standard_normal((16, 16))
    lam = 0.25
    x, _, _ = T.tv_prox(z, lam, n_iter=5000)
    # unconstrained prox via the same dual iteration without the clamp
    p1 = np.zeros_like(z)
    p2 = np.zeros_like(z)
    for _ in range(5000):
        g1, g2 = T.grad(z - lam * T.div(p1, p2))
        q1, q2 = p1 - g1 / (8 * lam), p2 - g2 / (8 * lam)
        sc = np.maximum(1.0, np.hypot(q1, q2))
        p1, p2 = q1 / sc, q2 / sc
    xc = np.maximum(0.0, z - lam * T.div(p1, p2))
    obj = lambda y: lam * T.tv_norm(y) + 0.5 * ((y - z) ** 2).sum()
    assert np.abs(x - xc).max() > 1e-3
    assert obj(x) < obj(xc) - 1e-6
