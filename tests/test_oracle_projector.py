"""Pins for the oracle's projector A and transpose A^T (system matrix, Sec. 2.1).

Each test ties the oracle to something other than its own formula:
closed-form line integrals, exact sums at 0 and 90 degrees, the adjoint
identity, and an independently derived pixel-driven form of A^T.
"""
import math

import numpy as np
import pytest

from oracle import projector as P
from oracle.geometry import row_branch
from paper_1609_06041_amd import synth as S


def _gauss_image(n, x0, y0, s):
    c = np.arange(n) - (n - 1) / 2.0
    return np.exp(-((c[None, :] - x0) ** 2 + (c[:, None] - y0) ** 2) / (2 * s * s))


def _gauss_sino(n, m, nb, x0, y0, s):
    # Line integral of exp(-|p - p0|^2 / 2s^2) along x cos + y sin = r.
    th = np.arange(m) * np.pi / m
    r = np.arange(nb) - (nb - 1) / 2.0
    d = r[None, :] - x0 * np.cos(th)[:, None] - y0 * np.sin(th)[:, None]
    return math.sqrt(2 * math.pi) * s * np.exp(-d * d / (2 * s * s))


def test_column_sums_at_zero_degrees():
    rng = np.random.default_rng(1)
    n, m, nb = 10, 4, 14            # nb - n even: rays at 0 deg hit column centres
    x = rng.standard_normal((n, n))
    y = P.forward_project(x, m, nb)
    off = (nb - n) // 2
    np.testing.assert_allclose(y[0, off:off + n], x.sum(axis=0), rtol=0, atol=1e-12)
    assert np.all(y[0, :off] == 0) and np.all(y[0, off + n:] == 0)


def test_row_sums_at_ninety_degrees():
    rng = np.random.default_rng(2)
    n, m, nb = 10, 4, 14            # view 2 of 4 is at 90 degrees
    x = rng.standard_normal((n, n))
    y = P.forward_project(x, m, nb)
    off = (nb - n) // 2
    np.testing.assert_allclose(y[2, off:off + n], x.sum(axis=1), rtol=0, atol=1e-12)


def test_gaussian_blob_projection_converges_second_order():
    # Point-sampled Gaussian, width proportional to N: Joseph's linear
    # interpolation error is O(h^2 / s^2), so each doubling of N must cut
    # the error by about four.
    errs = []
    for n in (32, 64, 128):
        x0, y0, s = 0.12 * n, -0.08 * n, 0.065 * n     # > 6 s from the border
        m, nb = 36, int(1.5 * n)
        got = P.forward_project(_gauss_image(n, x0, y0, s), m, nb)
        ref = _gauss_sino(n, m, nb, x0, y0, s)
        errs.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    assert errs[1] < 0.3 * errs[0] and errs[2] < 0.3 * errs[1], errs
    assert errs[1] < 5e-3, errs


def test_ellipse_chords_match_rasterised_projection():
    # An off-centre rotated ellipse: any error in the geometry convention
    # (bin or pixel centring, angle direction, stepping weight) moves or
    # rescales the projection far beyond the interpolation blur.
    errs = []
    for n in (32, 64, 128):
        ell = [S.Ellipse(0.1 * n, -0.05 * n, 0.24 * n, 0.2 * n, 0.4, 1.0)]
        m, nb = 45, int(1.5 * n)
        got = P.forward_project(S.rasterise(ell, n, sub=8), m, nb)
        ref = S.line_integrals(ell, n, m, nb)
        errs.append(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    assert errs[1] < 0.025 and errs[2] < 0.6 * errs[1], errs


@pytest.mark.parametrize("n,m,nb", [(16, 12, 24), (15, 13, 21), (8, 8, 11), (7, 4, 7), (1, 1, 1)])
def test_adjoint_identity(n, m, nb):
    rng = np.random.default_rng(n * 100 + m)
    x = rng.standard_normal((n, n))
    y = rng.standard_normal((m, nb))
    lhs = np.dot(P.forward_project(x, m, nb).ravel(), y.ravel())
    rhs = np.dot(x.ravel(), P.back_project(y, n).ravel())
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.linalg.norm(x) * np.linalg.norm(y))


def _pixel_driven_transpose(y, n):
    # A^T written the other way round: pixel (ix, iy) and view v collect the
    # bins within one step-length of t = X cos + Y sin with the hat weight
    # max(0, 1 - |r_u - t| / s_v) / s_v, s_v = |cos| (row views) or |sin|.
    m, nb = y.shape
    c = np.arange(n) - (n - 1) / 2.0
    r = np.arange(nb) - (nb - 1) / 2.0
    rows = row_branch(m)
    out = np.zeros((n, n))
    for v in range(m):
        th = v * np.pi / m
        sv = abs(math.cos(th)) if rows[v] else abs(math.sin(th))
        t = c[None, :] * math.cos(th) + c[:, None] * math.sin(th)
        wgt = np.maximum(0.0, 1.0 - np.abs(r[None, None, :] - t[:, :, None]) / sv) / sv
        out += wgt @ y[v]
    return out


@pytest.mark.parametrize("n,m,nb", [(12, 16, 18), (9, 7, 13), (10, 4, 14)])
def test_transpose_equals_pixel_driven_form(n, m, nb):
    rng = np.random.default_rng(3)
    y = rng.standard_normal((m, nb))
    np.testing.assert_allclose(P.back_project(y, n), _pixel_driven_transpose(y, n), rtol=0, atol=1e-12)


def test_dense_matrix_columns_and_transpose():
    n, m, nb = 6, 8, 9
    a = P.dense_matrix(n, m, nb)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((n, n))
    y = rng.standard_normal((m, nb))
    np.testing.assert_allclose(a @ x.ravel(), P.forward_project(x, m, nb).ravel(), atol=1e-12)
    np.testing.assert_allclose(a.T @ y.ravel(), P.back_project(y, n).ravel(), atol=1e-12)
    # every entry is a hat weight over a step length: 0 <= a_ij <= sqrt(2)
    assert a.min() >= 0.0 and a.max() <= math.sqrt(2) + 1e-12


def test_forty_five_degree_ties_use_row_branch():
    # With m = 8, views 2 and 6 are 45 and 135 degrees: both step over rows,
    # weight 1/|cos| = sqrt(2).
    flags = row_branch(8)
    assert list(flags) == [True, True, True, False, False, False, True, True]


# ---- given view angles --------------------------------------------------

def _gauss_sino_at(n, theta, nb, x0, y0, s):
    r = np.arange(nb) - (nb - 1) / 2.0
    d = r[None, :] - x0 * np.cos(theta)[:, None] - y0 * np.sin(theta)[:, None]
    return math.sqrt(2 * math.pi) * s * np.exp(-d * d / (2 * s * s))


def test_given_angles_match_the_line_integrals_of_a_blob():
    # irregular angles over more than a half turn, negative ones included:
    # the projection of a smooth blob is its closed-form line integral, to
    # the interpolation error of the default scan at the same width
    n, nb = 96, 140
    theta = np.array([-0.9, -0.2, 0.05, 0.61, 1.3, 1.9, 2.45, 3.0, 3.9, 5.1])
    x = _gauss_image(n, 7.0, -11.0, 6.0)
    y = P.forward_project(x, len(theta), nb, theta=theta)
    ref = _gauss_sino_at(n, theta, nb, 7.0, -11.0, 6.0)
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    y0 = P.forward_project(x, 10, nb)
    err0 = np.linalg.norm(y0 - _gauss_sino(n, 10, nb, 7.0, -11.0, 6.0)) / np.linalg.norm(y0)
    assert err < 2e-3 and err < 2.0 * err0, (err, err0)


def test_half_turn_reverses_the_bins():
    # p(r, theta + pi) = p(-r, theta): on the symmetric bin grid a view turned
    # by pi is the same view with its bins reversed (sign and branch rules of
    # the given-angle path)
    rng = np.random.default_rng(7)
    n, nb = 20, 31
    theta = rng.uniform(0.0, np.pi, 9)
    x = rng.standard_normal((n, n))
    y = P.forward_project(x, 9, nb, theta=theta)
    yt = P.forward_project(x, 9, nb, theta=theta + np.pi)
    np.testing.assert_allclose(yt, y[:, ::-1], rtol=0, atol=1e-12 * np.abs(y).max())


def test_uniform_angles_given_equal_the_default():
    # the default scan spelled out, away from the 45-degree ties (m = 10)
    rng = np.random.default_rng(8)
    n, m, nb = 14, 10, 21
    x = rng.standard_normal((n, n))
    yb = rng.standard_normal((m, nb))
    th = np.arange(m) * np.pi / m
    np.testing.assert_array_equal(row_branch(m, th), row_branch(m))
    np.testing.assert_allclose(P.forward_project(x, m, nb, theta=th), P.forward_project(x, m, nb), atol=1e-12)
    np.testing.assert_allclose(P.back_project(yb, n, theta=th), P.back_project(yb, n), atol=1e-12)


def test_given_angles_adjoint_identity_and_diagonal_ties():
    rng = np.random.default_rng(9)
    n, nb = 11, 17
    theta = np.array([np.pi / 4, 3 * np.pi / 4, -np.pi / 4, 0.3, 2.2, 7.0])
    # the diagonals take the row branch however cos and sin round
    assert list(row_branch(6, theta)[:3]) == [True, True, True]
    x = rng.standard_normal((n, n))
    y = rng.standard_normal((6, nb))
    lhs = np.dot(P.forward_project(x, 6, nb, theta=theta).ravel(), y.ravel())
    rhs = np.dot(x.ravel(), P.back_project(y, n, theta=theta).ravel())
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.linalg.norm(x) * np.linalg.norm(y))
