"""The seeded input generator: exact chords, reproducibility, noise model."""
import math

import numpy as np
import pytest

from paper_1609_06041_amd import synth as S


def test_disk_chord_is_closed_form():
    n, m, nb = 32, 6, 40
    disk = [S.Ellipse(3.0, -2.0, 7.0, 7.0, 0.3, 0.8)]
    got = S.line_integrals(disk, n, m, nb)
    th = np.arange(m) * math.pi / m
    r = np.arange(nb) - (nb - 1) / 2.0
    d = r[None, :] - 3.0 * np.cos(th)[:, None] + 2.0 * np.sin(th)[:, None]
    ref = 0.8 / n * 2.0 * np.sqrt(np.maximum(49.0 - d * d, 0.0))
    np.testing.assert_allclose(got, ref, atol=1e-13)


def test_ellipse_integral_mass():
    # integral over r of the projection = density * area, for every view
    n, m, nb = 64, 8, 96
    e = [S.Ellipse(-4.0, 5.0, 12.0, 5.0, 1.1, 0.6)]
    p = S.line_integrals(e, n, m, nb)
    area = math.pi * 12.0 * 5.0 * 0.6 / n
    np.testing.assert_allclose(p.sum(axis=1), area, rtol=1.5e-2)   # unit-spacing Riemann sum


def test_seeded_problems_are_reproducible_and_inside_the_grid():
    a = S.make_problem(0, 3, 64, 30, 96, 8, 1e4, with_x_true=False)
    b = S.make_problem(0, 3, 64, 30, 96, 8, 1e4, with_x_true=False)
    assert np.array_equal(a.b, b.b) and np.array_equal(a.w, b.w)
    for e in a.ellipses:
        assert math.hypot(e.x0, e.y0) + max(e.a, e.b) <= 64 / 2 - 1
    assert np.all(a.w >= 1.0) and np.all(np.isfinite(a.b))
    c = S.make_problem(0, 4, 64, 30, 96, 8, 1e4, with_x_true=False)
    assert not np.array_equal(a.b, c.b)


def test_rasterised_phantom_matches_density_scale():
    e = [S.Ellipse(0.0, 0.0, 10.0, 10.0, 0.0, 1.0)]
    x = S.rasterise(e, 32)
    assert x.max() == 1.0 / 32
    assert abs(x.sum() - math.pi * 100 / 32) < 0.01 * math.pi * 100 / 32


def test_too_small_image_is_rejected_not_looped():
    with pytest.raises(ValueError):
        S.draw_ellipses(2, 3, S.rng_for(0, 0, 0))
