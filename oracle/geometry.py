"""Parallel-beam geometry (Sec. 2.1: standard parallel-beam geometry, the
sinogram sampling p(r, theta) on a regular grid; Eq. 24 counts m views over
[0, pi)).

Readings (the paper fixes none of these): unit pixels and unit detector
spacing, grids centred on the rotation axis, theta_v = v*pi/m unless view
angles are given.  The choice of
stepping axis for each view (rows when |cos| >= |sin|) is decided from the
integer view index so that the 45 and 135 degree ties never depend on
floating-point rounding.
"""
import numpy as np


def angles(m, theta=None):
    """theta_v = v*pi/m, v = 0..m-1, or the given view angles (radians)."""
    if theta is not None:
        theta = np.asarray(theta, dtype=np.float64)
        assert theta.shape == (m,)
        return theta
    return np.arange(m, dtype=np.float64) * (np.pi / m)


# Given angles take the row branch where |cos| >= |sin| (1 - ROW_TIE): angles
# within that margin of a 45 degree diagonal go to the row branch whichever
# way cos and sin round.
ROW_TIE = 1e-12


def row_branch(m, theta=None):
    """True where the view steps over image rows (|cos| >= |sin|).

    For theta = v*pi/m that is theta <= pi/4 or theta >= 3pi/4, i.e.
    4v <= m or 4v >= 3m, ties included in the row branch.
    """
    if theta is not None:
        th = angles(m, theta)
        return np.abs(np.cos(th)) >= np.abs(np.sin(th)) * (1.0 - ROW_TIE)
    v = np.arange(m)
    return (4 * v <= m) | (4 * v >= 3 * m)


def pixel_centres(n):
    return np.arange(n, dtype=np.float64) - (n - 1) / 2.0


def bin_centres(nb):
    return np.arange(nb, dtype=np.float64) - (nb - 1) / 2.0
