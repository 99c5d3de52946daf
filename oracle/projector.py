"""Forward projector A and its transpose (Sec. 2.1, the system matrix A = {a_ij}).

The paper only states that b samples the parallel-beam line integrals on a
regular grid.  This oracle reads A as Joseph's ray-driven model:

* a view whose rays are closer to vertical (|cos theta| >= |sin theta|) steps
  over the N image rows; at row centre y the ray ``x cos + y sin = r`` crosses
  ``x = (r - y sin)/cos``; the image is linearly interpolated along that row
  between its two neighbouring pixel centres, and the step contributes that
  value times the path length per row, 1/|cos theta|;
* the other views do the same over columns with weight 1/|sin theta|;
* interpolation partners outside the image are zero.

The transpose is computed as the literal scatter-add of those same weights
(``np.bincount``), i.e. as A^T by definition, not by a separate formula.
"""
import numpy as np

from .geometry import angles, row_branch, pixel_centres, bin_centres


def _view_samples(n, nb, theta, rowflag):
    """Fractional interpolation coordinate s[t, u] for step t, ray u, and the
    per-step path length.  For row views t is the row index and s an x index;
    for column views t is the column index and s a y index."""
    c = pixel_centres(n)
    r = bin_centres(nb)
    cs, sn = np.cos(theta), np.sin(theta)
    if rowflag:
        s = (r[None, :] - c[:, None] * sn) / cs + (n - 1) / 2.0
        length = 1.0 / abs(cs)
    else:
        s = (r[None, :] - c[:, None] * cs) / sn + (n - 1) / 2.0
        length = 1.0 / abs(sn)
    return s, length


def _pick(plane, t, k):
    """plane[t, k] with zero outside 0 <= k < n."""
    n = plane.shape[1]
    ok = (k >= 0) & (k < n)
    return np.where(ok, plane[t, np.clip(k, 0, n - 1)], 0.0)


def forward_project(x, m, nb, views=None, theta=None):
    """y = A x, y[v, u] = sum over steps of the interpolated image times the step length.

    ``views`` (optional) restricts the output to those view indices of the
    m-view scan, in that order (rows of the returned array); ``theta``
    (optional) gives the m view angles instead of v*pi/m.
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    assert x.shape == (n, n)
    th = angles(m, theta)
    rows = row_branch(m, theta)
    views = range(m) if views is None else list(views)
    y = np.zeros((len(views), nb))
    t = np.arange(n)[:, None]
    for i, v in enumerate(views):
        s, length = _view_samples(n, nb, th[v], rows[v])
        plane = x if rows[v] else x.T
        k = np.floor(s).astype(np.int64)
        f = s - k
        val = (1.0 - f) * _pick(plane, t, k) + f * _pick(plane, t, k + 1)
        y[i] = length * val.sum(axis=0)
    return y


def back_project(y, n, m=None, views=None, theta=None):
    """x = A^T y: every weight of ``forward_project`` scattered back onto its pixel.

    By default y holds all m = y.shape[0] views; with ``m`` and ``views`` given,
    row i of y is view ``views[i]`` of the m-view scan and the others are zero.
    ``theta`` (optional) gives the m view angles instead of v*pi/m.
    """
    y = np.asarray(y, dtype=np.float64)
    nb = y.shape[1]
    if views is None:
        m = y.shape[0]
        views = range(m)
    th = angles(m, theta)
    rows = row_branch(m, theta)
    acc_rows = np.zeros(n * n)   # indexed [iy, ix]
    acc_cols = np.zeros(n * n)   # indexed [ix, iy]
    t = np.broadcast_to(np.arange(n)[:, None], (n, nb))
    for i, v in enumerate(views):
        s, length = _view_samples(n, nb, th[v], rows[v])
        k = np.floor(s).astype(np.int64)
        f = s - k
        acc = acc_rows if rows[v] else acc_cols
        yv = np.broadcast_to(y[i][None, :], (n, nb))
        for kk, wt in ((k, 1.0 - f), (k + 1, f)):
            ok = (kk >= 0) & (kk < n)
            acc += np.bincount(t[ok] * n + kk[ok], weights=length * wt[ok] * yv[ok], minlength=n * n)
    return acc_rows.reshape(n, n) + acc_cols.reshape(n, n).T


def dense_matrix(n, m, nb):
    """Dense I x J matrix of A, built column by column as A e_j (small n only)."""
    a = np.zeros((m * nb, n * n))
    for j in range(n * n):
        e = np.zeros(n * n)
        e[j] = 1.0
        a[:, j] = forward_project(e.reshape(n, n), m, nb).ravel()
    return a
