"""Seeded synthetic inputs: ellipse phantoms, their exact parallel-beam line
integrals, and transmission Poisson noise.

This module produces the data both the HIP path and the FP64 oracle consume.
It holds none of the reconstruction method's arithmetic (no projector,
filter, TV or primal-dual step): only the continuous object model and the
measurement model the paper's simulations use (Sec. 4: parallel-beam data
with transmission Poisson noise; Sec. 2.1: b is a vector of point samples of
the continuous projection p(r, theta)).

Conventions shared with the rest of the package:

* image x is N x N, row-major ``x[iy, ix]``, unit pixels, pixel centre
  ``(ix - (N-1)/2, iy - (N-1)/2)``;
* sinogram is view-major ``[m, nb]``, view v at angle ``theta_v = v*pi/m``,
  bin u at signed distance ``r_u = u - (nb-1)/2``;
* the ray of (v, u) is the line ``x cos(theta) + y sin(theta) = r_u``.

Attenuation scale: an ellipse of density rho contributes ``rho / N`` per unit
length, i.e. densities are per field-of-view width, which keeps line
integrals O(1) at every image size (the paper gives no phantom values).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Ellipse:
    x0: float
    y0: float
    a: float
    b: float
    alpha: float
    rho: float


@dataclass
class Problem:
    """One synthetic reconstruction problem (all arrays float64 unless noted)."""

    n: int
    m: int
    nb: int
    ellipses: list = field(default_factory=list)
    b_true: np.ndarray | None = None   # exact line integrals [m, nb]
    b: np.ndarray | None = None        # measured (noisy) data [m, nb]
    w: np.ndarray | None = None        # statistical weights = counts [m, nb] (None: noiseless)
    x_true: np.ndarray | None = None   # rasterised phantom [n, n]
    i0: float | None = None


def rng_for(config_id: int, problem_id: int, stream: int) -> np.random.Generator:
    """Independent, reproducible stream: 0 = phantom, 1 = noise."""
    return np.random.default_rng(np.random.SeedSequence([config_id, problem_id, stream]))


def draw_ellipses(n: int, count: int, rng: np.random.Generator) -> list:
    """Draw ``count`` ellipses with ranges scaled from a 64-pixel reference grid.

    centre ~ U[-24s, 24s]^2, semi-axes ~ U[3s, 20s], angle ~ U[0, pi),
    density ~ U[0, 1], with s = n/64.  An ellipse whose bounding circle leaves
    the disk of radius n/2 - 1 is redrawn, so every ray meeting the object
    also meets the pixel grid.
    """
    if n < 3:   # the smallest ellipse (semi-axis 3n/64) only fits inside radius n/2 - 1 from n = 3 on
        raise ValueError(f"ellipse phantoms need n >= 3, got {n}")
    s = n / 64.0
    out = []
    while len(out) < count:
        x0, y0 = rng.uniform(-24 * s, 24 * s, size=2)
        a, b = rng.uniform(3 * s, 20 * s, size=2)
        alpha = rng.uniform(0.0, math.pi)
        rho = rng.uniform(0.0, 1.0)
        if math.hypot(x0, y0) + max(a, b) > n / 2.0 - 1.0:
            continue
        out.append(Ellipse(float(x0), float(y0), float(a), float(b), float(alpha), float(rho)))
    return out


def line_integrals(ellipses: list, n: int, m: int, nb: int, angles=None) -> np.ndarray:
    """Exact line integrals of the ellipse sum along every (view, bin) ray.

    For an ellipse with semi-axes (a, b) rotated by alpha and centred at
    (x0, y0), the chord along ``x cos t + y sin t = r`` has length
    ``2 a b sqrt(s2 - d^2) / s2`` with ``s2 = a^2 cos^2(t-alpha) + b^2 sin^2(t-alpha)``
    and ``d = r - x0 cos t - y0 sin t`` (zero when d^2 >= s2).
    """
    th = np.arange(m, dtype=np.float64) * (math.pi / m) if angles is None else np.asarray(angles, np.float64)
    r = np.arange(nb, dtype=np.float64) - (nb - 1) / 2.0
    c, s = np.cos(th)[:, None], np.sin(th)[:, None]
    out = np.zeros((th.size, nb))
    scale = 1.0 / n
    for e in ellipses:
        ca, sa = np.cos(th - e.alpha)[:, None], np.sin(th - e.alpha)[:, None]
        s2 = (e.a * ca) ** 2 + (e.b * sa) ** 2
        d = r[None, :] - e.x0 * c - e.y0 * s
        inside = np.maximum(s2 - d * d, 0.0)
        out += scale * e.rho * 2.0 * e.a * e.b * np.sqrt(inside) / s2
    return out


def rasterise(ellipses: list, n: int, sub: int = 8) -> np.ndarray:
    """Mean of ``sub x sub`` point samples of the ellipse sum inside each pixel."""
    c = np.arange(n, dtype=np.float64) - (n - 1) / 2.0
    off = (np.arange(sub, dtype=np.float64) + 0.5) / sub - 0.5
    img = np.zeros((n, n))
    for oy in off:
        yy = (c + oy)[:, None]
        for ox in off:
            xx = (c + ox)[None, :]
            acc = np.zeros((n, n))
            for e in ellipses:
                ca, sa = math.cos(e.alpha), math.sin(e.alpha)
                u = (xx - e.x0) * ca + (yy - e.y0) * sa
                v = -(xx - e.x0) * sa + (yy - e.y0) * ca
                acc += e.rho * (((u / e.a) ** 2 + (v / e.b) ** 2) <= 1.0)
            img += acc
    return np.maximum(img / (sub * sub), 0.0) / n


def poisson_data(b_true: np.ndarray, i0: float, rng: np.random.Generator):
    """Transmission Poisson measurement: counts ~ Poisson(I0 exp(-b_true)).

    Zero counts are raised to one before the log so b and 1/w stay finite.
    Returns ``(b, w)`` with ``b = -log(counts/I0)`` and ``w = counts``.
    """
    counts = rng.poisson(i0 * np.exp(-b_true)).astype(np.float64)
    counts = np.maximum(counts, 1.0)
    return -np.log(counts / i0), counts


def make_problem(config_id: int, problem_id: int, n: int, m: int, nb: int,
                 n_ellipses: int, i0: float | None, with_x_true: bool = True) -> Problem:
    """Build one seeded problem.  ``i0=None`` gives noiseless data (w=None)."""
    ells = draw_ellipses(n, n_ellipses, rng_for(config_id, problem_id, 0))
    bt = line_integrals(ells, n, m, nb)
    prob = Problem(n=n, m=m, nb=nb, ellipses=ells, b_true=bt, i0=i0)
    if i0 is None:
        prob.b = bt.copy()
    else:
        prob.b, prob.w = poisson_data(bt, i0, rng_for(config_id, problem_id, 1))
    if with_x_true:
        prob.x_true = rasterise(ells, n)
    return prob


# Workload definitions (sizes follow the paper's two experiments, Sec. 4,
# rescaled to synthetic ellipse phantoms).
WORKLOADS = {
    "lowdose_64": dict(config_id=0, n=64, m=90, nb=96, n_ellipses=8, i0=1e4, beta=0.01, iters=50),
    "lowdose_512": dict(config_id=1, n=512, m=720, nb=736, n_ellipses=20, i0=5e4, beta=0.005, iters=20),
    "fewview_512": dict(config_id=2, n=512, m=32, nb=736, n_ellipses=20, i0=None, beta=None, iters=3),
}


# The batched uneven workload: independent low-dose problems whose image side
# N, view count m, phantom size and dose are drawn per problem; nb = ceil(1.42 N)
# so the detector covers the image diagonal.
BATCH_SIDES = (256, 384, 512)
BATCH_VIEWS = (32, 90, 360, 720)


def batch_spec(problem_id: int, config_id: int = 3) -> dict:
    rng = rng_for(config_id, problem_id, 2)
    n = int(BATCH_SIDES[rng.integers(len(BATCH_SIDES))])
    m = int(BATCH_VIEWS[rng.integers(len(BATCH_VIEWS))])
    return dict(config_id=config_id, problem_id=problem_id, n=n, m=m, nb=int(math.ceil(1.42 * n)),
                n_ellipses=int(rng.integers(10, 21)), i0=float(rng.uniform(1e4, 1e5)), beta=0.005, iters=20)


def batch_problem(problem_id: int, config_id: int = 3, with_x_true: bool = False) -> tuple[Problem, dict]:
    spec = batch_spec(problem_id, config_id)
    prob = make_problem(config_id, problem_id, spec["n"], spec["m"], spec["nb"], spec["n_ellipses"], spec["i0"],
                        with_x_true=with_x_true)
    return prob, spec


def workload_problem(name: str, problem_id: int = 0, with_x_true: bool = True) -> tuple[Problem, dict]:
    spec = dict(WORKLOADS[name])
    prob = make_problem(spec["config_id"], problem_id, spec["n"], spec["m"], spec["nb"],
                        spec["n_ellipses"], spec["i0"], with_x_true=with_x_true)
    return prob, spec


def as_f32_inputs(prob: Problem):
    """The exact float32 arrays the GPU receives, and their float64 images for the oracle."""
    b32 = np.ascontiguousarray(prob.b, dtype=np.float32)
    w32 = None if prob.w is None else np.ascontiguousarray(prob.w, dtype=np.float32)
    return b32, w32
