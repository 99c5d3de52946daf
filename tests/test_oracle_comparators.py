"""Pins for the comparators of Sec. 4 (GIST for Eq. 1, Chambolle-Pock for the
few-view problem), each tied to something other than itself:

* GIST with beta = 0 is projected gradient descent on the weighted least
  squares term (the penalty's dual stays zero), checked against that textbook
  iteration on the dense system matrix.
* GIST with beta > 0 reaches the optimum of Eq. 1 that Algorithm 1 reaches
  (two different algorithms, one convex problem).
* Chambolle-Pock on consistent noiseless data drives Ax - b to zero with a TV
  no larger than the true image's, and its TV at convergence equals
  Algorithm 2's.
* The first Chambolle-Pock iterate from zero is P+(s t A^T b) in closed form.
* The step-size norms equal dense eigenvalues.
"""
import numpy as np
import pytest

from oracle import app as AP
from oracle import comparators as C
from oracle import projector as P
from oracle import tv as T


def _problem(seed, n=8, m=12, nb=12, noise=0.05):
    rng = np.random.default_rng(seed)
    xt = np.zeros((n, n))
    xt[2:6, 3:7] = 1.0
    xt[4:7, 1:3] = 0.5
    b = P.forward_project(xt, m, nb) + noise * rng.standard_normal((m, nb))
    w = rng.uniform(0.5, 2.0, (m, nb))
    return xt, b, w


def test_step_norms_match_dense_eigenvalues():
    n, m, nb = 8, 12, 12
    _, b, w = _problem(1, n, m, nb)
    a = P.dense_matrix(n, m, nb)
    st = C.gist_steps(w, n)
    ref = np.linalg.eigvalsh(a.T @ (w.ravel()[:, None] * a))[-1]
    assert st.norm == pytest.approx(ref, rel=1e-12)
    assert st.primal == pytest.approx(0.95 * 2.0 / ref, rel=1e-12)
    cs = C.cp_steps(n, m, nb)
    ref2 = np.linalg.eigvalsh(a.T @ a)[-1]
    assert cs.norm == pytest.approx(ref2, rel=1e-12)
    assert cs.primal == cs.dual == pytest.approx(0.95 / np.sqrt(ref2 + 8.0), rel=1e-12)


def test_gist_without_penalty_is_projected_gradient():
    n, m, nb = 8, 12, 12
    _, b, w = _problem(2, n, m, nb, noise=0.3)
    a = P.dense_matrix(n, m, nb)
    gamma = C.gist_steps(w, n).primal
    x, (v1, v2), _ = C.gist_lowdose(b, w, 0.0, n, 25, gamma)
    ref = np.zeros(n * n)
    for _ in range(25):
        ref = np.maximum(0.0, ref - gamma * (a.T @ (w.ravel() * (a @ ref - b.ravel()))))
    np.testing.assert_allclose(x.ravel(), ref, atol=1e-12)
    assert not v1.any() and not v2.any()


@pytest.mark.slow
def test_gist_reaches_the_algorithm1_optimum():
    n, m, nb = 8, 12, 12
    _, b, w = _problem(7, n, m, nb, noise=0.1)
    beta = 0.5
    gamma = C.gist_steps(w, n).primal
    xg, _, hist = C.gist_lowdose(b, w, beta, n, 6000, gamma,
                                 monitor=lambda x: AP.cost_lowdose(x, b, w, beta))
    res, _ = AP.lowdose_solve(b, w, beta, n, 600)
    f_app = AP.cost_lowdose(res.x, b, w, beta)
    assert abs(hist[-1] - f_app) <= 1e-7 * f_app
    np.testing.assert_allclose(xg, res.x, atol=2e-5)
    # and the cost went down along the way (first vs last hundred iterations)
    assert max(hist[-100:]) < min(hist[:100])


def test_cp_first_iterate_closed_form():
    n, m, nb = 10, 7, 15
    _, b, _ = _problem(3, n, m, nb)
    s, t = 0.013, 0.021
    x, (y1, q1, q2), _ = C.cp_fewview(b, n, 1, s, t)
    np.testing.assert_allclose(x, np.maximum(0.0, s * t * P.back_project(b, n)), atol=1e-14)
    np.testing.assert_allclose(y1, -s * b, atol=1e-15)
    assert not q1.any() and not q2.any()


@pytest.mark.slow
def test_cp_reaches_consistent_data_and_algorithm2_tv():
    n, m, nb = 16, 6, 24
    xt = np.zeros((n, n))
    xt[4:12, 5:11] = 1.0
    xt[7:10, 2:6] = 0.5
    b = P.forward_project(xt, m, nb)
    st = C.cp_steps(n, m, nb)
    x, _, _ = C.cp_fewview(b, n, 20000, st.dual, st.primal)
    assert AP.data_residual(x, b) < 1e-4
    assert x.min() >= 0.0
    assert T.tv_norm(x) <= T.tv_norm(xt) * (1 + 1e-3)
    res, _ = AP.fewview_solve(b, n, 3000)
    assert T.tv_norm(x) == pytest.approx(T.tv_norm(res.x), rel=2e-3)
