"""GPU parity of the comparators (GIST for Eq. 1, Chambolle-Pock for the
few-view problem) against the FP64 oracle, through the C ABI.

Same bars as the APP solvers: iterate x^k relative l2 <= 1e-4, recorded
cost relative <= 3e-5 per iteration, step sizes from the GPU's float64
Lanczos within 1e-6 of the oracle's eigenvalues.
"""
import numpy as np
import pytest
import torch

from oracle import app as OA
from oracle import comparators as OC
from oracle import tv as OT
from paper_1609_06041_amd import ctpd
from paper_1609_06041_amd import synth as S

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def max_rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b) / np.abs(b)))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def lowdose_inputs(n, m, nb, seed, n_ell=8, i0=1e4):
    prob = S.make_problem(93, seed, n, m, nb, n_ell, i0, with_x_true=False)
    b32, w32 = S.as_f32_inputs(prob)
    return b32.astype(np.float64), w32.astype(np.float64)


@pytest.mark.parametrize("n,m,nb,beta,iters", [(64, 90, 96, 0.01, 100), (45, 30, 70, 0.05, 40),
                                               (33, 17, 49, 0.0, 30)])
def test_gist_matches_oracle(gpu, parity, n, m, nb, beta, iters):
    b, w = lowdose_inputs(n, m, nb, seed=n + m)
    st = OC.gist_steps(w, n)
    ref, (v1, v2), hist = OC.gist_lowdose(b, w, beta, n, iters, st.primal,
                                          monitor=lambda x: OA.cost_lowdose(x, b, w, beta))
    with ctpd.Operator(n, m, nb) as op:
        x, info = op.gist_lowdose_solve(dev(b), dev(w), beta, iters, record_cost=True, return_state=True)
        x, v = host(x), host(info["p"])
    assert info["lambda_a"] == pytest.approx(st.norm, rel=1e-6)
    assert info["tau"] == pytest.approx(st.primal, rel=1e-6)
    assert info["sigma"] == pytest.approx(OC.GIST_LAM)
    parity("x", rel(x, ref), 1e-4)
    if beta > 0:
        parity("v", rel(v, np.stack([v1, v2])), 1e-4)
    parity("cost history (max rel)", max_rel(info["cost"], hist), 3e-5)
    assert x.min() >= 0.0


@pytest.mark.parametrize("n,m,nb,iters", [(64, 32, 96, 60), (50, 12, 75, 30)])
def test_chambolle_pock_matches_oracle(gpu, parity, n, m, nb, iters):
    prob = S.make_problem(94, n, n, m, nb, 8, None, with_x_true=False)
    b = np.asarray(prob.b, np.float32).astype(np.float64)
    st = OC.cp_steps(n, m, nb)
    ref, (y1, q1, q2), hist = OC.cp_fewview(b, n, iters, st.dual, st.primal, monitor=OT.tv_norm)
    with ctpd.Operator(n, m, nb) as op:
        x, info = op.cp_fewview_solve(dev(b), iters, record_cost=True, return_state=True)
        x, y, q = host(x), host(info["mu"]), host(info["p"])
    assert info["lambda_a"] == pytest.approx(st.norm, rel=1e-6)
    assert info["tau"] == pytest.approx(st.primal, rel=1e-6)
    assert info["sigma"] == pytest.approx(st.dual, rel=1e-6)
    parity("x", rel(x, ref), 1e-4)
    parity("y", rel(y, y1), 1e-4)
    parity("q", rel(q, np.stack([q1, q2])), 1e-4)
    parity("cost history (max rel)", max_rel(info["cost"], hist), 3e-5)


def test_gist_full_size_first_iterations(gpu, parity):
    n, m, nb = 512, 720, 736
    prob, spec = S.workload_problem("lowdose_512", with_x_true=False)
    b32, w32 = S.as_f32_inputs(prob)
    b, w = b32.astype(np.float64), w32.astype(np.float64)
    gamma, beta = 4e-11, 50.0   # fixed steps (no full-size eigenvalue); beta large enough that TV acts
    ref, _, _ = OC.gist_lowdose(b, w, beta, n, 2, gamma)
    with ctpd.Operator(n, m, nb) as op:
        x, _ = op.gist_lowdose_solve(dev(b), dev(w), beta, 2, gamma=gamma)
        x = host(x)
    parity("x", rel(x, ref), 1e-4)


def test_chambolle_pock_full_size_first_iterations(gpu, parity):
    n, m, nb = 512, 32, 736
    prob, _ = S.workload_problem("fewview_512", with_x_true=False)
    b = np.asarray(prob.b, np.float32).astype(np.float64)
    s = t = 2e-3
    ref, _, _ = OC.cp_fewview(b, n, 3, s, t)
    with ctpd.Operator(n, m, nb) as op:
        x, _ = op.cp_fewview_solve(dev(b), 3, t=t, s=s)
        x = host(x)
    parity("x", rel(x, ref), 1e-4)


def test_gist_rejects_bad_dual_step(gpu):
    n, m, nb = 16, 8, 24
    b, w = lowdose_inputs(n, m, nb, seed=4)
    with ctpd.Operator(n, m, nb) as op:
        with pytest.raises(ctpd.CtpdError) as e:
            op.gist_lowdose_solve(dev(b), dev(w), 0.1, 3, lam=0.2)
        assert e.value.code == ctpd.CTPD_EINVAL
        w_bad = w.copy()
        w_bad[0, 0] = -1.0
        with pytest.raises(ctpd.CtpdError) as e:
            op.gist_lowdose_solve(dev(b), dev(w_bad), 0.1, 3)
        assert e.value.code == ctpd.CTPD_EDOMAIN


@pytest.mark.parametrize("n,m,nb,beta,iters", [(64, 90, 96, 0.01, 40), (45, 30, 70, 0.0, 25)])
def test_app_identity_matches_oracle(gpu, parity, n, m, nb, beta, iters):
    # Algorithm 1 with D = I (the ablation without the preconditioner)
    b, w = lowdose_inputs(n, m, nb, seed=2 * n + m)
    ref, st = OA.lowdose_identity_solve(b, w, beta, n, iters, record_cost=True)
    with ctpd.Operator(n, m, nb) as op:
        x, info = op.app_identity_lowdose_solve(dev(b), dev(w), beta, iters, record_cost=True)
        x = host(x)
        x2, _ = op.app_identity_lowdose_solve(dev(b), dev(w), beta, iters)   # fused filter inputs
        x2 = host(x2)
    assert info["lambda_a"] == pytest.approx(st.lambda_a, rel=1e-6)
    assert info["lambda_h"] == pytest.approx(st.lambda_h, rel=1e-12)
    assert info["tau"] == pytest.approx(st.tau, rel=1e-6)
    assert info["sigma"] == pytest.approx(st.sigma, rel=1e-6)
    parity("x", rel(x, ref.x), 1e-4)
    parity("cost history (max rel)", max_rel(info["cost"], ref.history), 3e-5)
    np.testing.assert_array_equal(x2, x)
