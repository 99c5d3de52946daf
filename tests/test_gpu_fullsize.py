"""Solver parity at the full 512 x 512 sizes, with the default set-up.

The FP64 oracle needs minutes to hours at these sizes (the operator norms at
720 views take tens of applications of A^T D A), so its values come from
``tests/golden/fullsize_512.json``, written by ``tests/golden/make_fullsize.py``
which calls only the oracle on the same seeded float32 inputs.  Each stored
iterate is 2048 seeded pixel samples plus whole-image scalars.

* Algorithm 1 on the 512^2 / 720 x 736 workload: the default set-up (kappa,
  tau, lambda_A by the first solve on the handle, the per-view lambda_h
  chains, sigma of Eq. 16) against the oracle's eigenvalues; x^3 at beta =
  1000, where the TV term moves the iterate by > 1e-2 relative (recorded by the
  generator), and x^20 at the workload's beta = 0.005 -- the trajectory the
  benchmark times -- on the second solve, which reuses the cached lambda_A.
* Algorithm 2 on the 512^2 / 32 x 736 noiseless workload: default sigma and
  tau, x^3 and x^20.
* The error-tolerant few-view solve on the same data (eps = 1e-4 ||b||, the
  ball binding after a few iterations): default sigma (the split norm
  lambda_max(K^T D(1) K)) and tau, x^3 and x^20.

Bars: step sizes 1e-6 (tau and kappa 1e-12 where they are closed forms),
sampled x^k relative l2 1e-4, ||x^k|| 1e-4, the Eq. 1 cost (or psi) 1e-5.
"""
import json
import os

import numpy as np
import pytest
import torch

from paper_1609_06041_amd import ctpd
from paper_1609_06041_amd import synth as S

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_512.json")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


def check_inputs(b, w, sums):
    # the stored values belong to these exact float32 inputs
    assert float(b.sum()) == pytest.approx(sums["b_sum"], rel=1e-12)
    assert float((b * b).sum()) == pytest.approx(sums["b_sumsq"], rel=1e-12)
    if w is not None:
        assert float(w.sum()) == pytest.approx(sums["w_sum"], rel=1e-12)
        assert float((1.0 / w).sum()) == pytest.approx(sums["winv_sum"], rel=1e-12)


def compare_iterate(parity, x, case, idx, what):
    parity(f"{what} x samples", rel(x.ravel()[idx], np.array(case["x_samples"])), 1e-4)
    parity(f"{what} ||x||", abs(np.linalg.norm(x) - case["x_norm"]) / case["x_norm"], 1e-4)


def test_lowdose_full_size_default_setup(gpu, parity, golden):
    g = golden["lowdose_512"]
    idx = np.array(golden["sample_indices"])
    prob, spec = S.workload_problem("lowdose_512", problem_id=0, with_x_true=False)
    b32, w32 = S.as_f32_inputs(prob)
    check_inputs(b32.astype(np.float64), w32.astype(np.float64), g["inputs"])
    tv, bench = g["cases"]
    assert tv["rel_diff_vs_beta0"] >= 100 * 1e-4   # the TV term acts at this beta
    st = g["steps"]
    n, m, nb = spec["n"], spec["m"], spec["nb"]
    b, w = torch.from_numpy(b32).cuda(), torch.from_numpy(w32).cuda()
    with ctpd.Operator(n, m, nb) as op:
        x, info = op.lowdose_solve(b, w, tv["beta"], tv["iters"], record_cost=True)
        x = x.cpu().numpy().astype(np.float64)
        assert info["norm_steps_a"] > 0   # the first solve computes lambda_A
        assert info["kappa"] == pytest.approx(st["kappa"], rel=1e-12)
        assert info["tau"] == pytest.approx(st["tau"], rel=1e-12)
        parity("lambda_A", abs(info["lambda_a"] - st["lambda_a"]) / st["lambda_a"], 1e-6)
        parity("lambda_h", abs(info["lambda_h"] - st["lambda_h"]) / st["lambda_h"], 1e-6)
        parity("sigma", abs(info["sigma"] - st["sigma"]) / st["sigma"], 1e-6)
        compare_iterate(parity, x, tv, idx, f"beta={tv['beta']:g} k={tv['iters']}")
        parity("cost", abs(info["cost"][-1] - tv["cost"]) / tv["cost"], 1e-5)
        # the benchmark's trajectory, with lambda_A from the handle's cache
        x, info = op.lowdose_solve(b, w, bench["beta"], bench["iters"], record_cost=True)
        x = x.cpu().numpy().astype(np.float64)
        assert info["norm_steps_a"] == 0
        parity("sigma (cached lambda_A)", abs(info["sigma"] - st["sigma"]) / st["sigma"], 1e-6)
        compare_iterate(parity, x, bench, idx, f"beta={bench['beta']:g} k={bench['iters']}")
        parity("cost", abs(info["cost"][-1] - bench["cost"]) / bench["cost"], 1e-5)


def test_fewview_full_size_default_setup(gpu, parity, golden):
    g = golden["fewview_512"]
    idx = np.array(golden["sample_indices"])
    prob, spec = S.workload_problem("fewview_512", problem_id=0, with_x_true=False)
    b32, _ = S.as_f32_inputs(prob)
    check_inputs(b32.astype(np.float64), None, g["inputs"])
    n, m, nb = spec["n"], spec["m"], spec["nb"]
    b = torch.from_numpy(b32).cuda()
    with ctpd.Operator(n, m, nb) as op:
        for case in g["cases"]:
            x, info = op.fewview_solve(b, case["iters"], record_cost=True, monitors=("resid",))
            x = x.cpu().numpy().astype(np.float64)
            parity("sigma", abs(info["sigma"] - g["sigma"]) / g["sigma"], 1e-6)
            parity("tau", abs(info["tau"] - g["tau"]) / g["tau"], 1e-6)
            compare_iterate(parity, x, case, idx, f"k={case['iters']}")
            parity("psi", abs(info["cost"][-1] - case["psi"]) / case["psi"], 1e-5)
            parity("||Ax-b||/||b||", abs(info["resid"][-1] - case["resid"]) / case["resid"], 1e-4)


def test_fewview_eps_full_size_default_setup(gpu, parity, golden):
    g = golden["fewview_eps_512"]
    idx = np.array(golden["sample_indices"])
    prob, spec = S.workload_problem("fewview_512", problem_id=0, with_x_true=False)
    b32, _ = S.as_f32_inputs(prob)
    check_inputs(b32.astype(np.float64), None, g["inputs"])
    n, m, nb = spec["n"], spec["m"], spec["nb"]
    b = torch.from_numpy(b32).cuda()
    with ctpd.Operator(n, m, nb) as op:
        for case in g["cases"]:
            x, info = op.fewview_eps_solve(b, g["eps"], case["iters"], record_cost=True, monitors=("resid",))
            x = x.cpu().numpy().astype(np.float64)
            parity("sigma", abs(info["sigma"] - g["sigma"]) / g["sigma"], 1e-6)
            parity("tau", abs(info["tau"] - g["tau"]) / g["tau"], 1e-6)
            compare_iterate(parity, x, case, idx, f"eps k={case['iters']}")
            parity("psi", abs(info["cost"][-1] - case["psi"]) / case["psi"], 1e-5)
            parity("||Ax-b||/||b||", abs(info["resid"][-1] - case["resid"]) / case["resid"], 1e-4)
