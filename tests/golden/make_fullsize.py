"""Writes ``fullsize_512.json``: FP64 oracle values for the GPU parity tests at
the full 512 x 512 sizes, where the oracle takes minutes to hours (the
operator norms at 720 views need tens of applications of A^T D A at ~25 s
each), too long to run inside a GPU test.

It calls only the oracle (``oracle/``) and the seeded input generator, on the
same float32 inputs the GPU receives:

* lowdose_512 (512^2, 720 views x 736 bins, problem 0): the default set-up of
  Algorithm 1 (kappa, tau = 0.3 pi kappa / (2m), lambda_A, lambda_h, sigma;
  Eq. 16), then x^3 at a TV weight large enough that the TV term moves the
  iterate (beta = 1000: x^3 differs from the beta = 0 iterate by > 1e-2
  relative, recorded), and x^20 at the workload's beta = 0.005 (the
  trajectory the benchmark times);
* fewview_512 (512^2, 32 views x 736 bins, noiseless, problem 0): the default
  set-up of Algorithm 2 (sigma = rho / lambda_max(A^T D(1) A), tau = mean
  |sigma A^T D(1) b|), then x^3 and x^20.

* fewview_eps_512 (the same data): the error-tolerant few-view iteration
  (min psi s.t. ||Ax - b|| <= eps, x >= 0, eps = 1e-4 ||b||: with one tau for
  both blocks y moves by about 3e-4 ||b|| in 20 iterations, so the ball binds
  from a few iterations on only at a small eps) with its
  default set-up (sigma = rho / lambda_max(K^T D(1) K), K = [A, -I], and the
  default tau), then x^3 and x^20.

Each iterate is stored as 2048 seeded pixel samples plus whole-image scalars
(norm, psi of Eq. 2, the Eq. 1 cost or ||Ax - b|| / ||b||).  Run from the
repository root:

    python tests/golden/make_fullsize.py            # everything (about 45 minutes)
    python tests/golden/make_fullsize.py --only eps # recompute fewview_eps_512 only
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "fullsize_512.json")
N_SAMPLES = 2048
BETA_TV = 1000.0


def sample_indices(n: int) -> np.ndarray:
    rng = np.random.default_rng(np.random.SeedSequence([512, 2048]))
    return np.sort(rng.choice(n * n, size=N_SAMPLES, replace=False))


def inputs(name: str):
    from paper_1609_06041_amd import synth as S
    prob, spec = S.workload_problem(name, problem_id=0, with_x_true=False)
    b32, w32 = S.as_f32_inputs(prob)
    b = b32.astype(np.float64)
    w = None if w32 is None else w32.astype(np.float64)
    sums = {"b_sum": float(b.sum()), "b_sumsq": float((b * b).sum())}
    if w is not None:
        sums["w_sum"] = float(w.sum())
        sums["winv_sum"] = float((1.0 / w).sum())
    return b, w, spec, sums


def describe(x: np.ndarray, idx: np.ndarray) -> dict:
    from oracle import tv as OT
    return {"x_samples": [float(f"{v:.10g}") for v in x.ravel()[idx]], "x_norm": float(np.linalg.norm(x)),
            "psi": OT.tv_norm(x)}


def lowdose_steps():
    from oracle import app as OA
    b, w, spec, sums = inputs("lowdose_512")
    t0 = time.time()
    st = OA.steps_lowdose(w, spec["n"])
    return {"inputs": sums, "kappa": st.kappa, "tau": st.tau, "lambda_a": st.lambda_a, "lambda_h": st.lambda_h,
            "sigma": st.sigma, "seconds": time.time() - t0}


def lowdose_run(beta: float, iters: int, tau: float, sigma: float):
    from oracle import app as OA
    b, w, spec, _ = inputs("lowdose_512")
    idx = sample_indices(spec["n"])
    res, _ = OA.lowdose_solve(b, w, beta, spec["n"], iters, tau=tau, sigma=sigma)
    out = describe(res.x, idx)
    out.update({"beta": beta, "iters": iters, "cost": OA.cost_lowdose(res.x, b, w, beta)})
    return out, res.x


def fewview_all():
    from oracle import app as OA
    b, _, spec, sums = inputs("fewview_512")
    n = spec["n"]
    idx = sample_indices(n)
    t0 = time.time()
    st = OA.steps_fewview(b, n)
    snaps = {}

    def monitor(x, mu):
        snaps[len(snaps) + 1] = x.copy()
        return 0.0

    m, nb = b.shape
    from oracle.filters import ramp_taps
    res = OA.app_solve(b, n, 20, st.tau, st.sigma, ramp_taps(nb, m, st.tau), beta=1.0, winv=None,
                       monitor=monitor)
    cases = []
    for k in (3, 20):
        x = snaps[k]
        c = describe(x, idx)
        c.update({"iters": k, "resid": OA.data_residual(x, b)})
        cases.append(c)
    assert np.array_equal(snaps[20], res.x)
    return {"inputs": sums, "tau": st.tau, "sigma": st.sigma, "lambda_a1": st.lambda_a * st.tau, "cases": cases,
            "seconds": time.time() - t0}


EPS_FRAC = 1e-4


def fewview_eps_all():
    from oracle import app as OA
    b, _, spec, sums = inputs("fewview_512")
    n = spec["n"]
    idx = sample_indices(n)
    t0 = time.time()
    eps = EPS_FRAC * float(np.linalg.norm(b))
    st = OA.steps_fewview_eps(b, n)
    snaps = {}

    def monitor(x, y, mu):
        snaps[len(snaps) + 1] = (x.copy(), float(np.linalg.norm(y - b)))
        return 0.0

    OA.fewview_eps_solve(b, n, eps, 20, tau=st.tau, sigma=st.sigma, monitor=monitor)
    cases = []
    for k in (3, 20):
        x, ydist = snaps[k]
        c = describe(x, idx)
        c.update({"iters": k, "resid": OA.data_residual(x, b), "y_dist": ydist})
        cases.append(c)
    return {"inputs": sums, "eps_frac": EPS_FRAC, "eps": eps, "tau": st.tau, "sigma": st.sigma,
            "lambda_split1": st.lambda_a * st.tau, "cases": cases, "seconds": time.time() - t0}


def main() -> int:
    t0 = time.time()
    if "--only" in sys.argv and sys.argv[-1] == "eps":
        with open(OUT) as f:
            doc = json.load(f)
        doc["fewview_eps_512"] = fewview_eps_all()
        with open(OUT, "w") as f:
            json.dump(doc, f, indent=1)
        print(f"updated {OUT} in {time.time() - t0:.0f} s", flush=True)
        return 0
    with cf.ProcessPoolExecutor(max_workers=4) as ex:
        fv = ex.submit(fewview_all)
        steps = lowdose_steps()
        print(f"lowdose steps in {steps['seconds']:.0f} s: {steps}", flush=True)
        tau, sigma = steps["tau"], steps["sigma"]
        jobs = {"tv": ex.submit(lowdose_run, BETA_TV, 3, tau, sigma),
                "tv0": ex.submit(lowdose_run, 0.0, 3, tau, sigma),
                "bench": ex.submit(lowdose_run, 0.005, 20, tau, sigma)}
        (tv, x_tv), (_, x_tv0), (bench, _) = jobs["tv"].result(), jobs["tv0"].result(), jobs["bench"].result()
        tv["rel_diff_vs_beta0"] = float(np.linalg.norm(x_tv - x_tv0) / np.linalg.norm(x_tv0))
        fewview = fv.result()
        fewview_eps = fewview_eps_all()
    doc = {
        "generator": "tests/golden/make_fullsize.py: FP64 oracle (oracle/) on the seeded float32 inputs",
        "n_samples": N_SAMPLES,
        "sample_indices": [int(i) for i in sample_indices(512)],
        "lowdose_512": {"steps": {k: v for k, v in steps.items() if k != "inputs"}, "inputs": steps["inputs"],
                        "cases": [tv, bench]},
        "fewview_512": fewview,
        "fewview_eps_512": fewview_eps,
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
