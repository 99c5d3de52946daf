#!/usr/bin/env python3
"""Throughput of the FBP-preconditioned APP reconstruction on one MI355X.

Workload (lowdose_512): 512 x 512 image, 720 views over [0, pi) x 736 bins,
seeded 20-ellipse phantom, exact line integrals with transmission Poisson
noise (I0 = 5e4), beta = 0.005, 20 iterations of Algorithm 1.

One step = one complete ``pd_lowdose_solve`` call on the next of three
independent inputs (phantom and noise draws): set-up (kappa, W^-1, taps, the
float64 Lanczos norm lambda_h of the data, step sizes) plus 20 iterations,
inputs resident in HBM.  kappa * lambda_A is a property of the geometry at the
default tau; the handle computes it at its first solve (reported as
``setup_ms_cold``, in the warm-up) and reuses it.  ``value`` = PD iterations
per second over the whole job (20 * steps / elapsed).  Also reported: the iteration loop alone, A and A^T
throughput in G(pixel, view) updates/s, the filter's matrix-core rate, the
TV step's bandwidth, the roofline of the dominant kernel (A, the forward
projector; A^T's is reported beside it), and the FP64 oracle timed on the host
on a bounded sample of the same workload (one BLAS thread, then all host
cores).

The same line carries the rest of the metric: the few-view workload (512^2,
32 views: A, A^T and Algorithm-2 iterations/s), the batched uneven workload
(64 problems of 256^2-512^2 and 32-720 views solved as one batch vs one after
another) and the unrolled differentiable solve (16 x 256^2, 180 views, 10
iterations, forward + reverse pass for all problems in one call vs one problem
at a time, and vs 16 plain solves).

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu-baseline] [--no-extras]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X FP32 vector peak: 256 CU x 128 FMA lanes x 2.4 GHz x 2 FLOP = 157.3
# TFLOP/s.  gfx950 issues plain (non-packed) v_fma_f32 at more than 64 lanes a
# CU per clock (a register-only FMA loop reaches 95 TFLOP/s), so this is the
# peak even though no kernel here uses packed FP32 instructions.
PEAK_FP32_VECTOR_TFLOPS = 157.3
# Algorithmic FLOP per (pixel, view) update of A^T: bin coordinate
# t = X cos + Y sin + c (2 FMA = 4), its fraction (1), the two hat weights
# max(0, len -+ f len2 ...) (2 x (FMA + max) = 6), the two weighted taps
# accumulated (2 FMA = 4).
AT_FLOP_PER_UPDATE = 15.0
# Algorithmic FLOP per in-image ray step of A: sample position
# s = s0 + u su + t st (2 FMA = 4), its fraction (1), the interpolation
# a + f (b - a) (sub + FMA = 3), the accumulation (1).
A_FLOP_PER_STEP = 9.0
PEAK_FP32_MFMA_TFLOPS = 157.3
# The filter forms each FP32 product from 6 bf16 term products on the bf16
# matrix cores (dense peak 2500 TFLOP/s), so its FP32-equivalent peak is
# 2500 / 6.
PEAK_BF16_MFMA_TFLOPS = 2500.0
FILTER_TERM_PRODUCTS = 6
PEAK_FILTER_TFLOPS = PEAK_BF16_MFMA_TFLOPS / FILTER_TERM_PRODUCTS
PEAK_HBM_GBS = 8000.0
N_INSTANCES = 3   # independent inputs cycled through by the timed solves
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "lowdose512_kernels_traffic.md")
# the source file of each kernel whose HBM traffic the counter summary records
KERNEL_SOURCES = {"forward": "projector.hip", "adjoint": "projector.hip", "filter": "filter.hip", "tv": "tv.hip"}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash(kernel: str) -> str:
    src = os.path.join(ROOT, "paper_1609_06041_amd", "csrc", KERNEL_SOURCES[kernel])
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def forward_ray_steps(n: int, m: int, nb: int) -> int:
    """In-image (ray, step) pairs of the Joseph forward projector: the steps t of
    ray (v, u) whose sample s(t, u) = s0 + u su + t st lies in (-1, n), i.e. that
    have a nonzero tap (views at v pi / m; row views step over rows)."""
    import numpy as np
    c, cd = 0.5 * (n - 1), 0.5 * (nb - 1)
    u = np.arange(nb, dtype=np.float64)
    total = 0
    for v in range(m):
        th = v * np.pi / m
        cs, sn = np.cos(th), np.sin(th)
        row = 4 * v <= m or 4 * v >= 3 * m
        a, o = (cs, sn) if row else (sn, cs)
        base = (c * o - cd) / a + c + u / a
        st = -o / a
        if st == 0.0:
            total += int(np.count_nonzero((base > -1.0) & (base < n))) * n
            continue
        t1, t2 = (-1.0 - base) / st, (n - base) / st
        lo, hi = np.minimum(t1, t2), np.maximum(t1, t2)
        first = np.maximum(np.floor(lo) + 1, 0)
        last = np.minimum(np.ceil(hi) - 1, n - 1)
        total += int(np.clip(last - first + 1, 0, None).sum())
    return total


def read_traffic(kernel: str):
    """HBM bytes per launch of `kernel` ("forward", "adjoint", "filter", "tv") from
    the committed rocprofv3 counter summary, if it was taken on the kernel's
    current source file."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get(f"{kernel}_source_sha256_16") != kernel_source_hash(kernel):
        return None
    try:
        return float(vals[f"{kernel}_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_op(fn, stream, reps: int, warm: int = 5) -> float:
    """Average ms per call from HIP events recorded on the op's stream."""
    import torch
    for _ in range(warm):
        fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_baseline(b64, w64, beta, n, m, nb, tau, sigma, stride: int = 4, threads: int = 1) -> dict:
    """The FP64 oracle, as it stands, timed for one Algorithm-1 iteration of the
    same workload on a bounded sample: A and A^T over every ``stride``-th view
    (scaled by ``stride``), D, the TV prox and the pointwise steps in full.
    ``threads`` caps the BLAS thread pool; only the filter's matrix product
    uses it (the projector and TV loops are single-threaded NumPy)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import filters as OF
    from oracle import projector as OP
    from oracle import tv as OT

    views = list(range(0, m, stride))
    winv = 1.0 / w64
    kappa = float(winv.mean())
    rng = np.random.default_rng(0)
    x = np.abs(rng.standard_normal((n, n))) * 1e-3
    mu = 1e-3 * rng.standard_normal((m, nb))
    mup = 1e-3 * rng.standard_normal((m, nb))
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        h = OF.smoothed_ramp_taps(nb, m, tau, kappa)
        t_taps = time.perf_counter() - t0
        t0 = time.perf_counter()
        mubar = 2 * mu - mup - sigma * OF.apply_filter(winv * (mu - mup), h)
        t_d1 = time.perf_counter() - t0
        t0 = time.perf_counter()
        z = x - tau * OP.back_project(mubar[views], n, m=m, views=views)
        t_at = (time.perf_counter() - t0) * stride
        t0 = time.perf_counter()
        x1, _, _ = OT.tv_prox(z, tau * beta, n_iter=10)
        t_tv = time.perf_counter() - t0
        t0 = time.perf_counter()
        q = OP.forward_project(x1, m, nb, views=views)
        t_a = (time.perf_counter() - t0) * stride
        t0 = time.perf_counter()
        _ = mu + sigma * OF.apply_filter(np.zeros((m, nb)) - b64 - winv * mu, h)
        t_d2 = time.perf_counter() - t0
    it_s = t_d1 + t_at + t_tv + t_a + t_d2
    return {
        "value": 1.0 / it_s, "unit": "PD iters/s", "cores": threads, "kind": "oracle",
        "sample": (f"one Algorithm-1 iteration of the same 512^2/720x736 workload in float64 NumPy, "
                   f"{threads} BLAS thread(s): A and A^T on every {stride}th view ({len(views)} of {m}) "
                   f"scaled x{stride}, D twice, 10 TV steps and the pointwise steps in full"),
        "seconds_per_iteration": it_s,
        "parts_s": {"A": t_a, "AT": t_at, "D": t_d1 + t_d2, "tv_prox": t_tv, "taps_setup": t_taps},
        "host_cpus": os.cpu_count(),
    }


def compare(dev) -> int:
    """Iterations of the preconditioned solvers needed to match 1000 iterations of
    the unpreconditioned comparators (the paper's Sec. 4 comparison), and the
    same iteration without its preconditioner (D = I) as an ablation."""
    import numpy as np
    import torch

    from paper_1609_06041_amd import ctpd, synth

    out = {"kind": "iterations_to_match", "data": "synthetic", "dtype": "f32"}
    # low-dose: Eq. 1 cost per iteration
    prob, spec = synth.workload_problem("lowdose_512", with_x_true=True)
    n, m, nb, beta = spec["n"], spec["m"], spec["nb"], spec["beta"]
    b32, w32 = synth.as_f32_inputs(prob)
    b, w = torch.from_numpy(b32).to(dev), torch.from_numpy(w32).to(dev)
    xt = prob.x_true
    with ctpd.Operator(n, m, nb) as op:
        log("Algorithm 1, 20 iterations, cost recorded")
        xa, ia = op.lowdose_solve(b, w, beta, 20, record_cost=True)
        xa = xa.cpu().numpy()
        log("GIST, 1000 iterations, cost recorded")
        xg, ig = op.gist_lowdose_solve(b, w, beta, 1000, record_cost=True)
        xg = xg.cpu().numpy()
        _, ig_t = op.gist_lowdose_solve(b, w, beta, 1000)
        _, ia_t = op.lowdose_solve(b, w, beta, 20)
        log("Algorithm 1 with D = I (no preconditioner), 1000 iterations, cost recorded")
        xi, ii = op.app_identity_lowdose_solve(b, w, beta, 1000, record_cost=True)
        xi = xi.cpu().numpy()
    fa, fg, fi = ia["cost"], ig["cost"], ii["cost"]
    k_match = next((k + 1 for k in range(len(fa)) if fa[k] <= fg[-1]), None)
    out["lowdose_512"] = {
        "algorithm1_cost": [float(v) for v in fa],
        "gist_cost_at": {str(k): float(fg[k - 1]) for k in (1, 10, 100, 300, 1000)},
        "algorithm1_iters_to_reach_gist1000_cost": k_match,
        "gist_iters_to_reach_algorithm1_k10_cost": next((k + 1 for k in range(len(fg)) if fg[k] <= fa[9]), None),
        "rmse_algorithm1_20": float(np.sqrt(((xa - xt) ** 2).mean())),
        "rmse_gist_1000": float(np.sqrt(((xg - xt) ** 2).mean())),
        "rel_diff_algorithm1_20_vs_gist_1000": float(np.linalg.norm(xa - xg) / np.linalg.norm(xg)),
        "identity_cost_at": {str(k): float(fi[k - 1]) for k in (1, 10, 100, 300, 1000)},
        "identity_iters_to_reach_algorithm1_k10_cost": next((k + 1 for k in range(len(fi)) if fi[k] <= fa[9]),
                                                            None),
        "rmse_identity_1000": float(np.sqrt(((xi - xt) ** 2).mean())),
        "identity_steps": {"tau": ii["tau"], "sigma": ii["sigma"], "lambda_a": ii["lambda_a"],
                           "lambda_h": ii["lambda_h"]},
        "gist_step": ig_t["tau"], "gist_lipschitz": ig_t["lambda_a"],
        "ms": {"algorithm1_20_loop": ia_t["loop_ms"], "algorithm1_setup": ia_t["setup_ms"],
               "gist_1000_loop": ig_t["loop_ms"], "gist_setup": ig_t["setup_ms"]},
    }
    # few-view: RMSE against the phantom and distance to the CP-1000 image
    prob, spec = synth.workload_problem("fewview_512", with_x_true=True)
    n, m, nb = spec["n"], spec["m"], spec["nb"]
    bf = torch.from_numpy(np.asarray(prob.b, np.float32)).to(dev)
    xt = prob.x_true
    with ctpd.Operator(n, m, nb) as op:
        log("Chambolle-Pock, 1000 iterations")
        xc, ic = op.cp_fewview_solve(bf, 1000)
        xc = xc.cpu().numpy()
        rows = []
        for k in (1, 2, 3, 5, 10, 20):
            xk, ik = op.fewview_solve(bf, k)
            xk = xk.cpu().numpy()
            rows.append({"k": k, "rmse": float(np.sqrt(((xk - xt) ** 2).mean())),
                         "rel_diff_vs_cp1000": float(np.linalg.norm(xk - xc) / np.linalg.norm(xc)),
                         "loop_ms": ik["loop_ms"]})
        cp_rmse = {}
        for k in (3, 10, 100, 300):
            xk, _ = op.cp_fewview_solve(bf, k)
            cp_rmse[str(k)] = float(np.sqrt(((xk.cpu().numpy() - xt) ** 2).mean()))
    cp_rmse["1000"] = float(np.sqrt(((xc - xt) ** 2).mean()))
    out["fewview_512"] = {"algorithm2": rows, "cp_rmse_at": cp_rmse,
                          "algorithm2_iters_to_reach_cp1000_rmse":
                              next((r["k"] for r in rows if r["rmse"] <= cp_rmse["1000"]), None),
                          "ms": {"cp_1000_loop": ic["loop_ms"], "cp_setup": ic["setup_ms"]}}
    out["paper_context"] = ("paper (hardware not stated): ~10 Algorithm-1 iterations match GIST at 1000; "
                            "3 Algorithm-2 iterations match Chambolle-Pock at 1000")
    print(json.dumps(out), flush=True)
    return 0


def batch_speedup(dev, count: int, steps: int, warmup: int) -> int:
    out = batch_measure(dev, count, steps, warmup)
    print(json.dumps(out), flush=True)
    return 0 if out["results_identical_to_sequential"] else 1


def batch_measure(dev, count: int, steps: int, warmup: int) -> dict:
    """Batched uneven workload: one batched solve (set-up of every problem, then
    the 20-iteration loop of all problems as one graph replay) against the
    per-problem solver called once per problem."""
    import numpy as np
    import torch

    from paper_1609_06041_amd import ctpd, synth

    log(f"generating {count} seeded problems of the batched uneven workload")
    specs, bs, ws, betas = [], [], [], []
    for p in range(count):
        prob, spec = synth.batch_problem(p)
        b32, w32 = synth.as_f32_inputs(prob)
        specs.append(spec)
        bs.append(torch.from_numpy(b32).to(dev))
        ws.append(torch.from_numpy(w32).to(dev))
        betas.append(spec["beta"])
    geoms = [(sp["n"], sp["m"], sp["nb"]) for sp in specs]
    iters = specs[0]["iters"]
    outs = [torch.empty((n, n), device=dev) for n, _, _ in geoms]
    log("per-problem solves")
    ops = [ctpd.Operator(*g) for g in geoms]
    for op, b, w, beta, x in zip(ops, bs, ws, betas, outs):   # warm-up
        op.lowdose_solve(b, w, beta, iters, out=x)
    seq_total, seq_loop, seq_setup = [], [], []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loops = setups = 0.0
        for op, b, w, beta, x in zip(ops, bs, ws, betas, outs):
            _, info = op.lowdose_solve(b, w, beta, iters, out=x)
            loops += info["loop_ms"]
            setups += info["setup_ms"]
        torch.cuda.synchronize()
        seq_total.append(1e3 * (time.perf_counter() - t0))
        seq_loop.append(loops)
        seq_setup.append(setups)
    ref = [x.clone() for x in outs]
    for op in ops:
        op.close()
    log("batched solves: autotuning tile shapes")
    from paper_1609_06041_amd import autotune
    bouts = [torch.empty((n, n), device=dev) for n, _, _ in geoms]
    with ctpd.Batch(geoms) as bt:
        tuned = autotune.autotune(bt, bs, ws, betas, iters)
        log(f"chosen tiles {tuned['tiles']}")
        for _ in range(warmup):
            bt.lowdose_solve(bs, ws, betas, iters, outs=bouts)
        bat_total, bat_loop, bat_setup = [], [], []
        for _ in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, infos = bt.lowdose_solve(bs, ws, betas, iters, outs=bouts)
            torch.cuda.synchronize()
            bat_total.append(1e3 * (time.perf_counter() - t0))
            bat_loop.append(infos[0]["loop_ms"])
            bat_setup.append(infos[0]["setup_ms"])
        graph_ms = bt.time_loop(iters, 10, 5)
    identical = all(bool(torch.equal(a, b)) for a, b in zip(ref, bouts))
    med = lambda v: float(np.median(v))
    work = sum(m * n * n for n, m, _ in geoms)
    out = {
        "kind": "batched_uneven", "problems": count, "iterations": iters, "data": "synthetic", "dtype": "f32",
        "sizes": {f"{n}x{m}": sum(1 for g in geoms if g[0] == n and g[1] == m) for n, m, _ in sorted(set(geoms))},
        "sequential_ms": {"total": med(seq_total), "loop_sum": med(seq_loop), "setup_sum": med(seq_setup)},
        "batched_ms": {"total": med(bat_total), "loop": med(bat_loop), "setup": med(bat_setup)},
        "speedup_total": med(seq_total) / med(bat_total),
        "speedup_loop": med(seq_loop) / med(bat_loop),
        "batched_graph_replay_ms": graph_ms,
        "speedup_loop_graph_replay": med(seq_loop) / graph_ms,
        "batched_loop_gupdates_per_s": 2 * iters * work / (graph_ms * 1e-3) / 1e9,
        "tiles": tuned["tiles"], "autotune_ms": tuned.get("timings_ms"),
        "results_identical_to_sequential": identical,
    }
    return out


def unrolled_speedup(dev, steps: int) -> int:
    print(json.dumps(unrolled_measure(dev, steps)), flush=True)
    return 0


def unrolled_measure(dev, steps: int) -> dict:
    """16 independent 256^2 / 180-view problems, 10 unrolled iterations: forward
    and forward + reverse pass (the many-problem calls, each problem on its own
    stream) against 16 plain solves of the same 10 iterations and against the
    same forward + reverse passes one problem at a time, all at the same fixed
    step sizes."""
    import numpy as np
    import torch

    from paper_1609_06041_amd import ctpd, synth
    from paper_1609_06041_amd.unrolled import unrolled_lowdose, unrolled_lowdose_batch

    B, n, m, nb, K, beta = 16, 256, 180, 368, 10, 0.005
    log(f"generating {B} seeded 256^2 problems")
    probs = [synth.make_problem(4, p, n, m, nb, 15, 2e4, with_x_true=True) for p in range(B)]
    bs = [torch.from_numpy(np.asarray(pr.b, np.float32)).to(dev) for pr in probs]
    ws = [torch.from_numpy(np.asarray(pr.w, np.float32)).to(dev) for pr in probs]
    xts = [torch.from_numpy(np.asarray(pr.x_true, np.float32)).to(dev) for pr in probs]
    streams = [torch.cuda.Stream(device=dev) for _ in range(B)]
    ops = [ctpd.Operator(n, m, nb, stream=s) for s in streams]
    steps_ = []
    for op, b, w in zip(ops, bs, ws):
        _, info = op.lowdose_solve(b, w, beta, 0)
        steps_.append((info["tau"], info["sigma"]))
    torch.cuda.synchronize()

    def plain():
        for op, b, w, (ta, si) in zip(ops, bs, ws, steps_):
            op.lowdose_solve(b, w, beta, K, tau=ta, sigma=si)

    def forward():
        return unrolled_lowdose_batch(ops, bs, ws, [beta] * B, [ta for ta, _ in steps_], [si for _, si in steps_], K)

    def fwd_bwd():
        bts = [b.clone().requires_grad_(True) for b in bs]
        pars = [[torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in (beta, ta, si)]
                for ta, si in steps_]
        xs = unrolled_lowdose_batch(ops, bts, ws, [p[0] for p in pars], [p[1] for p in pars], [p[2] for p in pars],
                                    K)
        torch.stack([((x - xt) ** 2).sum() for x, xt in zip(xs, xts)]).sum().backward()
        return bts, pars

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(max(steps, 3)):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(1e3 * (time.perf_counter() - t0))
        return float(np.median(ts))

    def fwd_bwd_sequential():
        # the same 16 problems one after another on one stream, each waited for
        main = torch.cuda.current_stream()
        for op, st, b, w, xt, (ta, si) in zip(ops, streams, bs, ws, xts, steps_):
            bt = b.clone().requires_grad_(True)
            pars = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in (beta, ta, si)]
            st.wait_stream(main)
            with torch.cuda.stream(st):
                x = unrolled_lowdose(op, bt, w, *pars, K)
                loss = ((x - xt) ** 2).sum()
            main.wait_stream(st)
            loss.backward()
            torch.cuda.synchronize()

    log("timing plain solves, forward passes, forward + reverse passes (concurrent and one after another)")
    t_plain = timed(plain)
    t_fwd = timed(forward)
    t_fb = timed(fwd_bwd)
    t_fb_seq = timed(fwd_bwd_sequential)
    bts, pars = fwd_bwd()
    torch.cuda.synchronize()
    finite = all(bool(torch.isfinite(b.grad).all()) for b in bts) and all(
        all(p.grad is not None and np.isfinite(float(p.grad)) for p in ps) for ps in pars)
    out = {"kind": "unrolled_gradient", "problems": B, "image": f"{n}x{n}", "views": m, "bins": nb, "iterations": K,
           "data": "synthetic", "dtype": "f32", "plain_solves_ms": t_plain, "forward_ms": t_fwd,
           "forward_backward_ms": t_fb, "forward_backward_sequential_ms": t_fb_seq,
           "speedup_concurrent_vs_sequential": t_fb_seq / t_fb,
           "backward_over_forward": (t_fb - t_fwd) / t_fwd,
           "forward_backward_over_plain": t_fb / t_plain, "gradients_finite": finite,
           "accuracy": "reverse pass vs float64 central differences of the oracle, 1e-3 relative on 32^2 "
                       "(tests/test_gpu_unrolled.py)"}
    for op in ops:
        op.close()
    return out


def fewview_measure(dev, reps: int) -> dict:
    """The few-view workload (512^2, 32 views x 736 bins, noiseless): A and A^T
    per call, and Algorithm 2's iteration rate (20 iterations, default set-up,
    loop time from the solver's report, median of 5 solves), and the same for
    the error-tolerant few-view solve at eps = 1e-4 ||b|| (the ball binds after
    a few iterations)."""
    import numpy as np
    import torch

    from paper_1609_06041_amd import ctpd, synth

    prob, spec = synth.workload_problem("fewview_512", with_x_true=False)
    n, m, nb = spec["n"], spec["m"], spec["nb"]
    b = torch.from_numpy(np.asarray(prob.b, np.float32)).to(dev)
    with ctpd.Operator(n, m, nb) as op:
        img = torch.rand((n, n), device=dev, dtype=torch.float32)
        sino = torch.empty((m, nb), device=dev, dtype=torch.float32)
        img_out = torch.empty((n, n), device=dev, dtype=torch.float32)
        t_a = time_op(lambda: op.project(img, out=sino), op.stream, reps)
        t_at = time_op(lambda: op.backproject(b, out=img_out), op.stream, reps)
        _, cold = op.fewview_solve(b, 20)
        infos = [op.fewview_solve(b, 20)[1] for _ in range(5)]
        eps = 1e-4 * float(torch.linalg.vector_norm(b.double()))
        _, eps_cold = op.fewview_eps_solve(b, eps, 20)
        eps_infos = [op.fewview_eps_solve(b, eps, 20)[1] for _ in range(5)]
    loop_ms = float(np.median([i["loop_ms"] for i in infos]))
    setup_ms = float(np.median([i["setup_ms"] for i in infos]))
    eps_loop_ms = float(np.median([i["loop_ms"] for i in eps_infos]))
    updates = float(m) * n * n
    return {"workload": "fewview_512", "image": f"{n}x{n}", "views": m, "bins": nb,
            "A_ms": t_a, "AT_ms": t_at, "A_gupdates_per_s": updates / (t_a * 1e-3) / 1e9,
            "AT_gupdates_per_s": updates / (t_at * 1e-3) / 1e9,
            "algorithm2_iters": 20, "algorithm2_loop_ms": loop_ms, "algorithm2_setup_ms": setup_ms,
            "algorithm2_setup_ms_cold": cold["setup_ms"],
            "algorithm2_loop_iters_per_s": 20.0 / (loop_ms * 1e-3),
            "eps_constrained": {"eps": "1e-4 ||b||", "iters": 20, "loop_ms": eps_loop_ms,
                                "loop_iters_per_s": 20.0 / (eps_loop_ms * 1e-3),
                                "setup_ms": float(np.median([i["setup_ms"] for i in eps_infos])),
                                "setup_ms_cold": eps_cold["setup_ms"]}}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--op-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="leave out the few-view, batched and unrolled measurements of the default line")
    ap.add_argument("--compare", action="store_true",
                    help="instead of the throughput line: Algorithm 1 vs 1000 GIST iterations (lowdose_512) and "
                         "Algorithm 2 vs 1000 Chambolle-Pock iterations (fewview_512), iterations to match")
    ap.add_argument("--batch", type=int, default=0, metavar="P",
                    help="instead of the throughput line: P problems of the batched uneven workload solved as one "
                         "batch (graph replay) vs the same problems solved one after another")
    ap.add_argument("--unrolled", action="store_true",
                    help="instead of the throughput line: 16 unrolled 10-iteration solves (256^2, 180 views) forward "
                         "and reverse pass vs 16 plain solves")
    ap.add_argument("--fewview", action="store_true",
                    help="only the few-view workload (512^2, 32 views): A, A^T, Algorithm 2 and the "
                         "error-tolerant solve")
    ap.add_argument("--counters", action="store_true",
                    help="short run for rocprofv3 --pmc: a plain 256 MiB device copy (counter calibration) "
                         "followed by 5 launches each of A, A^T, the filter D and the 10-step TV prox on the "
                         "workload; prints nothing else")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (independent problems "
              "would shard one per GPU with no exchange). Run with --gpus 1.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1609_06041_amd import ctpd, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.compare:
        return compare(dev)
    if args.batch:
        return batch_speedup(dev, args.batch, args.steps, args.warmup)
    if args.fewview:
        print(json.dumps(fewview_measure(dev, args.op_reps)), flush=True)
        return 0
    if args.unrolled:
        return unrolled_speedup(dev, args.steps)
    log("generating the seeded lowdose_512 inputs (3 independent phantoms / noise draws)")
    insts = []
    for pid in range(N_INSTANCES):
        prob, spec = synth.workload_problem("lowdose_512", problem_id=pid, with_x_true=False)
        b32_i, w32_i = synth.as_f32_inputs(prob)
        insts.append((torch.from_numpy(b32_i).to(dev), torch.from_numpy(w32_i).to(dev)))
        if pid == 0:
            b32, w32 = b32_i, w32_i
    n, m, nb, beta, iters = spec["n"], spec["m"], spec["nb"], spec["beta"], spec["iters"]
    b, w = insts[0]
    op = ctpd.Operator(n, m, nb)
    stream = op.stream
    if args.counters:
        src = torch.ones(64 * 1024 * 1024, device=dev, dtype=torch.float32)   # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        img_out = torch.empty((n, n), device=dev, dtype=torch.float32)
        sino = torch.empty((m, nb), device=dev, dtype=torch.float32)
        img = torch.rand((n, n), device=dev, dtype=torch.float32)
        for _ in range(5):
            op.project(img, out=sino)
        for _ in range(5):
            op.backproject(b, out=img_out)
        for _ in range(5):
            op.ramp_filter(b, 2.0e-8, 3.5e-5, out=sino)
        pz = torch.zeros((2, n, n), device=dev, dtype=torch.float32)
        for _ in range(5):
            op.tv_prox(img, 1e-3, pz, n_iter=10, out=img_out)
        torch.cuda.synchronize()
        op.close()
        log("counter run done")
        return 0

    log(f"warmup: {args.warmup} solve(s); the first one on the fresh handle is the cold set-up")
    cold = None
    for i in range(max(args.warmup, 1)):
        _, info = op.lowdose_solve(*insts[i % N_INSTANCES], beta, iters)
        cold = info if cold is None else cold
    torch.cuda.synchronize()
    log(f"timing {args.steps} solves, cycling through {N_INSTANCES} inputs")
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, info = op.lowdose_solve(*insts[i % N_INSTANCES], beta, iters)
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = iters * args.steps / elapsed
    setup_ms = float(np.median([i["setup_ms"] for i in infos]))
    loop_ms = float(np.median([i["loop_ms"] for i in infos]))
    last = infos[-1]

    log("timing the single operators")
    img = torch.rand((n, n), device=dev, dtype=torch.float32)
    sino = torch.empty((m, nb), device=dev, dtype=torch.float32)
    img_out = torch.empty((n, n), device=dev, dtype=torch.float32)
    reps = args.op_reps
    t_a = time_op(lambda: op.project(img, out=sino), stream, reps)
    t_at = time_op(lambda: op.backproject(b, out=img_out), stream, reps)
    t_d = time_op(lambda: op.ramp_filter(b, last["tau"], last["kappa"], out=sino), stream, reps)
    pz = torch.zeros((2, n, n), device=dev, dtype=torch.float32)
    t_tv10 = time_op(lambda: op.tv_prox(img, 1e-3, pz, n_iter=10, out=img_out), stream, max(reps // 5, 5))
    updates = float(m) * n * n
    ray_steps = float(forward_ray_steps(n, m, nb))
    a_tflops = A_FLOP_PER_STEP * ray_steps / (t_a * 1e-3) / 1e12
    d_tflops = 2.0 * m * nb * nb / (t_d * 1e-3) / 1e12
    tv_gbs = 24.0 * n * n / (t_tv10 * 1e-3) / 1e9
    at_tflops = AT_FLOP_PER_UPDATE * updates / (t_at * 1e-3) / 1e12
    peak_note = ("FP32 vector peak: 256 CU x 128 FMA lanes x 2.4 GHz x 2 (plain v_fma_f32 exceeds 64 lanes/CU/clock "
                 "on gfx950: a register-only FMA loop reaches 95 TFLOP/s)")
    rec = {
        "metric": "512x512/720-view PD iters/s (Algorithm 1, set-up included) + A, A^T Gupdates/s; "
                  "batched & unrolled-grad speedup",
        "value": value,
        "unit": "PD iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "lowdose_512", "image": f"{n}x{n}", "views": m, "bins": nb,
                   "phantom": "20 seeded ellipses, Poisson I0=5e4", "beta": beta, "iterations_per_step": iters,
                   "tv_iters": 10},
        "loop_iters_per_s": iters / (loop_ms * 1e-3),
        "setup_ms": setup_ms,
        "setup_ms_cold": cold["setup_ms"],
        "setup_note": "per solve: kappa, W^-1, taps, lambda_h (Lanczos, data-dependent) and sigma; "
                      "kappa*lambda_A is a property of the geometry at the default tau and is computed by the "
                      "first solve on a handle (setup_ms_cold) and reused",
        "loop_ms": loop_ms,
        "step_sizes": {"tau": last["tau"], "sigma": last["sigma"], "lambda_a": last["lambda_a"],
                       "lambda_h": last["lambda_h"], "lanczos_steps": [last["norm_steps_a"],
                                                                       last["norm_steps_h"]],
                       "lanczos_steps_cold": [cold["norm_steps_a"], cold["norm_steps_h"]]},
        "A_gupdates_per_s": updates / (t_a * 1e-3) / 1e9,
        "AT_gupdates_per_s": updates / (t_at * 1e-3) / 1e9,
        "op_ms": {"A": t_a, "AT": t_at, "D": t_d, "tv_step": t_tv10 / 10.0},
        "filter_mfma_tflops": d_tflops,
        "tv_step_gbs": 20.0 * n * n / (t_tv10 / 10.0 * 1e-3) / 1e9,
        "roofline": {"kernel": "forward_slab_kernel (A; timed per ctpd_project call, which also pads the image planes)", "bound": "alu",
                     "achieved": a_tflops, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": a_tflops / PEAK_FP32_VECTOR_TFLOPS, "traffic": read_traffic("forward"),
                     "work_per_launch": f"{ray_steps:.4g} in-image ray steps x {A_FLOP_PER_STEP:.0f} FLOP",
                     "peak_note": peak_note},
        "roofline_at": {"kernel": "adjoint_kernel (A^T, one launch per ctpd_backproject)", "bound": "alu",
                        "achieved": at_tflops, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                        "frac": at_tflops / PEAK_FP32_VECTOR_TFLOPS, "traffic": read_traffic("adjoint"),
                        "work_per_launch": f"{updates:.4g} (pixel, view) updates x {AT_FLOP_PER_UPDATE:.0f} FLOP",
                        "peak_note": peak_note},
        "roofline_filter": {"kernel": "filter_mfma_kernel (D, one launch per ctpd_filter after its taps kernel)",
                            "bound": "mfma", "achieved": d_tflops, "peak": PEAK_FILTER_TFLOPS, "unit": "TFLOP/s",
                            "frac": d_tflops / PEAK_FILTER_TFLOPS, "traffic": read_traffic("filter"),
                            "work_per_launch": f"dense Toeplitz contraction 2 x {m} x {nb} x {nb} FP32 FLOP",
                            "peak_note": f"each FP32 product is {FILTER_TERM_PRODUCTS} bf16 term products "
                                         f"(three-term bf16 splits, FP32 accumulation): bf16 dense "
                                         f"{PEAK_BF16_MFMA_TFLOPS:.0f} / {FILTER_TERM_PRODUCTS}; the FP32 MFMA "
                                         f"peak is {PEAK_FP32_MFMA_TFLOPS}"},
        "roofline_tv": {"kernel": "tv_prox_kernel (10 dual steps fused, one launch per ctpd_tv_prox)",
                        "bound": "alu", "achieved_gbs": tv_gbs, "hbm_frac": tv_gbs / PEAK_HBM_GBS,
                        "traffic": read_traffic("tv"),
                        "work_per_launch": f"algorithmic bytes 24 x {n}^2 (z, p in; p, x out; FP32)"},
        "accuracy": "parity-tested vs the FP64 oracle: A, A^T, D rel l2 <= 1e-5; x^k rel l2 <= 1e-4; "
                    "cost rel <= 1e-5 (tests/test_gpu_*.py)",
        "paper_context": "paper (no hardware stated): ~10 Algorithm-1 iterations match GIST at 1000; "
                         "3 Algorithm-2 iterations match Chambolle-Pock at 1000",
    }
    op.close()
    if not args.no_extras:
        log("few-view workload: A, A^T and Algorithm-2 iterations")
        rec["fewview_512"] = fewview_measure(dev, reps)
        log("batched uneven workload (64 problems): batched vs one after another")
        rec["batched"] = batch_measure(dev, 64, 3, 1)
        log("unrolled differentiable solve (16 x 256^2, 180 views, 10 iterations)")
        rec["unrolled"] = unrolled_measure(dev, 3)
        rec["speedups"] = {
            "batched_vs_sequential_total": rec["batched"]["speedup_total"],
            "batched_vs_sequential_loop_graph_replay": rec["batched"]["speedup_loop_graph_replay"],
            "unrolled_fwd_bwd_concurrent_vs_sequential": rec["unrolled"]["speedup_concurrent_vs_sequential"],
            "unrolled_fwd_bwd_over_plain_solves": rec["unrolled"]["forward_backward_over_plain"],
        }
    if not args.no_cpu_baseline:
        b64 = b32.astype(np.float64)
        w64 = w32.astype(np.float64)
        log("timing the FP64 oracle on a bounded sample, one thread (cpu_baseline)")
        rec["cpu_baseline"] = cpu_baseline(b64, w64, beta, n, m, nb, last["tau"], last["sigma"])
        ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        log(f"timing the FP64 oracle on the same sample with {ncpu} BLAS threads")
        rec["cpu_baseline_all_cores"] = cpu_baseline(b64, w64, beta, n, m, nb, last["tau"], last["sigma"],
                                                     threads=ncpu)
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
