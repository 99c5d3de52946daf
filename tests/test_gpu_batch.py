"""Batched uneven solves (one flattened launch per kernel and step over many
problems, the loop replayed from a captured HIP graph) against the per-problem
solver and the FP64 oracle.

The batch runs the same kernel bodies with the same float32 step sizes as
``ctpd_pd_lowdose_solve``, so each problem's result must equal its single
solve bit for bit; the single solver is itself held to the oracle, and one
small problem of each batch is also compared with the oracle directly
(x^k relative l2 <= 1e-4).
"""
import numpy as np
import pytest
import torch

from oracle import app as OA
from paper_1609_06041_amd import ctpd
from paper_1609_06041_amd import synth as S

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _inputs(geoms, seed0):
    out = []
    for i, (n, m, nb) in enumerate(geoms):
        if n < 3:   # too small for an ellipse phantom: positive random data
            rng = np.random.default_rng(seed0 + i)
            out.append((rng.uniform(0.0, 0.5, (m, nb)).astype(np.float32),
                        rng.uniform(1e3, 2e4, (m, nb)).astype(np.float32)))
            continue
        prob = S.make_problem(95, seed0 + i, n, m, nb, 8, 2e4, with_x_true=False)
        b32, w32 = S.as_f32_inputs(prob)
        out.append((b32, w32))
    return out


def _singles(geoms, data, betas, iters):
    xs, infos = [], []
    for (n, m, nb), (b, w), beta in zip(geoms, data, betas):
        with ctpd.Operator(n, m, nb) as op:
            x, info = op.lowdose_solve(dev(b), dev(w), beta, iters)
            xs.append(host(x))
            infos.append(info)
    return xs, infos


SMALL = [(32, 20, 48), (48, 33, 70), (64, 90, 96), (24, 7, 35), (40, 16, 57), (1, 3, 2)]


def test_batch_equals_single_solves_and_oracle(gpu, parity):
    data = _inputs(SMALL, 0)
    betas = [0.01, 0.02, 0.01, 0.0, 0.05, 0.1]
    iters = 12
    ref_x, ref_info = _singles(SMALL, data, betas, iters)
    with ctpd.Batch(SMALL) as bt:
        xs, infos = bt.lowdose_solve([dev(b) for b, _ in data], [dev(w) for _, w in data], betas, iters)
        xs = [host(x) for x in xs]
    for i in range(len(SMALL)):
        assert infos[i]["sigma"] == ref_info[i]["sigma"]
        assert infos[i]["tau"] == ref_info[i]["tau"]
        np.testing.assert_array_equal(xs[i], ref_x[i])
    # problem 2 directly against the oracle
    n, m, nb = SMALL[2]
    b, w = (a.astype(np.float64) for a in data[2])
    res, _ = OA.lowdose_solve(b, w, betas[2], n, iters, tau=infos[2]["tau"], sigma=infos[2]["sigma"])
    parity("xs[2]", rel(xs[2], res.x), 1e-4)


def test_batch_graph_replay_with_new_inputs(gpu):
    geoms = SMALL[:4]
    betas = [0.01, 0.03, 0.0, 0.02]
    with ctpd.Batch(geoms) as bt:
        for seed in (10, 20):   # the second call replays the captured loop
            data = _inputs(geoms, seed)
            ref_x, _ = _singles(geoms, data, betas, 8)
            xs, _ = bt.lowdose_solve([dev(b) for b, _ in data], [dev(w) for _, w in data], betas, 8)
            for x, r in zip(xs, ref_x):
                np.testing.assert_array_equal(host(x), r)


def test_batch_of_the_uneven_workload_sizes(gpu):
    # six problems of the 64-problem uneven workload (sizes 256-512, 32-720 views), 20 iterations,
    # under every tile choice (the TV prox of 512- and 1024-thread workgroups, the slab and
    # the gather forward projector) against the per-problem solver
    from paper_1609_06041_amd import autotune
    ids = [0, 5, 11, 17, 23, 42]
    probs = [S.batch_problem(p) for p in ids]
    geoms = [(sp["n"], sp["m"], sp["nb"]) for _, sp in probs]
    data = [S.as_f32_inputs(pr) for pr, _ in probs]
    betas = [sp["beta"] for _, sp in probs]
    ref_x, _ = _singles(geoms, data, betas, 20)
    bs, ws = [dev(b) for b, _ in data], [dev(w) for _, w in data]
    with ctpd.Batch(geoms) as bt:
        for cand in autotune.CANDIDATES:
            bt.set_tiles(**cand)
            xs, _ = bt.lowdose_solve(bs, ws, betas, 20)
            for x, r in zip(xs, ref_x):
                np.testing.assert_array_equal(host(x), r, err_msg=str(cand))


def test_batch_rejects_bad_arguments(gpu):
    with pytest.raises(ctpd.CtpdError) as e:
        ctpd.Batch([(16, 8, 0)])
    assert e.value.code == ctpd.CTPD_EINVAL
    geoms = [(16, 8, 24), (20, 9, 30)]
    data = _inputs(geoms, 30)
    with ctpd.Batch(geoms) as bt:
        w_bad = data[1][1].copy()
        w_bad[0, 0] = 0.0
        with pytest.raises(ctpd.CtpdError) as e:
            bt.lowdose_solve([dev(data[0][0]), dev(data[1][0])], [dev(data[0][1]), dev(w_bad)], [0.1, 0.1], 3)
        assert e.value.code == ctpd.CTPD_EDOMAIN
        with pytest.raises(ctpd.CtpdError) as e:
            bt.lowdose_solve([dev(b) for b, _ in data], [dev(w) for _, w in data], [0.1, -1.0], 3)
        assert e.value.code == ctpd.CTPD_EINVAL


def test_every_tile_choice_gives_the_same_result(gpu):
    from paper_1609_06041_amd import autotune
    geoms = [(48, 33, 70), (64, 90, 96), (40, 16, 57)]
    data = _inputs(geoms, 40)
    betas = [0.01, 0.02, 0.03]
    bs, ws = [dev(b) for b, _ in data], [dev(w) for _, w in data]
    with ctpd.Batch(geoms) as bt:
        ref, _ = bt.lowdose_solve(bs, ws, betas, 5)
        ref = [host(x) for x in ref]
        for cand in autotune.CANDIDATES:
            bt.set_tiles(**cand)
            assert bt.get_tiles() == cand
            xs, _ = bt.lowdose_solve(bs, ws, betas, 5)
            for x, r in zip(xs, ref):
                np.testing.assert_array_equal(host(x), r)
        assert bt.time_loop(5, 10, 2) > 0.0
        with pytest.raises(ctpd.CtpdError):
            bt.set_tiles(placement=0, tv_threads=256, fwd_form=0)


def test_batch_with_chunked_inner_steps(gpu):
    # 12 inner TV steps (two prox chunks per iteration)
    geoms = SMALL[:3]
    data = _inputs(geoms, 50)
    betas = [0.02, 0.0, 0.04]
    ref = []
    for (n, m, nb), (b, w), beta in zip(geoms, data, betas):
        with ctpd.Operator(n, m, nb) as op:
            x, _ = op.lowdose_solve(dev(b), dev(w), beta, 6, tv_iters=12)
            ref.append(host(x))
    with ctpd.Batch(geoms) as bt:
        xs, _ = bt.lowdose_solve([dev(b) for b, _ in data], [dev(w) for _, w in data], betas, 6, tv_iters=12)
        for x, r in zip(xs, ref):
            np.testing.assert_array_equal(host(x), r)
