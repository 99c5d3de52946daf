// Batched low-dose solves: many independent problems of uneven image sizes
// and view counts (Algorithm 1 on each), set up together and iterated
// together.  Each problem keeps its own operator handle (geometry tables,
// taps, workspaces); the iteration runs one flattened launch per kernel and
// step for the whole batch, and the whole K-iteration loop is captured once
// in a HIP graph and replayed.
//
// Workgroup placement: consecutive workgroups of a launch go to the eight
// XCDs in turn, and each XCD has its own L2.  Problems are assigned to XCDs
// (largest first, onto the least-loaded XCD, weighted by m * n^2, the work of
// A and A^T), and a problem's workgroups are placed only at grid positions of
// its XCD, so its image, sinogram and views stay in one L2 across kernels.
#include <algorithm>
#include <numeric>

#include "op.h"

using namespace ctpd;
using namespace ctpd_host;

namespace {

enum Kind { K_INIT, K_FILT, K_NFILT, K_ADJ, K_TV, K_PAD, K_FWD, K_COPY, K_COUNT };

}  // namespace

namespace ctpd_host {

Placement plan_xcds(const std::vector<double>& work) {
    const int P = (int)work.size();
    Placement pl;
    pl.order.resize(P);
    std::iota(pl.order.begin(), pl.order.end(), 0);
    std::stable_sort(pl.order.begin(), pl.order.end(), [&](int a, int b) { return work[a] > work[b]; });
    std::vector<double> load(kXcds, 0.0);
    pl.xcd.assign(P, 0);
    for (int p : pl.order) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        pl.xcd[p] = x;
        load[x] += work[p];
    }
    return pl;
}

std::vector<BlockRef> place_blocks(const Placement& pl, const std::vector<int>& counts, int placement) {
    std::vector<BlockRef> flat;
    if (placement == 0) {   // XCD-binned
        std::vector<std::vector<BlockRef>> bins(kXcds);
        for (int p : pl.order)
            for (int l = 0; l < counts[p]; ++l) bins[pl.xcd[p]].push_back(BlockRef{p, l});
        size_t len = 0;
        for (auto& b : bins) len = std::max(len, b.size());
        flat.assign(len * kXcds, BlockRef{-1, 0});
        for (int x = 0; x < kXcds; ++x)
            for (size_t i = 0; i < bins[x].size(); ++i) flat[i * kXcds + x] = bins[x][i];
    } else {   // problem-major, largest first: consecutive workgroups of a problem spread over all XCDs
        for (int p : pl.order)
            for (int l = 0; l < counts[p]; ++l) flat.push_back(BlockRef{p, l});
    }
    return flat;
}

}  // namespace ctpd_host

struct ctpd_batch {
    int count = 0;
    hipStream_t user = nullptr;   // caller's stream
    hipStream_t gs = nullptr;     // internal stream: set-up joins here, the loop graph runs here
    hipEvent_t ev = nullptr;
    std::vector<ctpd_op*> ops;
    std::vector<hipStream_t> streams;   // one per problem for the set-up
    std::vector<int> xcd;               // XCD of each problem
    int max_nb = 0, max_n = 0;
    BatchItem* items = nullptr;         // device table
    BatchItem* items_host = nullptr;    // pinned mirror
    NormItem* nitems = nullptr;         // lambda_h chains: device table
    NormItem* nitems_host = nullptr;    // pinned mirror
    RowRef* rows = nullptr;             // every (problem, view)
    int nrows = 0;
    double* hsum = nullptr;             // lambda_h chain summaries, 3 per problem (device)
    double* hsum_host = nullptr;        // pinned, two slots of 3 per problem
    hipEvent_t hev[2] = {nullptr, nullptr};   // behind the copies into the two slots
    BlockRef* map[K_COUNT] = {};
    int nblk[K_COUNT] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int g_iters = -1, g_tv = -1;
    ctpd_batch_tiles tiles{0, 1024, 0, 0};
    bool slab_ok = true;   // every problem's image fits the slab projector
    bool solved = false;   // items hold a valid set-up (a solve has run)
};

namespace {

int blocks_of(const ctpd_op* op, int kind, int fwd_form) {
    const size_t J = op->J, I = op->I;
    switch (kind) {
        case K_INIT: return (int)((3 * J + 2 * I + 2047) / 2048);
        case K_FILT: return filter_blocks_x(op->nb) * filter_blocks_y(op->m);
        case K_NFILT: return norm_blocks_x(op->nb) * norm_blocks_y(op->m);
        case K_ADJ: return adjoint_tiles(op->n) * adjoint_tiles(op->n);
        case K_TV: return tv_tiles(op->n) * tv_tiles(op->n);
        case K_PAD: return pad_tiles(op->n) * pad_tiles(op->n);
        case K_FWD: return fwd_form == 0 ? op->bat_groups : forward_blocks_x(op->nb) * op->m;
        default: return (int)((J + 2047) / 2048);
    }
}

int build_maps(ctpd_batch* bt) {
    const int P = bt->count;
    std::vector<double> work(P);
    for (int p = 0; p < P; ++p) work[p] = (double)bt->ops[p]->m * bt->ops[p]->n * bt->ops[p]->n;
    const Placement pl = plan_xcds(work);
    bt->xcd = pl.xcd;
    for (int kind = 0; kind < K_COUNT; ++kind) {
        std::vector<int> counts(P);
        for (int p = 0; p < P; ++p) counts[p] = blocks_of(bt->ops[p], kind, bt->tiles.fwd_form);
        const std::vector<BlockRef> flat = place_blocks(pl, counts, bt->tiles.placement);
        if (bt->map[kind]) (void)hipFree(bt->map[kind]);
        bt->map[kind] = nullptr;
        ALLOC(bt->map[kind], flat.size());
        HIP_TRY(hipMemcpy(bt->map[kind], flat.data(), sizeof(BlockRef) * flat.size(), hipMemcpyHostToDevice));
        bt->nblk[kind] = (int)flat.size();
    }
    return CTPD_OK;
}

// The K-iteration loop of Algorithm 1 over the whole batch (queued on bt->gs).
int queue_loop(ctpd_batch* bt, int iters, int tv_iters) {
    hipStream_t s = bt->gs;
    const BatchItem* it = bt->items;
    HIP_TRY(launch_batch_init(it, bt->map[K_INIT], bt->nblk[K_INIT], s));
    int pc = 0;
    const int chunk = tv_chunk_max();
    for (int k = 0; k < iters; ++k) {
        const int rot = (3 - k % 3) % 3;
        // Step 1: mubar = 2 mu - mu_prev - sigma D W^-1 (mu - mu_prev) (k >= 1)
        // Step 2: z = x - tau A^T mubar; x = prox(z).  At k = 0 (x = 0, mubar =
        // -sigma D b) z = -sigma (x - tau A^T D b), the single solve's order.
        HIP_TRY(launch_filter_batched(it, bt->map[K_FILT], bt->nblk[K_FILT], k == 0 ? FILT_PLAIN : FILT_EXTRAP,
                                      rot, bt->max_nb, s));
        HIP_TRY(launch_adjoint_batched(it, bt->map[K_ADJ], bt->nblk[K_ADJ], false, rot, s));
        if (k == 0) HIP_TRY(launch_batch_scale_z(it, bt->map[K_COPY], bt->nblk[K_COPY], s));
        int left = tv_iters;
        do {
            const int st = std::min(left, chunk);
            left -= st;
            HIP_TRY(launch_tv_prox_batched(it, bt->map[K_TV], bt->nblk[K_TV], pc, st, left == 0,
                                           bt->tiles.tv_threads, s));
            pc = 1 - pc;
        } while (left > 0);
        // Step 3: mu^{k+1} = mu + sigma D (A x - b - W^-1 mu)
        HIP_TRY(launch_pad_planes_batched(it, bt->map[K_PAD], bt->nblk[K_PAD], s));
        HIP_TRY(launch_forward_batched(it, bt->map[K_FWD], bt->nblk[K_FWD], bt->tiles.fwd_form, bt->max_n, rot, s));
        HIP_TRY(launch_filter_batched(it, bt->map[K_FILT], bt->nblk[K_FILT], FILT_DUAL_LD, rot, bt->max_nb, s));
    }
    HIP_TRY(launch_batch_copy_out(it, bt->map[K_COPY], bt->nblk[K_COPY], s));
    return CTPD_OK;
}

int capture_loop(ctpd_batch* bt, int iters, int tv_iters) {
    if (bt->exec && bt->g_iters == iters && bt->g_tv == tv_iters) return CTPD_OK;
    if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
    if (bt->graph) (void)hipGraphDestroy(bt->graph);
    bt->exec = nullptr;
    bt->graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(bt->gs, hipStreamCaptureModeThreadLocal));
    const int r = queue_loop(bt, iters, tv_iters);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(bt->gs, &g);
    if (r) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    HIP_TRY(e);
    bt->graph = g;
    HIP_TRY(hipGraphInstantiate(&bt->exec, g, nullptr, nullptr, 0));
    bt->g_iters = iters;
    bt->g_tv = tv_iters;
    return CTPD_OK;
}

}  // namespace

extern "C" {

int ctpd_batch_create(const ctpd_geometry* geoms, int32_t count, void* stream, ctpd_batch** out) {
    g_errmsg[0] = 0;
    if (!geoms || !out) return einval("null pointer");
    if (count < 1 || count > CTPD_MAX_BATCH) return einval("count out of range [1, CTPD_MAX_BATCH]");
    *out = nullptr;
    ctpd_batch* bt = new ctpd_batch();
    bt->count = count;
    bt->user = (hipStream_t)stream;
    auto init = [&]() -> int {
        HIP_TRY(hipStreamCreateWithFlags(&bt->gs, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&bt->ev, hipEventDisableTiming));
        for (int p = 0; p < count; ++p) {
            hipStream_t st = nullptr;
            HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            bt->streams.push_back(st);
            ctpd_op* op = nullptr;
            const int r = ctpd_op_create(&geoms[p], st, &op);
            if (r) return r;
            bt->ops.push_back(op);
            bt->max_nb = std::max(bt->max_nb, geoms[p].n_bins);
            bt->max_n = std::max(bt->max_n, geoms[p].n);
        }
        bt->slab_ok = forward_slab_fits(bt->max_n);
        if (!bt->slab_ok) bt->tiles.fwd_form = 1;
        ALLOC(bt->items, count);
        HIP_TRY(hipHostMalloc((void**)&bt->items_host, sizeof(BatchItem) * count, hipHostMallocDefault));
        ALLOC(bt->nitems, count);
        HIP_TRY(hipHostMalloc((void**)&bt->nitems_host, sizeof(NormItem) * count, hipHostMallocDefault));
        std::vector<RowRef> rows;
        for (int p = 0; p < count; ++p)
            for (int v = 0; v < geoms[p].n_views; ++v) rows.push_back(RowRef{p, v});
        bt->nrows = (int)rows.size();
        ALLOC(bt->rows, rows.size());
        HIP_TRY(hipMemcpy(bt->rows, rows.data(), sizeof(RowRef) * rows.size(), hipMemcpyHostToDevice));
        ALLOC(bt->hsum, 3 * count);
        HIP_TRY(hipHostMalloc((void**)&bt->hsum_host, sizeof(double) * 6 * count, hipHostMallocDefault));
        for (auto& e : bt->hev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        return build_maps(bt);
    };
    const int r = init();
    if (r) {
        ctpd_batch_destroy(bt);
        return r;
    }
    *out = bt;
    return CTPD_OK;
}

void ctpd_batch_destroy(ctpd_batch* bt) {
    if (!bt) return;
    if (bt->gs) (void)hipStreamSynchronize(bt->gs);
    if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
    if (bt->graph) (void)hipGraphDestroy(bt->graph);
    for (ctpd_op* op : bt->ops) ctpd_op_destroy(op);
    for (hipStream_t st : bt->streams) (void)hipStreamDestroy(st);
    for (BlockRef* m : bt->map)
        if (m) (void)hipFree(m);
    if (bt->items) (void)hipFree(bt->items);
    if (bt->items_host) (void)hipHostFree(bt->items_host);
    if (bt->nitems) (void)hipFree(bt->nitems);
    if (bt->nitems_host) (void)hipHostFree(bt->nitems_host);
    if (bt->rows) (void)hipFree(bt->rows);
    if (bt->hsum) (void)hipFree(bt->hsum);
    if (bt->hsum_host) (void)hipHostFree(bt->hsum_host);
    for (auto e : bt->hev)
        if (e) (void)hipEventDestroy(e);
    if (bt->ev) (void)hipEventDestroy(bt->ev);
    if (bt->gs) (void)hipStreamDestroy(bt->gs);
    delete bt;
}

int ctpd_batch_lowdose_solve(ctpd_batch* bt, const float* const* b, const float* const* w, const double* beta,
                             int32_t iters, const ctpd_params* p, float* const* x_out, ctpd_report* reps) {
    g_errmsg[0] = 0;
    if (!bt || !b || !w || !beta || !x_out) return einval("null pointer");
    if (iters < 0) return einval("iters < 0");
    const int P = bt->count;
    for (int i = 0; i < P; ++i) {
        if (!b[i] || !w[i] || !x_out[i]) return einval("null problem pointer");
        if (!(beta[i] >= 0.0) || !std::isfinite(beta[i])) return einval("beta must be finite and >= 0");
    }
    Knobs k;
    int r = read_params(p, &k);
    if (r) return r;
    if ((r = no_state(k))) return r;
    const auto t0 = std::chrono::steady_clock::now();
    // inputs are ready on the caller's stream: every problem stream waits for it
    HIP_TRY(hipEventRecord(bt->ev, bt->user));
    for (hipStream_t st : bt->streams) HIP_TRY(hipStreamWaitEvent(st, bt->ev, 0));
    HIP_TRY(hipStreamWaitEvent(bt->gs, bt->ev, 0));
    // a1 / a2 for every problem; the operator-norm chains of all problems run together
    std::vector<LowdoseSetup> S(P);
    std::vector<Lanczos*> chains;
    for (int i = 0; i < P; ++i) {
        if ((r = lowdose_setup_begin(bt->ops[i], b[i], w[i], k, &S[i]))) return r;
        if (S[i].run_a) chains.push_back(&S[i].La);
    }
    // lambda_A chains (first solve on the geometry only), one stream per problem
    if ((r = run_lanczos(chains))) return r;
    // per-view lambda_h chains of all problems together, on the batch stream
    for (int i = 0; i < P; ++i)
        if ((r = sync(bt->ops[i]))) return r;
    {
        std::vector<double> kap(P), lam(P);
        std::vector<int> st(P);
        for (int i = 0; i < P; ++i) kap[i] = S[i].kappa;
        if ((r = lambda_h_views(bt->ops, w, kap.data(), k.norm_steps, bt->gs, bt->nitems, bt->nitems_host, bt->rows,
                                bt->nrows, bt->map[K_NFILT], bt->nblk[K_NFILT], bt->hsum, bt->hsum_host, bt->hev,
                                lam.data(), st.data())))
            return r;
        for (int i = 0; i < P; ++i) {
            S[i].lam_h = lam[i];
            S[i].steps_h = st[i];
        }
    }
    for (int i = 0; i < P; ++i) {
        if ((r = lowdose_setup_end(bt->ops[i], k, &S[i]))) return r;
        if ((r = sync(bt->ops[i]))) return r;
    }
    const double setup_ms = ms_since(t0);
    const auto t1 = std::chrono::steady_clock::now();
    for (int i = 0; i < P; ++i) {
        const ctpd_op* op = bt->ops[i];
        BatchItem& it = bt->items_host[i];
        it = BatchItem{};
        it.n = op->n;
        it.m = op->m;
        it.nb = op->nb;
        it.lowdose = 1;
        it.views = op->views;
        it.taps = op->taps32;
        it.b = b[i];
        it.winv = op->winv;
        it.x = op->x;
        it.z = op->z;
        it.q = op->q;
        it.sx = op->sx;
        it.mubar = op->mubar;
        for (int j = 0; j < 3; ++j) it.mu[j] = op->mu[j];
        for (int j = 0; j < 2; ++j) it.p[j] = op->p[j];
        it.xp = op->xp;
        it.xTp = op->xTp;
        it.tasks = op->bat_tasks;
        it.x_out = x_out[i];
        it.sigma = (float)S[i].sigma;
        it.tau = (float)S[i].tau;
        it.lam = (float)(S[i].tau * beta[i]);
        it.tvstep = it.lam > 0 ? (float)(k.tv_step / (S[i].tau * beta[i])) : 0.f;
    }
    HIP_TRY(hipMemcpyAsync(bt->items, bt->items_host, sizeof(BatchItem) * P, hipMemcpyHostToDevice, bt->gs));
    if ((r = capture_loop(bt, iters, k.tv_iters))) return r;
    HIP_TRY(hipGraphLaunch(bt->exec, bt->gs));
    HIP_TRY(hipStreamSynchronize(bt->gs));
    const double loop_ms = ms_since(t1);
    bt->solved = true;
    if (reps) {
        for (int i = 0; i < P; ++i) {
            ctpd_report& rp = reps[i];
            rp.tau = S[i].tau;
            rp.sigma = S[i].sigma;
            rp.kappa = S[i].kappa;
            rp.lambda_a = S[i].lam_a;
            rp.lambda_h = S[i].lam_h;
            rp.norm_steps_a = S[i].steps_a;
            rp.norm_steps_h = S[i].steps_h;
            rp.iters_done = iters;
            rp.setup_ms = setup_ms;
            rp.loop_ms = loop_ms;
        }
    }
    return CTPD_OK;
}

int ctpd_batch_set_tiles(ctpd_batch* bt, const ctpd_batch_tiles* t) {
    g_errmsg[0] = 0;
    if (!bt || !t) return einval("null pointer");
    if (t->placement != 0 && t->placement != 1) return einval("placement must be 0 or 1");
    if (t->tv_threads != 512 && t->tv_threads != 1024) return einval("tv_threads must be 512 or 1024");
    if (t->fwd_form != 0 && t->fwd_form != 1) return einval("fwd_form must be 0 (slab) or 1 (gather)");
    if (t->fwd_form == 0 && !bt->slab_ok) return einval("an image of the batch is too large for the slab projector");
    const bool remap = t->placement != bt->tiles.placement || t->fwd_form != bt->tiles.fwd_form;
    bt->tiles = *t;
    bt->tiles.reserved = 0;
    bt->g_iters = -1;   // recapture the loop with the new choices
    if (remap) {
        HIP_TRY(hipStreamSynchronize(bt->gs));
        return build_maps(bt);
    }
    return CTPD_OK;
}

int ctpd_batch_get_tiles(const ctpd_batch* bt, ctpd_batch_tiles* t) {
    g_errmsg[0] = 0;
    if (!bt || !t) return einval("null pointer");
    *t = bt->tiles;
    return CTPD_OK;
}

int ctpd_batch_time_loop(ctpd_batch* bt, int32_t iters, int32_t tv_iters, int32_t reps, double* ms) {
    g_errmsg[0] = 0;
    if (!bt || !ms) return einval("null pointer");
    if (!bt->solved) return einval("no solve has set the batch up yet");
    if (iters < 1 || tv_iters < 1 || reps < 1) return einval("iters, tv_iters and reps must be >= 1");
    int r = capture_loop(bt, iters, tv_iters);
    if (r) return r;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    std::vector<float> t(reps);
    int rc = CTPD_OK;
    for (int i = 0; i < reps && rc == CTPD_OK; ++i) {
        hipError_t e = hipEventRecord(e0, bt->gs);
        if (e == hipSuccess) e = hipGraphLaunch(bt->exec, bt->gs);
        if (e == hipSuccess) e = hipEventRecord(e1, bt->gs);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&t[i], e0, e1);
        if (e != hipSuccess) rc = fail_hip(e, "timing the batched loop");
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    std::sort(t.begin(), t.end());
    *ms = t[reps / 2];
    return CTPD_OK;
}

}  // extern "C"
