// Algorithm 1 unrolled for a fixed number of iterations with given step sizes,
// as a differentiable function of the data b, the TV weight beta and the steps
// tau, sigma (the filter D = D(tau) of Eq. 24 depends on tau too).  The
// forward pass runs the solver's kernel bodies and keeps the state
// (x^k, mu^k, p^k) of every iteration in a caller-owned checkpoint buffer; the
// reverse pass walks the iterations backwards, recomputing each iteration's
// intermediates (the extrapolated dual variable, z, the inner TV dual fields)
// from its checkpoint, and applies the transposed operators: A^T for A, A for
// A^T, D and dD/dtau for themselves (symmetric Toeplitz), and the TV reverse
// kernels for the prox.  Scalar adjoints are float64 sums gathered into
// separate device slots and added on the host in a fixed order.
//
// Execution: each problem's pass is first recorded as a list of steps (one
// kernel launch each, with that problem's pointers and scalars); the lists of
// all problems of a call have the same kinds in the same order, so the call
// runs one flattened launch per step for every problem at once (the step
// table and the block maps are uploaded once per call).  Work that a problem
// skips (the TV steps when beta = 0) is recorded as an inactive step.
#include <algorithm>
#include <vector>

#include "op.h"

using namespace ctpd;

namespace ctpd_host {

struct UnrolledWs {
    bool bufs = false;   // reverse-pass buffers allocated
    int tv_cap = -1;
    int slot_cap = 0;
    double* dtaps64 = nullptr;
    float* dtaps32 = nullptr;
    double dtap_tau = -1.0, dtap_kappa = -1.0;
    float *ax = nullptr, *axt = nullptr, *zbar = nullptr, *tbar = nullptr, *prod = nullptr;
    float *amu = nullptr, *amu2 = nullptr, *amup = nullptr, *amup2 = nullptr;
    float *ap = nullptr, *pba = nullptr, *pbb = nullptr, *qbar = nullptr;
    float *e = nullptr, *r = nullptr, *dr = nullptr, *dm = nullptr, *rbar = nullptr, *az = nullptr, *daz = nullptr,
          *dpaz = nullptr;
    float* ps = nullptr;       // tv_cap dual fields of one outer iteration (after steps 1..n_tv)
    double* part = nullptr;    // scalar-adjoint terms: part_cap block sums per slot
    double* sums = nullptr;    // one total per slot
    int part_cap = 0;          // block sums per slot
    // step executor (used when this handle is the first of a call): step
    // table and block maps, device and pinned host, and the slot totals of
    // every problem of the call
    char* xdev = nullptr;
    char* xhost = nullptr;
    size_t xcap = 0;
    double* tot_dev = nullptr;
    double* tot_host = nullptr;
    size_t tot_cap = 0;
};

void free_unrolled(UnrolledWs* u) {
    if (!u) return;
    void* ptrs[] = {u->dtaps64, u->dtaps32, u->ax,   u->axt, u->zbar, u->tbar, u->prod, u->amu,  u->amu2,
                    u->amup,    u->amup2,   u->ap,   u->pba, u->pbb,  u->qbar, u->e,    u->r,    u->dr,
                    u->dm,      u->rbar,    u->az,   u->daz, u->dpaz, u->ps,   u->part, u->sums, u->xdev,
                    u->tot_dev};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (u->xhost) (void)hipHostFree(u->xhost);
    if (u->tot_host) (void)hipHostFree(u->tot_host);
    delete u;
}

}  // namespace ctpd_host

using namespace ctpd_host;

namespace {

UnrolledWs* ws(ctpd_op* op) {
    if (!op->uw) op->uw = new UnrolledWs();
    return op->uw;
}

int ensure_unrolled(ctpd_op* op, int tv_iters, int nslots) {
    UnrolledWs* u = ws(op);
    if (!u->bufs) {
        const size_t J = op->J, I = op->I, T = 2 * (size_t)op->nb - 1;
        ALLOC(u->dtaps64, T);
        ALLOC(u->dtaps32, T);
        for (float** p : {&u->ax, &u->axt, &u->zbar, &u->tbar, &u->prod}) ALLOC(*p, J);
        for (float** p : {&u->amu, &u->amu2, &u->amup, &u->amup2, &u->e, &u->r, &u->dr, &u->dm, &u->rbar, &u->az,
                          &u->daz, &u->dpaz})
            ALLOC(*p, I);
        for (float** p : {&u->ap, &u->pba, &u->pbb, &u->qbar}) ALLOC(*p, 2 * J);
        u->bufs = true;
    }
    if (u->tv_cap < tv_iters) {
        if (u->ps) (void)hipFree(u->ps);
        u->ps = nullptr;
        u->tv_cap = -1;
        ALLOC(u->ps, (size_t)std::max(tv_iters, 1) * 2 * op->J);
        u->tv_cap = tv_iters;
    }
    const int cap = std::max(tv_bwd_blocks(op->n), reduce_blocks_for(std::max(op->I, op->J)));
    if (u->slot_cap < nslots || u->part_cap != cap) {
        if (u->part) (void)hipFree(u->part);
        if (u->sums) (void)hipFree(u->sums);
        u->part = u->sums = nullptr;
        u->slot_cap = 0;
        ALLOC(u->part, (size_t)cap * nslots);
        ALLOC(u->sums, nslots);
        u->slot_cap = nslots;
        u->part_cap = cap;
    }
    return CTPD_OK;
}

int check_args(ctpd_op* op, const float* b, const float* w, double beta, double tau, double sigma, int iters) {
    if (!op || !b || !w) return einval("null pointer");
    if (!(beta >= 0.0) || !std::isfinite(beta)) return einval("beta must be finite and >= 0");
    if (!(tau > 0.0) || !std::isfinite(tau)) return einval("tau must be finite and > 0");
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return einval("sigma must be finite and > 0");
    if (iters < 1) return einval("iters must be >= 1");
    return CTPD_OK;
}

// Each problem keeps its set-up readback and workspaces in its operator, so
// an operator may appear once per call.
int check_distinct(ctpd_op* const* ops, int count) {
    std::vector<ctpd_op*> v(ops, ops + count);
    std::sort(v.begin(), v.end());
    if (std::adjacent_find(v.begin(), v.end()) != v.end()) return einval("an operator appears twice");
    return CTPD_OK;
}

struct Slots {
    size_t x, mu, p, stride;
};

Slots layout(const ctpd_op* op) {
    const size_t J = op->J, I = op->I;
    return Slots{0, J, J + I, 3 * J + I};
}

// ---------------------------------------------------------------------------
// Recorded schedules.  Map classes: the workgroup decomposition of a step
// (tiles of a kernel, or 256 elements of a buffer of a given length).
enum MapClass : int { MC_FILT, MC_ADJ, MC_TV, MC_PAD, MC_FWD, MC_PIX, MC_J, MC_2J, MC_I, MC_CK, MC_PART, MC_DOT,
                      MC_SLOTS, MC_COUNT };

int blocks_of_class(const ctpd_op* op, int cls, const UStep& st) {
    switch (cls) {
        case MC_FILT: return filter_blocks_x(op->nb) * filter_blocks_y(op->m);
        case MC_ADJ: return adjoint_tiles(op->n) * adjoint_tiles(op->n);
        case MC_TV: return tv_tiles(op->n) * tv_tiles(op->n);
        case MC_PAD: return pad_tiles(op->n) * pad_tiles(op->n);
        case MC_FWD: return forward_blocks_x(op->nb) * op->m;
        case MC_PIX: return tv_bwd_blocks(op->n);
        case MC_DOT: return reduce_blocks_for(st.len);
        case MC_SLOTS: return (int)st.len;
        default: return (int)((st.len + 255) / 256);
    }
}

struct Rec {
    ctpd_op* op;
    std::vector<UStep> st;
    std::vector<int> cls;

    UStep& add(int kind, int c) {
        UStep u{};
        u.kind = kind;
        u.active = 1;
        u.n = op->n;
        u.m = op->m;
        u.nb = op->nb;
        u.views = op->views;
        st.push_back(u);
        cls.push_back(c);
        return st.back();
    }
    // out = e0 E0 + e1 E1 + c D(taps) s, s formed by the mode's prologue
    void filter(int mode, const float* taps, const float* in0, const float* in1, const float* in2, const float* in3,
                const float* E0, float e0, const float* E1, float e1, float c, float* out) {
        UStep& u = add(SK_FILTER, MC_FILT);
        u.taps = taps;
        u.fa.in0 = in0;
        u.fa.in1 = in1;
        u.fa.in2 = in2;
        u.fa.in3 = in3;
        u.fa.E0 = E0;
        u.fa.E1 = E1;
        u.fa.e0 = e0;
        u.fa.e1 = e1;
        u.fa.c = c;
        u.fa.mode = mode;
        u.fa.out = out;
    }
    void plain(const float* taps, const float* in, float c, float* out) {
        filter(FILT_PLAIN, taps, in, nullptr, nullptr, nullptr, nullptr, 0.f, nullptr, 0.f, c, out);
    }
    // out = xin + c A^T y
    void adjoint(const float* y, const float* xin, float c, float* out) {
        UStep& u = add(SK_ADJOINT, MC_ADJ);
        u.in[0] = y;
        u.in[1] = xin;
        u.c0 = c;
        u.out[0] = out;
    }
    void project(const float* x, float* q) {
        UStep& a = add(SK_PAD, MC_PAD);
        a.in[0] = x;
        a.out[0] = op->xp;
        a.out[1] = op->xTp;
        UStep& b = add(SK_FORWARD, MC_FWD);
        b.in[0] = op->xp;
        b.in[1] = op->xTp;
        b.out[0] = q;
    }
    void tv(const float* z, const float* pin, float* pout, float* x, float lam, float step, int steps, float* store,
            bool active) {
        UStep& u = add(SK_TV, MC_TV);
        u.active = active;
        u.in[0] = z;
        u.in[1] = pin;
        u.out[0] = pout;
        u.out[1] = x;
        u.out[2] = store;
        u.lam = lam;
        u.step = step;
        u.steps = steps;
    }
    void bwd(int kind, const float* a, const float* b, const float* c, float* o0, float* o1, float lam, float step,
             double* part, bool active) {
        UStep& u = add(kind, MC_PIX);
        u.active = active;
        u.in[0] = a;
        u.in[1] = b;
        u.in[2] = c;
        u.out[0] = o0;
        u.out[1] = o1;
        u.lam = lam;
        u.step = step;
        u.part = part;
    }
    void vec(int kind, int c, size_t len, float* out, const float* a, float c0 = 0.f, const float* b = nullptr,
             float c1 = 0.f, const float* cc = nullptr, const float* d = nullptr, float c2 = 0.f) {
        UStep& u = add(kind, c);
        u.len = len;
        u.out[0] = out;
        u.in[0] = a;
        u.in[1] = b;
        u.in[2] = cc;
        u.in[3] = d;
        u.c0 = c0;
        u.c1 = c1;
        u.c2 = c2;
    }
    void copy(int c, size_t len, float* dst, const float* src) { vec(SK_COPY, c, len, dst, src); }
    void fill(int c, size_t len, float* dst, float v) { vec(SK_FILL, c, len, dst, nullptr, v); }
    void dot(const float* a, const float* b, size_t len, double* part) {
        UStep& u = add(SK_DOT, MC_DOT);
        u.len = len;
        u.in[0] = a;
        u.in[1] = b;
        u.part = part;
    }
    void fill64(double* part, size_t len) {
        UStep& u = add(SK_FILL64, MC_PART);
        u.len = len;
        u.part = part;
    }
    void slots(const double* part, int cap, int nslots, double* out) {
        UStep& u = add(SK_SLOTS, MC_SLOTS);
        u.len = (size_t)nslots;
        u.steps = cap;
        u.part = const_cast<double*>(part);
        u.dout = out;
    }
};

// Runs the recorded lists of all problems on stream s: one launch per step.
int run_steps(std::vector<Rec>& recs, UnrolledWs* xw, hipStream_t s) {
    const int P = (int)recs.size();
    const size_t ns = recs[0].st.size();
    int max_nb = 0;
    for (const Rec& r : recs) {
        if (r.st.size() != ns) return einval("internal: schedules of different lengths");
        max_nb = std::max(max_nb, r.op->nb);
    }
    for (size_t i = 0; i < ns; ++i)
        for (int p = 1; p < P; ++p)
            if (recs[p].st[i].kind != recs[0].st[i].kind || recs[p].cls[i] != recs[0].cls[i] ||
                (recs[0].st[i].kind == SK_FILTER && recs[p].st[i].fa.mode != recs[0].st[i].fa.mode))
                return einval("internal: schedules of different steps");
    // one block map per class, from the first step of that class
    std::vector<double> work(P);
    for (int p = 0; p < P; ++p) work[p] = (double)recs[p].op->m * recs[p].op->n * recs[p].op->n;
    const Placement pl = plan_xcds(work);
    // fewer problems than XCDs: spread each problem over all of them
    const int placement = P < kXcds ? 1 : 0;
    std::vector<std::vector<BlockRef>> maps(MC_COUNT);
    std::vector<char> have(MC_COUNT, 0);
    for (size_t i = 0; i < ns; ++i) {
        const int c = recs[0].cls[i];
        if (have[c]) continue;
        have[c] = 1;
        std::vector<int> counts(P);
        for (int p = 0; p < P; ++p) counts[p] = blocks_of_class(recs[p].op, c, recs[p].st[i]);
        maps[c] = place_blocks(pl, counts, placement);
    }
    // pack: the table (step-major, P entries per step), then the maps
    const size_t table_bytes = ns * P * sizeof(UStep);
    std::vector<size_t> moff(MC_COUNT, 0);
    size_t bytes = (table_bytes + 255) / 256 * 256;
    for (int c = 0; c < MC_COUNT; ++c) {
        moff[c] = bytes;
        bytes += (maps[c].size() * sizeof(BlockRef) + 255) / 256 * 256;
    }
    if (xw->xcap < bytes) {
        if (xw->xdev) (void)hipFree(xw->xdev);
        if (xw->xhost) (void)hipHostFree(xw->xhost);
        xw->xdev = xw->xhost = nullptr;
        xw->xcap = 0;
        HIP_TRY(hipMalloc((void**)&xw->xdev, bytes));
        HIP_TRY(hipHostMalloc((void**)&xw->xhost, bytes, hipHostMallocDefault));
        xw->xcap = bytes;
    }
    UStep* th = reinterpret_cast<UStep*>(xw->xhost);
    for (size_t i = 0; i < ns; ++i)
        for (int p = 0; p < P; ++p) th[i * P + p] = recs[p].st[i];
    for (int c = 0; c < MC_COUNT; ++c)
        if (!maps[c].empty()) std::copy(maps[c].begin(), maps[c].end(), reinterpret_cast<BlockRef*>(xw->xhost + moff[c]));
    HIP_TRY(hipMemcpyAsync(xw->xdev, xw->xhost, bytes, hipMemcpyHostToDevice, s));
    const UStep* td = reinterpret_cast<const UStep*>(xw->xdev);
    for (size_t i = 0; i < ns; ++i) {
        const int c = recs[0].cls[i];
        const BlockRef* map = reinterpret_cast<const BlockRef*>(xw->xdev + moff[c]);
        const int nblk = (int)maps[c].size();
        if (nblk == 0) continue;
        const UStep* t = td + i * P;
        switch (recs[0].st[i].kind) {
            case SK_FILTER: HIP_TRY(launch_step_filter(t, map, nblk, recs[0].st[i].fa.mode, max_nb, s)); break;
            case SK_ADJOINT:
            case SK_PAD:
            case SK_FORWARD: HIP_TRY(launch_step_projector(recs[0].st[i].kind, t, map, nblk, s)); break;
            case SK_TV:
            case SK_BWD_FINAL:
            case SK_BWD_GRADPROJ:
            case SK_BWD_MASK:
            case SK_BWD_GRAD: HIP_TRY(launch_step_tv(recs[0].st[i].kind, t, map, nblk, s)); break;
            default: HIP_TRY(launch_step_vec(recs[0].st[i].kind, t, map, nblk, s)); break;
        }
    }
    return CTPD_OK;
}

// kappa = mean(1/w) with the validity scan, queued on s for every problem;
// read back after one synchronisation.
int kappa_begin(ctpd_op* op, const float* b, const float* w, hipStream_t s) {
    HIP_TRY(launch_reduce(RED_INVW_CHECK, w, b, nullptr, op->I, op->partials, op->red, s));
    HIP_TRY(hipMemcpyAsync(op->red_host, op->red, sizeof(double) * 3, hipMemcpyDeviceToHost, s));
    return CTPD_OK;
}

int kappa_end(ctpd_op* op, double* kappa) {
    if (op->red_host[1] > 0 || op->red_host[2] > 0) {
        snprintf(g_errmsg, sizeof g_errmsg, "%.0f weights <= 0 or non-finite, %.0f non-finite data",
                 op->red_host[1], op->red_host[2]);
        return CTPD_EDOMAIN;
    }
    *kappa = op->red_host[0] / (double)op->I;
    return CTPD_OK;
}

// Taps of D(tau) (and of dD/dtau when d is set) at this kappa, on stream s.
int taps_on(ctpd_op* op, double tau, double kappa, bool d, hipStream_t s) {
    if (!d) {
        if (op->tap_tau == tau && op->tap_kappa == kappa) return CTPD_OK;
        HIP_TRY(launch_taps(op->taps64, op->taps32, op->nb, op->m, tau, kappa, s));
        op->tap_tau = tau;
        op->tap_kappa = kappa;
        return CTPD_OK;
    }
    UnrolledWs* u = op->uw;
    if (u->dtap_tau == tau && u->dtap_kappa == kappa) return CTPD_OK;
    HIP_TRY(launch_taps(u->dtaps64, u->dtaps32, op->nb, op->m, tau, kappa, s, true));
    u->dtap_tau = tau;
    u->dtap_kappa = kappa;
    return CTPD_OK;
}

// Common start of a call: argument checks, then kappa of every problem (one
// synchronisation, which also drains earlier work on the handles' streams).
int begin_call(int count, ctpd_op* const* ops, const float* const* b, const float* const* w, const double* beta,
               const double* tau, const double* sigma, int iters, std::vector<double>& kappa) {
    if (count < 1 || count > CTPD_MAX_BATCH) return einval("count must be in 1..CTPD_MAX_BATCH");
    if (!ops || !b || !w || !beta || !tau || !sigma) return einval("null pointer");
    int r;
    for (int i = 0; i < count; ++i)
        if ((r = check_args(ops[i], b[i], w[i], beta[i], tau[i], sigma[i], iters))) return r;
    if ((r = check_distinct(ops, count))) return r;
    hipStream_t s = ops[0]->stream;
    for (int i = 0; i < count; ++i)
        if (ops[i]->stream != s) HIP_TRY(hipStreamSynchronize(ops[i]->stream));
    for (int i = 0; i < count; ++i)
        if ((r = kappa_begin(ops[i], b[i], w[i], s))) return r;
    HIP_TRY(hipStreamSynchronize(s));
    kappa.assign(count, 0.0);
    for (int i = 0; i < count; ++i)
        if ((r = kappa_end(ops[i], &kappa[i]))) return r;
    return CTPD_OK;
}

// The forward iterations of one problem.
void record_forward(Rec& R, const float* b, const float* w, double beta, double tau, double sigma, int iters,
                    const Knobs& k, float* ckpt, float* x_out) {
    ctpd_op* op = R.op;
    const size_t J = op->J, I = op->I;
    const Slots L = layout(op);
    auto X = [&](int i) { return ckpt + (size_t)i * L.stride + L.x; };
    auto MU = [&](int i) { return ckpt + (size_t)i * L.stride + L.mu; };
    auto P = [&](int i) { return ckpt + (size_t)i * L.stride + L.p; };
    const float fs = (float)sigma, ft = (float)tau, lam = (float)(tau * beta);
    const float tvstep = lam > 0 ? (float)(k.tv_step / (tau * beta)) : 0.f;
    const float* taps = op->taps32;
    const int chunk = tv_chunk_max();
    R.vec(SK_INV, MC_I, I, op->winv, w);
    R.fill(MC_CK, L.stride, ckpt, 0.f);
    for (int it = 0; it < iters; ++it) {
        float *x = X(it), *mu = MU(it), *mup = MU(it > 0 ? it - 1 : 0);
        if (it == 0) {
            // x = 0, mubar = -sigma D b: z = -sigma (x - tau A^T D b), the solver's order
            R.plain(taps, b, 1.f, op->mubar);
            R.adjoint(op->mubar, x, -ft, op->z);
            R.vec(SK_LIN3, MC_J, J, op->z, op->z, -fs);
        } else {
            R.filter(FILT_EXTRAP, taps, op->winv, mu, mup, nullptr, mu, 2.f, mup, -1.f, -fs, op->mubar);
            R.adjoint(op->mubar, x, -ft, op->z);
        }
        R.copy(MC_2J, 2 * J, op->p[0], P(it));
        // the prox: chunks of dual steps ping-ponging p[0] / p[1], x on the last
        // (lam == 0: x = max(0, z) and p stays)
        float *src = op->p[0], *dst = op->p[1];
        int left = k.tv_iters;
        do {
            const int st = std::min(left, chunk);
            left -= st;
            R.tv(op->z, src, dst, left == 0 ? X(it + 1) : nullptr, lam, tvstep, st, nullptr, true);
            if (lam > 0) std::swap(src, dst);
        } while (left > 0);
        R.copy(MC_2J, 2 * J, P(it + 1), src);
        R.project(X(it + 1), op->q);
        R.filter(FILT_DUAL_LD, taps, op->q, b, op->winv, mu, mu, 1.f, nullptr, 0.f, fs, MU(it + 1));
    }
    R.copy(MC_J, J, x_out, X(iters));
}

enum Cat { C_SIGMA, C_TAU, C_LAM, C_STEP };

// The reverse pass of one problem; terms receives the category and factor of
// every scalar slot (totals land at tot[0 .. terms.size())).
void record_backward(Rec& R, const float* b, const float* w, double beta, double tau, double sigma, int iters,
                     const Knobs& k, const float* ckpt, const float* x_grad, float* b_grad, double* tot,
                     std::vector<std::pair<int, double>>& terms) {
    ctpd_op* op = R.op;
    UnrolledWs* u = op->uw;
    const int nt = k.tv_iters;
    const int per_iter = 2 * nt + 6;
    const size_t J = op->J, I = op->I;
    const Slots L = layout(op);
    auto X = [&](int i) { return ckpt + (size_t)i * L.stride + L.x; };
    auto MU = [&](int i) { return ckpt + (size_t)i * L.stride + L.mu; };
    auto P = [&](int i) { return ckpt + (size_t)i * L.stride + L.p; };
    const float fs = (float)sigma, ft = (float)tau, lam = (float)(tau * beta);
    const float tvstep = lam > 0 ? (float)(k.tv_step / (tau * beta)) : 0.f;
    const bool tv_on = lam > 0;
    const float* taps = op->taps32;
    const float* dtaps = u->dtaps32;
    // Scalar-adjoint terms: every term gets a slot of part_cap block sums
    // (written by the steps that produce it), reduced once at the end and
    // added up on the host by category in a fixed order.
    terms.clear();
    auto slot = [&](int cat, double factor) -> double* {
        terms.emplace_back(cat, factor);
        return u->part + (size_t)(terms.size() - 1) * u->part_cap;
    };
    auto dot = [&](int cat, double factor, const float* a, const float* bb) { R.dot(a, bb, I, slot(cat, factor)); };
    R.vec(SK_INV, MC_I, I, op->winv, w);
    R.fill64(u->part, (size_t)u->part_cap * iters * per_iter);
    // adjoint state of (x^{k+1}, mu^{k+1}, mu^k as the next iteration's mu_prev, p^{k+1})
    float *ax = u->ax, *zbar = u->zbar, *amu = u->amu, *amu2 = u->amu2, *amup = u->amup, *amup2 = u->amup2;
    float *ap = u->ap, *pba = u->pba;
    R.copy(MC_J, J, ax, x_grad);
    R.fill(MC_I, I, amu, 0.f);
    R.fill(MC_I, I, amup, 0.f);
    R.fill(MC_2J, 2 * J, ap, 0.f);
    R.fill(MC_I, I, b_grad, 0.f);
    const int chunk = tv_chunk_max();
    for (int it = iters - 1; it >= 0; --it) {
        const float *x = X(it), *mu = MU(it), *mup = MU(it > 0 ? it - 1 : 0), *x1 = X(it + 1);
        // recompute the extrapolated dual variable, z and the inner dual fields
        const float* e = b;
        if (it == 0) {
            // the forward pass's z (u->e holds D b), and mubar = -sigma D b for the tau term below
            R.plain(taps, b, 1.f, u->e);
            R.adjoint(u->e, x, -ft, op->z);
            R.vec(SK_LIN3, MC_J, J, op->z, op->z, -fs);
            R.vec(SK_LIN3, MC_I, I, op->mubar, u->e, -fs);
        } else {
            R.vec(SK_LIN3, MC_I, I, u->e, mu, 1.f, mup, -1.f, nullptr, op->winv, 0.f);
            e = u->e;
            R.filter(FILT_EXTRAP, taps, op->winv, mu, mup, nullptr, mu, 2.f, mup, -1.f, -fs, op->mubar);
            R.adjoint(op->mubar, x, -ft, op->z);
        }
        // PS(i): dual field after inner step i (PS(0) = p^k from the checkpoint)
        auto PS = [&](int i) -> const float* { return i == 0 ? P(it) : u->ps + (size_t)(i - 1) * 2 * J; };
        if (nt > 0) {
            if (nt <= chunk) {
                R.tv(op->z, P(it), u->ps + (size_t)(nt - 1) * 2 * J, nullptr, lam, tvstep, nt, u->ps, tv_on);
            } else {
                for (int i = 1; i <= nt; ++i)
                    R.tv(op->z, PS(i - 1), u->ps + (size_t)(i - 1) * 2 * J, nullptr, lam, tvstep, 1, nullptr, tv_on);
            }
        }
        R.project(x1, op->q);
        R.vec(SK_LINMIX, MC_I, I, u->r, op->q, 1.f, b, -1.f, op->winv, mu, -1.f);
        // mu^{k+1} = mu + sigma D r
        R.plain(taps, u->r, 1.f, u->dr);
        dot(C_SIGMA, 1.0, amu, u->dr);
        R.plain(dtaps, amu, 1.f, u->dm);
        dot(C_TAU, sigma, u->dm, u->r);
        R.plain(taps, amu, fs, u->rbar);
        // r = A x^{k+1} - b - W^-1 mu
        R.vec(SK_LINMIX, MC_I, I, amu2, amu, 1.f, amup, 1.f, op->winv, u->rbar, -1.f);
        R.adjoint(u->rbar, ax, 1.f, u->axt);
        R.vec(SK_LINMIX, MC_I, I, b_grad, b_grad, 1.f, u->rbar, -1.f);
        // x^{k+1}, p^{k+1} = prox(z, p^k); with lam == 0, x^{k+1} = max(0, z) and p passes through
        R.bwd(SK_BWD_FINAL, op->z, tv_on ? PS(nt) : P(it), u->axt, u->tbar, zbar, lam, 0.f,
              slot(C_LAM, tv_on ? 1.0 : 0.0), true);
        // the adjoint of p^{k+1} (ap) becomes the first qbar buffer
        for (int i = nt; i >= 1; --i) {
            R.bwd(SK_BWD_GRADPROJ, op->z, PS(i - 1), u->tbar, ap, nullptr, lam, tvstep,
                  tv_on ? slot(C_STEP, 1.0) : nullptr, tv_on);
            R.bwd(SK_BWD_MASK, op->z, PS(i - 1), ap, u->tbar, zbar, lam, tvstep, tv_on ? slot(C_LAM, 1.0) : nullptr,
                  tv_on);
        }
        R.bwd(SK_BWD_GRAD, ap, u->tbar, nullptr, pba, nullptr, lam, 0.f, nullptr, tv_on);
        if (tv_on) std::swap(ap, pba);
        // z = x^k - tau A^T mubar
        R.project(zbar, u->az);
        dot(C_TAU, -1.0, u->az, op->mubar);
        R.plain(taps, u->az, 1.f, u->daz);
        R.plain(dtaps, u->az, 1.f, u->dpaz);
        dot(C_SIGMA, tau, u->daz, e);
        dot(C_TAU, sigma * tau, u->dpaz, e);
        if (it == 0) {
            R.vec(SK_LINMIX, MC_I, I, b_grad, b_grad, 1.f, u->daz, (float)(sigma * tau));
        } else {
            R.vec(SK_LINMIX, MC_I, I, amu2, amu2, 1.f, u->az, (float)(-2.0 * tau), op->winv, u->daz,
                  (float)(sigma * tau));
            R.vec(SK_LINMIX, MC_I, I, amup2, u->az, ft, nullptr, 0.f, op->winv, u->daz, (float)(-sigma * tau));
        }
        std::swap(ax, zbar);
        std::swap(amu, amu2);
        std::swap(amup, amup2);
    }
    R.slots(u->part, u->part_cap, (int)terms.size(), tot);
}

// d/dbeta, d/dtau, d/dsigma from the scalar terms' totals.
void combine_terms(const double* tot, const std::vector<std::pair<int, double>>& terms, double beta, double tau,
                   double tv_step, double* grads) {
    double g_sigma = 0.0, g_tau = 0.0, g_lam = 0.0, g_step = 0.0;
    for (size_t i = 0; i < terms.size(); ++i) {
        const double v = terms[i].second * tot[i];
        switch (terms[i].first) {
            case C_SIGMA: g_sigma += v; break;
            case C_TAU: g_tau += v; break;
            case C_LAM: g_lam += v; break;
            default: g_step += v; break;
        }
    }
    if (tau * beta > 0) g_lam += g_step * (-tv_step / ((tau * beta) * (tau * beta)));
    grads[0] = tau * g_lam;            // d/dbeta  (lam = tau beta)
    grads[1] = g_tau + beta * g_lam;   // d/dtau
    grads[2] = g_sigma;                // d/dsigma
}

}  // namespace

extern "C" {

int ctpd_unrolled_ckpt_floats(const ctpd_op* op, int32_t iters, size_t* count) {
    g_errmsg[0] = 0;
    if (!op || !count) return einval("null pointer");
    if (iters < 1) return einval("iters must be >= 1");
    *count = (size_t)(iters + 1) * layout(op).stride;
    return CTPD_OK;
}

int ctpd_unrolled_lowdose_forward_many(int32_t count, ctpd_op* const* ops, const float* const* b,
                                       const float* const* w, const double* beta, const double* tau,
                                       const double* sigma, int32_t iters, const ctpd_params* p,
                                       float* const* ckpt, float* const* x_out) {
    g_errmsg[0] = 0;
    if (!ckpt || !x_out) return einval("null pointer");
    for (int i = 0; i < count && i < CTPD_MAX_BATCH; ++i)
        if (!ckpt[i] || !x_out[i]) return einval("null pointer");
    Knobs k;
    int r;
    if ((r = read_params(p, &k))) return r;
    if ((r = no_state(k))) return r;
    std::vector<double> kappa;
    if ((r = begin_call(count, ops, b, w, beta, tau, sigma, iters, kappa))) return r;
    hipStream_t s = ops[0]->stream;
    std::vector<Rec> recs(count);
    for (int i = 0; i < count; ++i) {
        if ((r = taps_on(ops[i], tau[i], kappa[i], false, s))) return r;
        recs[i].op = ops[i];
        record_forward(recs[i], b[i], w[i], beta[i], tau[i], sigma[i], iters, k, ckpt[i], x_out[i]);
    }
    return run_steps(recs, ws(ops[0]), s);
}

int ctpd_unrolled_lowdose_forward(ctpd_op* op, const float* b, const float* w, double beta, double tau,
                                  double sigma, int32_t iters, const ctpd_params* p, float* ckpt, float* x_out) {
    return ctpd_unrolled_lowdose_forward_many(1, &op, &b, &w, &beta, &tau, &sigma, iters, p, &ckpt, &x_out);
}

int ctpd_unrolled_lowdose_backward_many(int32_t count, ctpd_op* const* ops, const float* const* b,
                                        const float* const* w, const double* beta, const double* tau,
                                        const double* sigma, int32_t iters, const ctpd_params* p,
                                        const float* const* ckpt, const float* const* x_grad, float* const* b_grad,
                                        double* grads) {
    g_errmsg[0] = 0;
    if (!ckpt || !x_grad || !b_grad || !grads) return einval("null pointer");
    for (int i = 0; i < count && i < CTPD_MAX_BATCH; ++i)
        if (!ckpt[i] || !x_grad[i] || !b_grad[i]) return einval("null pointer");
    Knobs k;
    int r;
    if ((r = read_params(p, &k))) return r;
    if ((r = no_state(k))) return r;
    std::vector<double> kappa;
    if ((r = begin_call(count, ops, b, w, beta, tau, sigma, iters, kappa))) return r;
    hipStream_t s = ops[0]->stream;
    const int per_iter = 2 * k.tv_iters + 6;
    const size_t nslot = (size_t)iters * per_iter;
    UnrolledWs* xw = ws(ops[0]);
    if (xw->tot_cap < nslot * count) {
        if (xw->tot_dev) (void)hipFree(xw->tot_dev);
        if (xw->tot_host) (void)hipHostFree(xw->tot_host);
        xw->tot_dev = xw->tot_host = nullptr;
        xw->tot_cap = 0;
        ALLOC(xw->tot_dev, nslot * count);
        HIP_TRY(hipHostMalloc((void**)&xw->tot_host, sizeof(double) * nslot * count, hipHostMallocDefault));
        xw->tot_cap = nslot * count;
    }
    std::vector<Rec> recs(count);
    std::vector<std::vector<std::pair<int, double>>> terms(count);
    for (int i = 0; i < count; ++i) {
        if ((r = ensure_unrolled(ops[i], k.tv_iters, (int)nslot))) return r;
        if ((r = taps_on(ops[i], tau[i], kappa[i], false, s))) return r;
        if ((r = taps_on(ops[i], tau[i], kappa[i], true, s))) return r;
        recs[i].op = ops[i];
        record_backward(recs[i], b[i], w[i], beta[i], tau[i], sigma[i], iters, k, ckpt[i], x_grad[i], b_grad[i],
                        xw->tot_dev + nslot * i, terms[i]);
    }
    if ((r = run_steps(recs, xw, s))) return r;
    HIP_TRY(hipMemcpyAsync(xw->tot_host, xw->tot_dev, sizeof(double) * nslot * count, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int i = 0; i < count; ++i)
        combine_terms(xw->tot_host + nslot * i, terms[i], beta[i], tau[i], k.tv_step, grads + 3 * i);
    return CTPD_OK;
}

int ctpd_unrolled_lowdose_backward(ctpd_op* op, const float* b, const float* w, double beta, double tau,
                                   double sigma, int32_t iters, const ctpd_params* p, const float* ckpt,
                                   const float* x_grad, float* b_grad, double* grads) {
    return ctpd_unrolled_lowdose_backward_many(1, &op, &b, &w, &beta, &tau, &sigma, iters, p, &ckpt, &x_grad,
                                               &b_grad, grads);
}

}  // extern "C"
