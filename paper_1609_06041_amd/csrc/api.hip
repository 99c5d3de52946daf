// C ABI of libctpd: operator handle, single operators, and the two APP
// solvers (Algorithm 1 / 1' for low-dose data, Algorithm 2 for few-view
// data).  The host code here validates arguments, sets up the geometry and
// step sizes, and queues kernels; every array operation runs on the GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <vector>

#include "op.h"

using namespace ctpd;


namespace ctpd_host {

thread_local char g_errmsg[512] = "";

int fail_hip(hipError_t e, const char* what) {
    snprintf(g_errmsg, sizeof g_errmsg, "%s: %s", what, hipGetErrorString(e));
    return CTPD_EHIP;
}


int alloc_dev(void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes ? bytes : 1);
    if (e == hipErrorOutOfMemory) {
        snprintf(g_errmsg, sizeof g_errmsg, "hipMalloc(%zu bytes): out of memory", bytes);
        return CTPD_ENOMEM;
    }
    if (e != hipSuccess) return fail_hip(e, "hipMalloc");
    return CTPD_OK;
}


int einval(const char* msg) {
    snprintf(g_errmsg, sizeof g_errmsg, "invalid argument: %s", msg);
    return CTPD_EINVAL;
}

// Per-view geometry in float64 (see ViewGeom).
// View tables.  Default angles v pi / m take the row branch for 4v <= m or
// 4v >= 3m (the 45-degree ties decided from the index); given angles where
// |cos| >= |sin| (1 - 1e-12), so near-diagonal views go to the row branch
// whichever way cos and sin round.
std::vector<ViewGeom> make_views(int n, int m, int nb, const double* angles) {
    std::vector<ViewGeom> out(m);
    const double c = 0.5 * (n - 1), cd = 0.5 * (nb - 1);
    for (int v = 0; v < m; ++v) {
        const double th = angles ? angles[v] : (double)v * M_PI / (double)m;
        const double cs = std::cos(th), sn = std::sin(th);
        ViewGeom g{};
        g.row = angles ? (std::fabs(cs) >= std::fabs(sn) * (1.0 - 1e-12) ? 1 : 0)
                       : ((4 * v <= m || 4 * v >= 3 * m) ? 1 : 0);
        g.cs = cs;
        g.sn = sn;
        // row views:    s = (r_u - Y_t sin)/cos + c,  column views: s = (r_u - X_t cos)/sin + c
        const double a = g.row ? cs : sn, o = g.row ? sn : cs;
        g.su = 1.0 / a;
        g.st = -o / a;
        g.s0 = (c * o - cd) / a + c;
        g.len = 1.0 / std::fabs(a);
        g.len2 = g.len * g.len;
        out[v] = g;
    }
    return out;
}

int sync(ctpd_op* op) {
    HIP_TRY(hipStreamSynchronize(op->stream));
    return CTPD_OK;
}

int ensure_taps(ctpd_op* op, double tau, double kappa) {
    if (op->tap_tau == tau && op->tap_kappa == kappa) return CTPD_OK;
    HIP_TRY(launch_taps(op->taps64, op->taps32, op->nb, op->m, tau, kappa, op->stream));
    op->tap_tau = tau;
    op->tap_kappa = kappa;
    return CTPD_OK;
}

int ensure_sym(ctpd_op* op) {
    if (!op->hv_sym) ALLOC(op->hv_sym, 1 + kSymBlocks);
    return CTPD_OK;
}

int ensure_taps_default(ctpd_op* op, double kappa) {
    const double tau = kTauMultLowdose * M_PI * kappa / (2.0 * op->m);
    if (op->tap_tau == tau && op->tap_kappa == kappa) return CTPD_OK;
    const int ntap = 2 * op->nb - 1;
    if (!op->taps1) {
        ALLOC(op->taps1, ntap);
        ALLOC(op->sym1, 1 + kSymBlocks);
        // taps32 is overwritten below
        HIP_TRY(launch_taps(op->taps1, op->taps32, op->nb, op->m, kTauMultLowdose * M_PI / (2.0 * op->m), 1.0,
                            op->stream));
        HIP_TRY(launch_symbol_max(op->taps1, op->nb, op->sym1, op->stream));
    }
    int r;
    if ((r = ensure_sym(op))) return r;
    HIP_TRY(launch_taps_scale(op->taps1, ntap, kappa, op->taps64, op->taps32, op->sym1, op->hv_sym, op->stream));
    op->tap_tau = tau;
    op->tap_kappa = kappa;
    op->hv_sym_tau = tau;
    op->hv_sym_kappa = kappa;
    return CTPD_OK;
}

int ensure_f64(ctpd_op* op) {
    if (op->img64[0]) return CTPD_OK;
    for (auto& p : op->img64) ALLOC(p, op->J);
    for (auto& p : op->pad64) ALLOC(p, op->Jp);
    for (auto& p : op->sino64) ALLOC(p, op->I);
    return CTPD_OK;
}

// Reduction into slot `slot` of op->red (device); read back with read_red.
int reduce(ctpd_op* op, int kind, const void* a, const void* b, const void* c, size_t len, int slot) {
    HIP_TRY(launch_reduce(kind, a, b, c, len, op->partials, op->red + 3 * slot, op->stream));
    return CTPD_OK;
}

int read_red(ctpd_op* op) {
    HIP_TRY(hipMemcpyAsync(op->red_host, op->red, sizeof(double) * 3 * kRedSlots, hipMemcpyDeviceToHost,
                           op->stream));
    return sync(op);
}

// Largest eigenvalue of a symmetric operator M (float64) by the Lanczos
// recurrence without reorthogonalisation: for the extreme eigenvalue the
// Ritz value converges even after orthogonality is lost (at worst copies of
// it appear).  Stops when the top Ritz value changes by <= 1e-9 relative.
// The Ritz value is the top eigenvalue of the tridiagonal matrix (alpha, beta).
double tridiag_max(const std::vector<double>& a, const std::vector<double>& b) {
    // a: diagonal (k), b: off-diagonal (k-1).  Sturm-sequence bisection.
    const int k = (int)a.size();
    double lo = a[0], hi = a[0];
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i < k - 1 ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    auto count_below = [&](double x) {
        int cnt = 0;
        double d = 1.0;
        for (int i = 0; i < k; ++i) {
            d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
            if (d == 0.0) d = -1e-300;
            if (d < 0.0) ++cnt;
        }
        return cnt;
    };
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (count_below(mid) == k) hi = mid;
        else lo = mid;
    }
    return hi;
}

// Lanczos with the recurrence scalars kept on the device: the kernels read
// alpha_j and beta_j from device memory, and the host only copies them back
// every few steps to evaluate the top Ritz value (so the queue never drains
// between steps).  Device slots (3 doubles each): [0] start norm^2,
// [1 + j] alpha_j, [1 + cap + j] beta_{j+1}^2.  Two chains (the two operator
// norms of the low-dose solve) can run at once, each on its own stream with
// its own scalar and partial-sum buffers.
int ensure_lz(ctpd_op* op, int kmax) {
    if (op->lz_cap >= kmax) return CTPD_OK;
    for (int c = 0; c < 2; ++c) {
        if (op->lz[c]) (void)hipFree(op->lz[c]);
        if (op->lz_host[c]) (void)hipHostFree(op->lz_host[c]);
        op->lz[c] = nullptr;
        op->lz_host[c] = nullptr;
    }
    op->lz_cap = 0;
    const size_t cnt = (size_t)3 * (2 * kmax + 1);
    for (int c = 0; c < 2; ++c) {
        ALLOC(op->lz[c], cnt);
        HIP_TRY(hipHostMalloc((void**)&op->lz_host[c], sizeof(double) * cnt, hipHostMallocDefault));
        if (!op->lz_partials[c]) ALLOC(op->lz_partials[c], 3 * kReduceBlocks);
    }
    op->lz_cap = kmax;
    return CTPD_OK;
}


// Run Lanczos chains to convergence together: each round queues
// `per_round` steps of every unfinished chain on its own stream, then
// synchronises and checks them all.
int run_lanczos(const std::vector<Lanczos*>& chains) {
    for (;;) {
        bool any = false;
        for (Lanczos* c : chains)
            if (!c->finished()) {
                int r = c->enqueue(c->per_round);
                if (r) return r;
                any = true;
            }
        if (!any) return CTPD_OK;
        for (Lanczos* c : chains) HIP_TRY(hipStreamSynchronize(c->s));
        for (Lanczos* c : chains)
            if (!c->finished()) c->absorb();
    }
}

// lambda_max(A^T D A) with the float64 operators and the taps in op->taps64,
// on op->stream; with filt == false the middle factor is W = diag(wgt)
// (wgt given) or the identity instead of D.
int setup_lambda_a(ctpd_op* op, int kmax, Lanczos* L, bool filt, const float* wgt) {
    int r = ensure_f64(op);
    if (r) return r;
    if ((r = ensure_lz(op, kmax))) return r;
    double *s1 = op->sino64[4], *s2 = op->sino64[5];
    hipStream_t s = op->stream;
    L->op = op;
    L->chain = 0;
    L->per_round = 4;   // a step costs ~0.3 ms at 512^2: check often so little is queued past convergence
    L->s = s;
    L->q = op->img64[0];
    L->qp = op->img64[1];
    L->w = op->img64[2];
    L->kmax = kmax;
    L->apply = [op, s1, s2, s, filt, wgt](const double* in, double* out) -> int {
        HIP_TRY(launch_pad_planes<double>(in, op->pad64[0], op->pad64[1], op->n, s));
        HIP_TRY(launch_forward<double>(op->pad64[0], op->pad64[1], filt || wgt ? s1 : s2, op->views, op->n, op->m,
                                       op->nb, s));
        if (filt)
            HIP_TRY(launch_filter_f64(s1, s2, op->taps64, nullptr, nullptr, op->m, op->nb, s));
        else if (wgt)
            HIP_TRY(launch_mul_w_f64(s2, s1, wgt, op->I, s));
        HIP_TRY(launch_adjoint<double>(s2, nullptr, 1.0, 0.0, nullptr, 0.0, 1.0, out, op->views, op->n, op->m,
                                       op->nb, s));
        return CTPD_OK;
    };
    return L->start(op->n, op->n, 1, nullptr, 0.0);
}


int filter(ctpd_op* op, int mode, const float* in0, const float* in1, const float* in2, const float* in3,
           const float* E0, float e0, const float* E1, float e1, float c, float* out, const float* Sw,
           float* Sout) {
    FilterArgs a{};
    a.Sw = Sw;
    a.Sout = Sout;
    a.in0 = in0;
    a.in1 = in1;
    a.in2 = in2;
    a.in3 = in3;
    a.E0 = E0;
    a.E1 = E1;
    a.e0 = e0;
    a.e1 = e1;
    a.c = c;
    a.mode = mode;
    a.out = out;
    HIP_TRY(launch_filter_f32(a, op->taps32, op->m, op->nb, op->stream));
    return CTPD_OK;
}

// y = A x - rb - rw .* rm (rw null: A x - rb): the dual update's filter input
// written by the projector itself
int project_resid(ctpd_op* op, const float* x, const float* rb, const float* rw, const float* rm, float* y,
                  bool padded) {
    if (!padded) HIP_TRY(launch_pad_planes<float>(x, op->xp, op->xTp, op->n, op->stream));
    HIP_TRY(launch_forward_auto(op->xp, op->xTp, y, op->views, op->fwd_tasks, op->fwd_groups, op->n, op->m, op->nb,
                                rb, rw, rm, op->stream));
    return CTPD_OK;
}

int project(ctpd_op* op, const float* x, float* y) {
    return project_resid(op, x, nullptr, nullptr, nullptr, y);
}

// n_iter dual steps on p (warm start in pin; result pointer returned in *pout,
// which is either pin or scratch, both used as ping-pong buffers), then
// x = max(0, z - lam div p).  lam == 0 gives x = max(0, z) and leaves p alone.
int tv_prox(ctpd_op* op, const float* z, float lam, int n_iter, float step, float* pin, float* scratch, float* x,
            float** pout, bool planes) {
    float* pf = pin;
    if (lam > 0.0f)
        HIP_TRY(launch_tv_prox(z, pin, scratch, x, op->n, lam, step, n_iter, &pf, op->stream,
                               planes ? op->xp : nullptr, planes ? op->xTp : nullptr));
    else
        HIP_TRY(launch_tv_finalize(z, pin, x, op->n, 0.0f, op->stream));
    if (pout) *pout = pf;
    return CTPD_OK;
}


// Algorithm 1's iterations (Eqs. 18-20) from zero with the handle's taps as D
// and the given steps, queued on the handle's stream; *p_final receives the
// buffer holding the final dual field of the TV prox.
// x^0 = 0, mu^0 = 0 (and the mu^{-1} of the first extrapolation), p = 0
int lowdose_zero(ctpd_op* op) {
    const size_t I = op->I, J = op->J;
    hipStream_t s = op->stream;
    HIP_TRY(launch_zero4_f32(op->x, J, op->p[0], 2 * J, op->mu[0], I, op->mu[1], I, s));
    return CTPD_OK;
}

// z_ready: op->z holds x - tau A^T D b at x = 0 (the first iteration's z is
// -sigma times it); else the first iteration forms it
int lowdose_loop(ctpd_op* op, const float* b, const float* w, double beta, int iters, const Knobs& k, double tau,
                 double sigma, float** p_final, const Monitors& M, bool zeroed = false, bool z_ready = false) {
    int r = CTPD_OK;
    hipStream_t s = op->stream;
    if (k.record && (r = ensure_cost(op, iters))) return r;
    if (!zeroed && (r = lowdose_zero(op))) return r;
    float *mu = op->mu[0], *mup = op->mu[1], *mun = op->mu[2];
    float* pcur = op->p[0];
    const float fs = (float)sigma, ft = (float)tau, lam = (float)(tau * beta);
    const float tvstep = lam > 0 ? (float)(k.tv_step / (tau * beta)) : 0.f;
    // Without the cost monitor the two filters run on inputs written by the
    // kernels before them (same arithmetic as the fused prologues): the
    // projector writes r = A x - b - W^-1 mu, and the dual update writes
    // W^-1 (mu^{k+1} - mu^k) for the next extrapolation.
    const bool fused = !k.record;
    for (int it = 0; it < iters; ++it) {
        // Step 1: extrapolation (Eq. 18 / Algorithm 1); a resumed state's first
        // iteration forms W^-1 (mu^k - mu^{k-1}) in the filter's prologue.
        // Step 2: z = x - tau A^T mubar, x = prox(z; tau beta)
        if (it == 0 && !k.resumed()) {
            // x = 0, mubar = -sigma D b: z = -sigma (x - tau A^T D b)
            if (!z_ready) {
                if ((r = filter(op, FILT_PLAIN, b, nullptr, nullptr, nullptr, nullptr, 0.f, nullptr, 0.f, 1.f,
                                op->mubar)))
                    return r;
                HIP_TRY(launch_adjoint<float>(op->mubar, nullptr, 1.f, 0.f, op->x, 1.f, -ft, op->z, op->views,
                                              op->n, op->m, op->nb, s));
            }
            HIP_TRY(launch_lin3_f32(op->z, op->z, -fs, nullptr, 0.f, nullptr, 0.f, nullptr, op->J, s));
        } else {
            if (fused && it > 0)
                r = filter(op, FILT_PLAIN, op->sx, nullptr, nullptr, nullptr, mu, 2.f, mup, -1.f, -fs, op->mubar);
            else
                r = filter(op, FILT_EXTRAP, op->winv, mu, mup, nullptr, mu, 2.f, mup, -1.f, -fs, op->mubar);
            if (r) return r;
            HIP_TRY(launch_adjoint<float>(op->mubar, nullptr, 1.f, 0.f, op->x, 1.f, -ft, op->z, op->views, op->n,
                                          op->m, op->nb, s));
        }
        float* pnew = nullptr;
        // the prox also writes the projector's planes of x (not the beta = 0 clamp)
        const bool padded = lam > 0.f;
        if ((r = tv_prox(op, op->z, lam, k.tv_iters, tvstep, pcur, pcur == op->p[0] ? op->p[1] : op->p[0], op->x,
                         &pnew, true)))
            return r;
        pcur = pnew;
        // Step 3: mu^{k+1} = mu^k + sigma D (A x^{k+1} - b - W^-1 mu^k)
        if (fused) {
            if ((r = project_resid(op, op->x, b, op->winv, mu, op->q, padded))) return r;
            if ((r = filter(op, FILT_PLAIN, op->q, nullptr, nullptr, nullptr, mu, 1.f, nullptr, 0.f, fs, mun,
                            op->winv, op->sx)))
                return r;
        } else {
            if ((r = project_resid(op, op->x, nullptr, nullptr, nullptr, op->q, padded))) return r;
            if ((r = filter(op, FILT_DUAL_LD, op->q, b, op->winv, mu, mu, 1.f, nullptr, 0.f, fs, mun))) return r;
        }
        if (k.record && (r = record_monitors(op, it, M, op->x, op->q, b, w, mun))) return r;
        float* t = mup;
        mup = mu;
        mu = mun;
        mun = t;
    }
    (void)s;
    op->mu[0] = mu;
    op->mu[1] = mup;
    op->mu[2] = mun;
    *p_final = pcur;
    return CTPD_OK;
}

int read_params(const ctpd_params* p, Knobs* k) {
    k->tau = 0.0;
    k->sigma = 0.0;
    k->tv_step = 0.125;
    k->rho = 0.95;
    k->tv_iters = 10;
    k->norm_steps = 100;
    k->record = 0;
    k->state = nullptr;
    if (!p) return CTPD_OK;
    if (!(std::isfinite(p->tau) && std::isfinite(p->sigma) && std::isfinite(p->tv_step) &&
          std::isfinite(p->safety)))
        return einval("non-finite parameter");
    if (p->tau > 0) k->tau = p->tau;
    if (p->sigma > 0) k->sigma = p->sigma;
    if (p->tv_step > 0) k->tv_step = p->tv_step;
    if (p->safety > 0) {
        if (p->safety >= 1.0) return einval("safety must be < 1");
        k->rho = p->safety;
    }
    if (p->tv_iters > 0) k->tv_iters = p->tv_iters;
    if (p->norm_steps > CTPD_MAX_NORM_STEPS) return einval("norm_steps above CTPD_MAX_NORM_STEPS");
    if (p->norm_steps > 0) k->norm_steps = p->norm_steps;
    k->record = p->record_cost ? 1 : 0;
    if (ctpd_state* st = p->state) {
        if (st->k < 0) return einval("state k < 0");
        if (!st->x || !st->mu || !st->mu_prev || !st->p) return einval("null pointer in the state");
        if (st->k > 0) {
            if (!(st->tau > 0 && std::isfinite(st->tau) && st->sigma > 0 && std::isfinite(st->sigma)))
                return einval("a resumed state needs its tau and sigma (finite, > 0)");
            k->tau = st->tau;   // the state's step sizes (checked like given ones)
            k->sigma = st->sigma;
        }
        k->state = st;
    }
    return CTPD_OK;
}

// For the solvers without checkpoints.
int no_state(const Knobs& k) {
    return k.state ? einval("a checkpoint state is taken by the APP solvers only (low-dose, few-view, "
                            "error-tolerant few-view)")
                   : CTPD_OK;
}

// The iterates of a resumed state into the handle's buffers the loops start
// from (x, p[0], mu[0] = mu^k, mu[1] = mu^{k-1}, and y).
int load_state(ctpd_op* op, const ctpd_state* st, float* y) {
    const size_t I = op->I, J = op->J;
    hipStream_t s = op->stream;
    HIP_TRY(launch_copy_f32(op->x, st->x, J, s));
    HIP_TRY(launch_copy_f32(op->p[0], st->p, 2 * J, s));
    HIP_TRY(launch_copy_f32(op->mu[0], st->mu, I, s));
    HIP_TRY(launch_copy_f32(op->mu[1], st->mu_prev, I, s));
    if (y) HIP_TRY(launch_copy_f32(y, st->y, I, s));
    return CTPD_OK;
}

// The state after a loop (mu^K in op->mu[0], mu^{K-1} in op->mu[1]).
int save_state(ctpd_op* op, ctpd_state* st, const float* p_final, const float* y, int iters, double tau,
               double sigma) {
    const size_t I = op->I, J = op->J;
    hipStream_t s = op->stream;
    HIP_TRY(launch_copy_f32(st->x, op->x, J, s));
    HIP_TRY(launch_copy_f32(st->p, p_final, 2 * J, s));
    HIP_TRY(launch_copy_f32(st->mu, op->mu[0], I, s));
    HIP_TRY(launch_copy_f32(st->mu_prev, op->mu[1], I, s));
    if (y) HIP_TRY(launch_copy_f32(st->y, y, I, s));
    st->k += iters;
    st->tau = tau;
    st->sigma = sigma;
    return CTPD_OK;
}

int read_monitors(const ctpd_report* rep, bool gap_ok, Knobs* k, Monitors* M) {
    *M = Monitors{};
    M->cost = k->record != 0;
    if (rep) {
        M->gap = rep->gap != nullptr;
        M->resid = rep->resid != nullptr;
        M->rmse = rep->rmse != nullptr;
        M->x_ref = rep->x_ref;
        if (M->gap && !gap_ok) return einval("the partial gap is defined for the low-dose APP solvers only");
        if (M->rmse && !M->x_ref) return einval("rmse needs x_ref");
        M->cost = M->cost && rep->cost != nullptr;
    } else {
        M->cost = false;
    }
    k->record = M->any() ? 1 : 0;
    return CTPD_OK;
}

int monitor_bnorm(ctpd_op* op, const float* b, Monitors* M) {
    if (!M->resid) return CTPD_OK;
    int r;
    if ((r = reduce(op, RED_SQ_F32, b, nullptr, nullptr, op->I, 0))) return r;
    if ((r = read_red(op))) return r;
    M->bnorm2 = op->red_host[0];
    return CTPD_OK;
}

// The per-iteration monitors (Eq. 1 cost or psi, partial gap, data residual,
// Eq. 34 RMSE) as float64 sums into the iteration's slots of op->cost_dev.
int record_monitors(ctpd_op* op, int it, const Monitors& M, const float* x, const float* q, const float* b,
                    const float* w, const float* mu) {
    double* slot = op->cost_dev + (size_t)3 * kMonSlots * it;
    hipStream_t s = op->stream;
    if (M.cost) {
        HIP_TRY(launch_tv_norm(x, op->n, op->partials, slot + 3 * MON_TV, s));
        HIP_TRY(launch_reduce(w ? RED_WRES_F32 : RED_SQDIFF_F32, q, b, w, op->I, op->partials, slot + 3 * MON_DATA,
                              s));
    }
    if (M.gap) HIP_TRY(launch_reduce(RED_GAP_F32, q, b, w, op->I, op->partials, slot + 3 * MON_GAP, s, mu));
    if (M.resid) HIP_TRY(launch_reduce(RED_SQDIFF_F32, q, b, nullptr, op->I, op->partials, slot + 3 * MON_RES, s));
    if (M.rmse)
        HIP_TRY(launch_reduce(RED_SQDIFF_F32, x, M.x_ref, nullptr, op->J, op->partials, slot + 3 * MON_RMSE, s));
    return CTPD_OK;
}

int ensure_cost(ctpd_op* op, int iters) {
    if (op->cost_cap >= iters) return CTPD_OK;
    if (op->cost_dev) (void)hipFree(op->cost_dev);
    op->cost_dev = nullptr;
    op->cost_cap = 0;
    ALLOC(op->cost_dev, (size_t)3 * kMonSlots * std::max(iters, 1));
    op->cost_cap = iters;
    return CTPD_OK;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

int finish(ctpd_op* op, int iters, bool lowdose, double beta, float* p_final, ctpd_report* rep, float* x_out,
           const Monitors& M) {
    const size_t J = op->J, I = op->I;
    HIP_TRY(launch_copy_f32(x_out, op->x, J, op->stream));
    if (rep && rep->mu_out) HIP_TRY(launch_copy_f32(rep->mu_out, op->mu[0], I, op->stream));
    if (rep && rep->p_out) HIP_TRY(launch_copy_f32(rep->p_out, p_final, 2 * J, op->stream));
    if (rep && M.any() && iters > 0) {
        const size_t per = (size_t)3 * kMonSlots;
        std::vector<double> h(per * iters);
        HIP_TRY(hipMemcpyAsync(h.data(), op->cost_dev, sizeof(double) * h.size(), hipMemcpyDeviceToHost,
                               op->stream));
        int r = sync(op);
        if (r) return r;
        for (int k = 0; k < iters; ++k) {
            const double* v = h.data() + per * k;
            if (M.cost) rep->cost[k] = lowdose ? beta * v[3 * MON_TV] + 0.5 * v[3 * MON_DATA] : v[3 * MON_TV];
            if (M.gap) rep->gap[k] = 0.5 * v[3 * MON_GAP];
            if (M.resid) rep->resid[k] = M.bnorm2 > 0.0 ? std::sqrt(v[3 * MON_RES] / M.bnorm2) : 0.0;
            if (M.rmse) rep->rmse[k] = std::sqrt(v[3 * MON_RMSE] / (double)J);
        }
    }
    return sync(op);
}

int ensure_hv(ctpd_op* op, int kmax) {
    if (!op->hv_item) {
        ALLOC(op->hv_item, 1);
        HIP_TRY(hipHostMalloc((void**)&op->hv_item_host, sizeof(NormItem), hipHostMallocDefault));
        ALLOC(op->hv_sum, 3);
        HIP_TRY(hipHostMalloc((void**)&op->hv_sum_host, sizeof(double) * 6, hipHostMallocDefault));
        for (auto& e : op->hv_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&op->hv_start_ev, hipEventDisableTiming));
        std::vector<RowRef> rows(op->m);
        for (int v = 0; v < op->m; ++v) rows[v] = RowRef{0, v};
        ALLOC(op->hv_rows, op->m);
        HIP_TRY(hipMemcpy(op->hv_rows, rows.data(), sizeof(RowRef) * op->m, hipMemcpyHostToDevice));
        const int gx = norm_blocks_x(op->nb), gy = norm_blocks_y(op->m);
        std::vector<BlockRef> f(gx * gy);
        for (int l = 0; l < gx * gy; ++l) f[l] = BlockRef{0, l};
        ALLOC(op->hv_filt, f.size());
        HIP_TRY(hipMemcpy(op->hv_filt, f.data(), sizeof(BlockRef) * f.size(), hipMemcpyHostToDevice));
        op->hv_nfilt = (int)f.size();
        ALLOC(op->hv_b0, op->m);
        ALLOC(op->hv_theta, op->m);
        ALLOC(op->hv_done, op->m);
        ALLOC(op->hv_maxinv, op->m);
        ALLOC(op->hv_ubound, op->m);
        int r = ensure_sym(op);
        if (r) return r;
    }
    if (op->hv_cap < kmax) {
        if (op->hv_al) (void)hipFree(op->hv_al);
        if (op->hv_b2) (void)hipFree(op->hv_b2);
        op->hv_al = op->hv_b2 = nullptr;
        op->hv_cap = 0;
        ALLOC(op->hv_al, (size_t)kmax * op->m);
        ALLOC(op->hv_b2, (size_t)kmax * op->m);
        op->hv_cap = kmax;
    }
    return CTPD_OK;
}

int lambda_h_views(const std::vector<ctpd_op*>& ops, const float* const* w, const double* kappa, int kmax,
                   hipStream_t s, NormItem* items, NormItem* items_host, const RowRef* rows, int nrows,
                   const BlockRef* filt, int nfilt, double* summary, double* summary_host, const hipEvent_t* ev,
                   double* lam, int* steps, const std::function<int(hipEvent_t)>& side, hipEvent_t side_ev) {
    const int P = (int)ops.size();
    for (int i = 0; i < P; ++i) {
        ctpd_op* op = ops[i];
        int r = ensure_hv(op, kmax);
        if (r) return r;
        NormItem& it = items_host[i];
        it = NormItem{};
        it.m = op->m;
        it.nb = op->nb;
        it.taps64 = op->taps64;
        it.rs = op->sino64[3];
        it.w = w[i];
        it.inv_kappa = 1.0 / kappa[i];
        for (int q = 0; q < 3; ++q) it.v[q] = op->sino64[q];
        it.al = op->hv_al;
        it.b2 = op->hv_b2;
        it.b0 = op->hv_b0;
        it.theta = op->hv_theta;
        it.done = op->hv_done;
        it.maxinv = op->hv_maxinv;
        it.ubound = op->hv_ubound;
        it.fsym = op->hv_sym;
        if (op->hv_sym_tau != op->tap_tau || op->hv_sym_kappa != op->tap_kappa) {
            HIP_TRY(launch_symbol_max(op->taps64, op->nb, op->hv_sym, s));
            op->hv_sym_tau = op->tap_tau;
            op->hv_sym_kappa = op->tap_kappa;
        }
        it.summary = summary + 3 * i;
    }
    HIP_TRY(hipMemcpyAsync(items, items_host, sizeof(NormItem) * P, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_rows_start(items, rows, nrows, 2, s));
    HIP_TRY(launch_rows_prune(items, rows, nrows, P, s));
    if (side && side_ev) HIP_TRY(hipEventRecord(side_ev, s));
    int max_nb = 0;
    for (ctpd_op* op : ops) max_nb = std::max(max_nb, op->nb);
    // up to 1024 bins a round is one launch (the view's product and recurrence
    // in one workgroup); beyond, a batched FP64 MFMA filter and a step kernel per step
    const bool fused = rows_round_fits(max_nb);
    // the first round takes 16 steps (by then the residual bounds stop every
    // view but those near the top), the later ones 8
    constexpr int kRound = 8, kFirstRound = 16;
    // a chain stops when its top Ritz value moved by <= 1e-7 relative over the
    // last step: then it is within ~1e-8 of the view's eigenvalue (the Ritz
    // values converge geometrically), far inside what sigma = rho 2 / lambda_h
    // needs, and the 720-view chains stop after 24 steps instead of 32
    constexpr double kRowsTol = 1e-7;
    // steps j0 .. j1-1, the Ritz values and the summary, copied to a pinned
    // slot of 3 P doubles with an event behind it
    auto enqueue = [&](int j0, int j1, int slot) -> int {
        if (fused) {
            HIP_TRY(launch_rows_round(items, rows, nrows, P, j0, j1, max_nb, kRowsTol, s));
        } else {
            for (int j = j0; j < j1; ++j) {
                const int rot = (3 - j % 3) % 3;
                HIP_TRY(launch_norm_filter_batched(items, filt, nfilt, rot, s));
                HIP_TRY(launch_rows_step(items, rows, nrows, rot, j, s));
            }
            HIP_TRY(launch_rows_ritz(items, rows, nrows, P, j1, kRowsTol, s));
        }
        HIP_TRY(hipMemcpyAsync(summary_host + (size_t)3 * P * slot, summary, sizeof(double) * 3 * P,
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipEventRecord(ev[slot], s));
        return CTPD_OK;
    };
    // Rounds are queued one ahead: round r + 1 runs while the host reads round
    // r's summary.  It sees the stops that summary made, so when no chain was
    // left running it does nothing and its summary repeats round r's.
    int j = std::min(kmax, kFirstRound), slot = 0, r;
    if ((r = enqueue(0, j, 0))) return r;
    // the side work is queued after the first round, so that the round is
    // dispatched first and keeps its compute units
    if (side && side_ev && (r = side(side_ev))) return r;
    const double* res = summary_host;
    for (;;) {
        const int jn = std::min(kmax, j + kRound);
        const bool ahead = jn > j;
        if (ahead && (r = enqueue(j, jn, 1 - slot))) return r;
        HIP_TRY(hipEventSynchronize(ev[slot]));
        res = summary_host + (size_t)3 * P * slot;
        bool running = false;
        for (int i = 0; i < P; ++i) running = running || res[3 * i + 1] > 0.0;
        if (!running || !ahead) break;
        j = jn;
        slot = 1 - slot;
    }
    for (int i = 0; i < P; ++i) {
        lam[i] = res[3 * i + 0];
        steps[i] = res[3 * i + 1] > 0.0 ? j : (int)res[3 * i + 2];
    }
    return CTPD_OK;
}

// a1 and the start of a2 for Algorithm 1: validity scan of w and b, kappa =
// mean(1/w), tau, W^-1, the taps of Eq. 24; when sigma is not given, the two
// operator-norm chains are started (run them with run_lanczos, then call
// lowdose_setup_end).
int lowdose_setup_begin(ctpd_op* op, const float* b, const float* w, const Knobs& k, LowdoseSetup* S) {
    const size_t I = op->I;
    int r;
    if ((r = reduce(op, RED_INVW_CHECK, w, b, nullptr, I, 0))) return r;
    // W^-1 and W^-1/2 need no kappa: they run while the host reads it
    HIP_TRY(launch_inverse_f32(op->winv, w, I, op->stream));
    if ((r = ensure_f64(op))) return r;
    HIP_TRY(launch_rsqrt_f64(op->sino64[3], w, I, op->stream));
    if ((r = read_red(op))) return r;
    if (op->red_host[1] > 0 || op->red_host[2] > 0) {
        snprintf(g_errmsg, sizeof g_errmsg, "%.0f weights <= 0 or non-finite, %.0f non-finite data",
                 op->red_host[1], op->red_host[2]);
        return CTPD_EDOMAIN;
    }
    S->kappa = op->red_host[0] / (double)I;
    // a given tau equal to the default (a resumed state's) takes the default's
    // taps, so that a resumed solve repeats the same filter bit for bit
    const double tau_def = kTauMultLowdose * M_PI * S->kappa / (2.0 * op->m);
    const bool given = k.tau > 0 && k.tau != tau_def;
    S->tau = given ? k.tau : tau_def;
    if ((r = given ? ensure_taps(op, S->tau, S->kappa) : ensure_taps_default(op, S->kappa))) return r;
    // The two norms are computed whether sigma is given or not: they give the
    // default sigma, and a given one is checked against the bound they set.
    // H of Eq. 24 is (1/kappa) |w| / (a + |w|) with a = 2 m tau / kappa, so
    // kappa * lambda_max(A^T D A) depends on the geometry and a only (a is the
    // constant 0.3 pi at the default tau).
    S->a = given ? 2.0 * op->m * S->tau / S->kappa : kTauMultLowdose * M_PI;
    S->run_a = !(op->norm_ld > 0.0 && op->norm_ld_a == S->a && op->norm_ld_kmax == k.norm_steps);
    if (S->run_a && (r = setup_lambda_a(op, k.norm_steps, &S->La))) return r;
    return CTPD_OK;
}

int lowdose_setup_end(ctpd_op* op, const Knobs& k, LowdoseSetup* S) {
    if (S->run_a) {
        S->lam_a = S->La.theta;
        S->steps_a = S->La.steps;
        op->norm_ld = S->lam_a * S->kappa;
        op->norm_ld_a = S->a;
        op->norm_ld_kmax = k.norm_steps;
    } else {
        S->lam_a = op->norm_ld / S->kappa;
        S->steps_a = 0;
    }
    // Eq. 16 with the conditions of Algorithm 1: sigma < 2 / lambda_h and sigma tau lambda_A < 1
    const double bound = std::min(2.0 / S->lam_h, 1.0 / (S->tau * S->lam_a));
    if (k.sigma > 0) {
        if (!(k.sigma < bound)) {
            snprintf(g_errmsg, sizeof g_errmsg,
                     "invalid argument: sigma = %.6g violates the step-size bound (Eq. 16): needs sigma < "
                     "min(2/lambda_h, 1/(tau lambda_A)) = %.6g (lambda_h = %.6g, tau = %.6g, lambda_A = %.6g)",
                     k.sigma, bound, S->lam_h, S->tau, S->lam_a);
            return CTPD_EINVAL;
        }
        S->sigma = k.sigma;
    } else {
        S->sigma = k.rho * bound;
    }
    return CTPD_OK;
}

}  // namespace ctpd_host

using namespace ctpd_host;

extern "C" {

const char* ctpd_strerror(int code) {
    switch (code) {
        case CTPD_OK: return "ok";
        case CTPD_EINVAL: return g_errmsg[0] ? g_errmsg : "invalid argument";
        case CTPD_EDOMAIN: return g_errmsg[0] ? g_errmsg : "data outside the model";
        case CTPD_EHIP: return g_errmsg[0] ? g_errmsg : "HIP runtime error";
        case CTPD_ENOMEM: return g_errmsg[0] ? g_errmsg : "out of device memory";
        default: return "unknown error code";
    }
}

int ctpd_op_create(const ctpd_geometry* g, void* stream, ctpd_op** out) {
    g_errmsg[0] = 0;
    if (!g || !out) return einval("null pointer");
    if (g->n < 1 || g->n > 8192) return einval("n out of range [1, 8192]");
    if (g->n_views < 1 || g->n_views > 1000000) return einval("n_views out of range");
    if (g->n_bins < 1 || g->n_bins > CTPD_MAX_BINS) return einval("n_bins out of range");
    if (g->angles)
        for (int v = 0; v < g->n_views; ++v)
            if (!std::isfinite(g->angles[v])) return einval("view angles must be finite");
    *out = nullptr;
    ctpd_op* op = new ctpd_op();
    op->n = g->n;
    op->m = g->n_views;
    op->nb = g->n_bins;
    op->stream = (hipStream_t)stream;
    op->J = (size_t)op->n * op->n;
    op->Jp = (size_t)op->n * (op->n + 6);
    op->I = (size_t)op->m * op->nb;
    auto init = [&]() -> int {
        HIP_TRY(hipGetDevice(&op->device));
        ALLOC(op->views, op->m);
        std::vector<ViewGeom> hv = make_views(op->n, op->m, op->nb, g->angles);
        HIP_TRY(hipMemcpy(op->views, hv.data(), sizeof(ViewGeom) * op->m, hipMemcpyHostToDevice));
        {
            // the slab projector's groups: spread over the chip's compute units for the
            // solves, at their fullest for the batched launches
            int cus = 0, dense = 0;
            HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, op->device));
            const int per = forward_slab_tasks_per_group();
            const std::vector<int> bat = forward_slab_schedule(hv.data(), op->m, op->n, op->nb, 0, &dense);
            ALLOC(op->bat_tasks, bat.size());
            HIP_TRY(hipMemcpy(op->bat_tasks, bat.data(), sizeof(int) * bat.size(), hipMemcpyHostToDevice));
            op->bat_groups = (int)(bat.size() / per);
            const bool slab = forward_slab_preferred(dense, op->n);
            const std::vector<int> one = slab ? forward_slab_schedule(hv.data(), op->m, op->n, op->nb, cus, nullptr)
                                              : forward_split_order(hv.data(), op->m, op->n, op->nb);
            ALLOC(op->fwd_tasks, one.size());
            HIP_TRY(hipMemcpy(op->fwd_tasks, one.data(), sizeof(int) * one.size(), hipMemcpyHostToDevice));
            op->fwd_groups = slab ? (int)(one.size() / per) : 0;
        }
        ALLOC(op->xp, op->Jp + kPlaneSlack);
        ALLOC(op->xTp, op->Jp + kPlaneSlack);
        // the planes' pad columns stay zero for good: only interiors are written after this
        HIP_TRY(hipMemset(op->xp, 0, sizeof(float) * (op->Jp + kPlaneSlack)));
        HIP_TRY(hipMemset(op->xTp, 0, sizeof(float) * (op->Jp + kPlaneSlack)));
        ALLOC(op->x, op->J);
        ALLOC(op->z, op->J);
        for (auto& p : op->p) ALLOC(p, 2 * op->J);
        for (auto& p : op->mu) ALLOC(p, op->I);
        ALLOC(op->mubar, op->I);
        ALLOC(op->q, op->I);
        ALLOC(op->sx, op->I);
        ALLOC(op->winv, op->I);
        ALLOC(op->taps64, 2 * op->nb - 1);
        ALLOC(op->taps32, 2 * op->nb - 1);
        ALLOC(op->partials, 3 * kReduceBlocks);
        ALLOC(op->red, 3 * kRedSlots);
        HIP_TRY(hipHostMalloc((void**)&op->red_host, sizeof(double) * 3 * kRedSlots, hipHostMallocDefault));
        HIP_TRY(hipStreamCreateWithFlags(&op->aux, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&op->fork, hipEventDisableTiming));
        return CTPD_OK;
    };
    int r = init();
    if (r != CTPD_OK) {
        ctpd_op_destroy(op);
        return r;
    }
    *out = op;
    return CTPD_OK;
}

void ctpd_op_destroy(ctpd_op* op) {
    if (!op) return;
    if (op->stream || op->views) (void)hipStreamSynchronize(op->stream);
    if (op->aux) (void)hipStreamSynchronize(op->aux);   // a lambda_h round queued ahead may still run there
    void* ptrs[] = {op->views, op->fwd_tasks, op->bat_tasks, op->xp, op->xTp, op->x, op->z, op->p[0], op->p[1],
                    op->mu[0], op->mu[1], op->mu[2], op->mubar, op->q, op->sx, op->winv, op->taps64, op->taps32, op->partials, op->red, op->cost_dev,
                    op->img64[0], op->img64[1], op->img64[2], op->pad64[0], op->pad64[1], op->sino64[0], op->sino64[1],
                    op->sino64[2], op->sino64[3], op->sino64[4], op->sino64[5], op->lz[0], op->lz[1],
                    op->lz_partials[0], op->lz_partials[1], op->xbar, op->ball_y, op->split64, op->ball_dev};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (op->red_host) (void)hipHostFree(op->red_host);
    for (double* h : op->lz_host)
        if (h) (void)hipHostFree(h);
    if (op->aux) {
        (void)hipStreamSynchronize(op->aux);
        (void)hipStreamDestroy(op->aux);
    }
    if (op->fork) (void)hipEventDestroy(op->fork);
    free_unrolled(op->uw);
    void* hv[] = {op->hv_al,   op->hv_b2,   op->hv_b0,  op->hv_theta,  op->hv_done, op->hv_item, op->hv_rows,
                  op->hv_filt, op->hv_sum, op->hv_maxinv, op->hv_ubound, op->hv_sym, op->taps1,  op->sym1};
    for (void* p : hv)
        if (p) (void)hipFree(p);
    if (op->hv_item_host) (void)hipHostFree(op->hv_item_host);
    if (op->hv_sum_host) (void)hipHostFree(op->hv_sum_host);
    for (auto e : op->hv_ev)
        if (e) (void)hipEventDestroy(e);
    if (op->hv_start_ev) (void)hipEventDestroy(op->hv_start_ev);
    delete op;
}

int ctpd_project(ctpd_op* op, const float* x, float* y) {
    g_errmsg[0] = 0;
    if (!op || !x || !y) return einval("null pointer");
    return project(op, x, y);
}

int ctpd_backproject(ctpd_op* op, const float* y, float* x) {
    g_errmsg[0] = 0;
    if (!op || !x || !y) return einval("null pointer");
    HIP_TRY(launch_adjoint<float>(y, nullptr, 1.0f, 0.0f, nullptr, 0.0f, 1.0f, x, op->views, op->n, op->m, op->nb,
                                  op->stream));
    return CTPD_OK;
}

int ctpd_ramp_filter(ctpd_op* op, double tau, double kappa, const float* s, float* out) {
    g_errmsg[0] = 0;
    if (!op || !s || !out) return einval("null pointer");
    if (!(tau > 0.0) || !std::isfinite(tau)) return einval("tau must be finite and > 0");
    if (!(kappa >= 0.0) || !std::isfinite(kappa)) return einval("kappa must be finite and >= 0");
    int r = ensure_taps(op, tau, kappa);
    if (r) return r;
    return filter(op, FILT_PLAIN, s, nullptr, nullptr, nullptr, nullptr, 0.f, nullptr, 0.f, 1.0f, out);
}

int ctpd_ramp_filter_f64(ctpd_op* op, double tau, double kappa, const double* s, double* out) {
    g_errmsg[0] = 0;
    if (!op || !s || !out) return einval("null pointer");
    if (!(tau > 0.0) || !std::isfinite(tau)) return einval("tau must be finite and > 0");
    if (!(kappa >= 0.0) || !std::isfinite(kappa)) return einval("kappa must be finite and >= 0");
    int r = ensure_taps(op, tau, kappa);
    if (r) return r;
    HIP_TRY(launch_filter_f64(s, out, op->taps64, nullptr, nullptr, op->m, op->nb, op->stream));
    return CTPD_OK;
}

int ctpd_filter_taps(ctpd_op* op, double tau, double kappa, double* taps_host) {
    g_errmsg[0] = 0;
    if (!op || !taps_host) return einval("null pointer");
    if (!(tau > 0.0) || !std::isfinite(tau)) return einval("tau must be finite and > 0");
    if (!(kappa >= 0.0) || !std::isfinite(kappa)) return einval("kappa must be finite and >= 0");
    int r = ensure_taps(op, tau, kappa);
    if (r) return r;
    HIP_TRY(hipMemcpyAsync(taps_host, op->taps64, sizeof(double) * (2 * op->nb - 1), hipMemcpyDeviceToHost,
                           op->stream));
    return sync(op);
}

int ctpd_tv_prox(ctpd_op* op, const float* z, double lambda, int32_t n_iter, double tv_step, float* p_inout,
                 float* x) {
    g_errmsg[0] = 0;
    if (!op || !z || !p_inout || !x) return einval("null pointer");
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return einval("lambda must be finite and >= 0");
    if (n_iter < 0) return einval("n_iter < 0");
    if (!(tv_step > 0.0) || !std::isfinite(tv_step)) return einval("tv_step must be finite and > 0");
    float* pf = nullptr;
    const float lam = (float)lambda;
    int r = tv_prox(op, z, lam, n_iter, (float)(tv_step / lambda), p_inout, op->p[0], x, &pf);
    if (r) return r;
    if (pf != p_inout) HIP_TRY(launch_copy_f32(p_inout, pf, 2 * op->J, op->stream));
    return CTPD_OK;
}

int ctpd_pd_lowdose_solve(ctpd_op* op, const float* b, const float* w, double beta, int32_t iters,
                          const ctpd_params* p, float* x_out, ctpd_report* rep) {
    g_errmsg[0] = 0;
    if (!op || !b || !w || !x_out) return einval("null pointer");
    if (!(beta >= 0.0) || !std::isfinite(beta)) return einval("beta must be finite and >= 0");
    if (iters < 0) return einval("iters < 0");
    Knobs k;
    int r = read_params(p, &k);
    if (r) return r;
    Monitors M;
    if ((r = read_monitors(rep, true, &k, &M))) return r;
    const auto t0 = std::chrono::steady_clock::now();
    LowdoseSetup S;
    // the iterates' start (zero or the state) needs nothing of the set-up: it runs first
    if ((r = k.resumed() ? load_state(op, k.state, nullptr) : lowdose_zero(op))) return r;
    if ((r = lowdose_setup_begin(op, b, w, k, &S))) return r;
    if ((r = monitor_bnorm(op, b, &M))) return r;
    {
        // the lambda_A chain (first solve on the handle) runs on op->stream while the
        // per-view lambda_h chains run on op->aux
        if ((r = ensure_hv(op, k.norm_steps))) return r;
        HIP_TRY(hipEventRecord(op->fork, op->stream));
        HIP_TRY(hipStreamWaitEvent(op->aux, op->fork, 0));
        if (S.run_a) {
            for (int q = 0; q < 4 && !S.La.finished(); ++q)   // queue the first rounds before the h chains block
                if ((r = S.La.enqueue(S.La.per_round))) return r;
        }
        // From the zero start the first iteration's z is -sigma (x - tau A^T D b)
        // with x = 0 (the order of operations every solver of Algorithm 1 uses
        // for it), and the bracket needs no sigma: it runs on op->stream beside
        // the lambda_h chains on op->aux, made ready together with their first
        // round so that the round's few workgroups find their compute units.
        auto zstart = [&](hipEvent_t ev) -> int {
            HIP_TRY(hipStreamWaitEvent(op->stream, ev, 0));
            const int rf = filter(op, FILT_PLAIN, b, nullptr, nullptr, nullptr, nullptr, 0.f, nullptr, 0.f, 1.f,
                                  op->mubar);
            if (rf) return rf;
            HIP_TRY(launch_adjoint<float>(op->mubar, nullptr, 1.f, 0.f, op->x, 1.f, -(float)S.tau, op->z, op->views,
                                          op->n, op->m, op->nb, op->stream));
            return CTPD_OK;
        };
        const float* wp[1] = {w};
        if ((r = lambda_h_views({op}, wp, &S.kappa, k.norm_steps, op->aux, op->hv_item, op->hv_item_host,
                                op->hv_rows, op->m, op->hv_filt, op->hv_nfilt, op->hv_sum, op->hv_sum_host,
                                op->hv_ev, &S.lam_h, &S.steps_h,
                                k.resumed() ? std::function<int(hipEvent_t)>() : zstart, op->hv_start_ev)))
            return r;
        if (S.run_a) {
            HIP_TRY(hipStreamSynchronize(op->stream));
            S.La.absorb();
            if ((r = run_lanczos({&S.La}))) return r;
        }
    }
    if ((r = lowdose_setup_end(op, k, &S))) return r;
    const double kappa = S.kappa, tau = S.tau, sigma = S.sigma, lam_a = S.lam_a, lam_h = S.lam_h;
    const int steps_a = S.steps_a, steps_h = S.steps_h;
    if ((r = sync(op))) return r;
    const double setup_ms = ms_since(t0);
    const auto t1 = std::chrono::steady_clock::now();
    float* pcur = nullptr;
    if ((r = lowdose_loop(op, b, w, beta, iters, k, tau, sigma, &pcur, M, true, !k.resumed()))) return r;
    if (k.state && (r = save_state(op, k.state, pcur, nullptr, iters, tau, sigma))) return r;
    if ((r = finish(op, iters, true, beta, pcur, rep, x_out, M))) return r;
    if (rep) {
        rep->tau = tau;
        rep->sigma = sigma;
        rep->kappa = kappa;
        rep->lambda_a = lam_a;
        rep->lambda_h = lam_h;
        rep->norm_steps_a = steps_a;
        rep->norm_steps_h = steps_h;
        rep->iters_done = iters;
        rep->setup_ms = setup_ms;
        rep->loop_ms = ms_since(t1);
    }
    return CTPD_OK;
}

int ctpd_app_identity_lowdose_solve(ctpd_op* op, const float* b, const float* w, double beta, int32_t iters,
                                    const ctpd_params* p, float* x_out, ctpd_report* rep) {
    g_errmsg[0] = 0;
    if (!op || !b || !w || !x_out) return einval("null pointer");
    if (!(beta >= 0.0) || !std::isfinite(beta)) return einval("beta must be finite and >= 0");
    if (iters < 0) return einval("iters < 0");
    Knobs k;
    int r = read_params(p, &k);
    if (r) return r;
    if ((r = no_state(k))) return r;
    Monitors M;
    if ((r = read_monitors(rep, true, &k, &M))) return r;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = op->stream;
    // validity scan and kappa (reported), W^-1, lambda_h = max 1/w, D = I
    if ((r = reduce(op, RED_INVW_CHECK, w, b, nullptr, op->I, 0))) return r;
    HIP_TRY(launch_max_inv(w, op->I, op->partials, op->red + 3, s));
    if ((r = read_red(op))) return r;
    if (op->red_host[1] > 0 || op->red_host[2] > 0) {
        snprintf(g_errmsg, sizeof g_errmsg, "%.0f weights <= 0 or non-finite, %.0f non-finite data",
                 op->red_host[1], op->red_host[2]);
        return CTPD_EDOMAIN;
    }
    const double kappa = op->red_host[0] / (double)op->I, lam_h = op->red_host[3];
    HIP_TRY(launch_inverse_f32(op->winv, w, op->I, s));
    HIP_TRY(launch_identity_taps(op->taps64, op->taps32, op->nb, s));
    op->tap_tau = op->tap_kappa = -2.0;   // not the taps of any (tau, kappa)
    double tau = k.tau, sigma = k.sigma, lam_a = 0.0;
    int steps_a = 0;
    if (op->norm_ata > 0.0 && op->norm_ata_kmax == k.norm_steps) {   // a property of the geometry
        lam_a = op->norm_ata;
    } else {
        Lanczos L;
        if ((r = setup_lambda_a(op, k.norm_steps, &L, false, nullptr))) return r;
        if ((r = run_lanczos({&L}))) return r;
        lam_a = L.theta;
        steps_a = L.steps;
        op->norm_ata = lam_a;
        op->norm_ata_kmax = k.norm_steps;
    }
    // default tau balances the two bounds of sigma: 1 / (tau lambda_A) = 2 / lambda_h
    if (!(tau > 0)) tau = lam_h / (2.0 * lam_a);
    const double bound = std::min(2.0 / lam_h, 1.0 / (tau * lam_a));
    if (sigma > 0) {
        if (!(sigma < bound)) {
            snprintf(g_errmsg, sizeof g_errmsg,
                     "invalid argument: sigma = %.6g violates the step-size bound (Eq. 16 with D = I): needs sigma < "
                     "min(2/lambda_h, 1/(tau lambda_A)) = %.6g",
                     sigma, bound);
            return CTPD_EINVAL;
        }
    } else {
        sigma = k.rho * bound;
    }
    if ((r = monitor_bnorm(op, b, &M))) return r;
    if ((r = sync(op))) return r;
    const double setup_ms = ms_since(t0);
    const auto t1 = std::chrono::steady_clock::now();
    float* pcur = nullptr;
    if ((r = lowdose_loop(op, b, w, beta, iters, k, tau, sigma, &pcur, M))) return r;
    if ((r = finish(op, iters, true, beta, pcur, rep, x_out, M))) return r;
    if (rep) {
        rep->tau = tau;
        rep->sigma = sigma;
        rep->kappa = kappa;
        rep->lambda_a = lam_a;
        rep->lambda_h = lam_h;
        rep->norm_steps_a = steps_a;
        rep->norm_steps_h = 0;
        rep->iters_done = iters;
        rep->setup_ms = setup_ms;
        rep->loop_ms = ms_since(t1);
    }
    return CTPD_OK;
}

// The few-view default tau = mean |sigma A^T D(1) b| (a step size: formed in
// float64 like the norms).  In Algorithm 2 tau only weighs the TV term against
// the constraint (sigma D(tau) = sigma D(1) / tau).
static int fewview_default_tau(ctpd_op* op, const float* b, double sigma, double* tau) {
    int r;
    hipStream_t s = op->stream;
    if ((r = ensure_taps(op, 1.0, 0.0))) return r;
    if ((r = ensure_f64(op))) return r;
    HIP_TRY(launch_widen_f64(op->sino64[0], b, op->I, s));
    HIP_TRY(launch_filter_f64(op->sino64[0], op->sino64[1], op->taps64, nullptr, nullptr, op->m, op->nb, s));
    HIP_TRY(launch_adjoint<double>(op->sino64[1], nullptr, 1.0, 0.0, nullptr, 0.0, 1.0, op->img64[0], op->views,
                                   op->n, op->m, op->nb, s));
    if ((r = reduce(op, RED_ABS_F64, op->img64[0], nullptr, nullptr, op->J, 0))) return r;
    if ((r = read_red(op))) return r;
    *tau = sigma * op->red_host[0] / (double)op->J;
    if (!(*tau > 0)) *tau = 1.0;   // all-zero data: any tau works
    return CTPD_OK;
}

// The few-view iteration from x = 0, mu = 0 (Eqs. 29-31), shared by
// Algorithm 2 (y null: the data side is b itself) and the error-tolerant
// solve (y: the data-side variable, starting at b, projected onto the ball
// {||y - b|| <= eps} after each primal step).  Leaves the iterate in op->x and
// mu^K in op->mu[0]; *p_final gets the last TV dual field.
static int fewview_loop(ctpd_op* op, const float* b, float* y, double eps, int iters, double tau, double sigma,
                        const Knobs& k, const Monitors& M, float** p_final) {
    int r;
    hipStream_t s = op->stream;
    const size_t I = op->I, J = op->J;
    if (k.record && (r = ensure_cost(op, iters))) return r;
    const bool resumed = k.resumed();
    if (resumed) {
        if ((r = load_state(op, k.state, y))) return r;
    } else {
        HIP_TRY(launch_fill_f32(op->x, 0.f, J, s));
        HIP_TRY(launch_fill_f32(op->p[0], 0.f, 2 * J, s));
        HIP_TRY(launch_fill_f32(op->mu[0], 0.f, I, s));
        HIP_TRY(launch_fill_f32(op->mu[1], 0.f, I, s));
        if (y) HIP_TRY(launch_copy_f32(y, b, I, s));
    }
    const float* data = y ? y : b;   // the sinogram A x is driven to
    float *mu = op->mu[0], *mup = op->mu[1], *mun = op->mu[2];
    float* pcur = op->p[0];
    const float fs = (float)sigma, ft = (float)tau, lam = (float)tau;
    const float tvstep = (float)(k.tv_step / tau);
    for (int it = 0; it < iters; ++it) {
        // z = x - tau A^T mubar, mubar = -sigma D b (k = 0) or 2 mu - mu_prev
        const bool first = it == 0 && !resumed;
        if (first) {
            if ((r = filter(op, FILT_PLAIN, b, nullptr, nullptr, nullptr, nullptr, 0.f, nullptr, 0.f, -fs,
                            op->mubar)))
                return r;
            HIP_TRY(launch_adjoint<float>(op->mubar, nullptr, 1.f, 0.f, op->x, 1.f, -ft, op->z, op->views, op->n,
                                          op->m, op->nb, s));
        } else {
            HIP_TRY(launch_adjoint<float>(mu, mup, 2.f, -1.f, op->x, 1.f, -ft, op->z, op->views, op->n, op->m,
                                          op->nb, s));
        }
        float* pnew = nullptr;
        // the prox also writes the projector's planes of x
        const bool padded = lam > 0.f;
        if ((r = tv_prox(op, op->z, lam, k.tv_iters, tvstep, pcur, pcur == op->p[0] ? op->p[1] : op->p[0], op->x,
                         &pnew, true)))
            return r;
        pcur = pnew;
        // y^{k+1} = P_ball(y^k + tau mubar)
        if (y) {
            if (first)
                HIP_TRY(launch_ball_project(y, op->mubar, 1.f, nullptr, 0.f, ft, b, eps, I, op->partials,
                                            op->ball_dev, s));
            else
                HIP_TRY(launch_ball_project(y, mu, 2.f, mup, -1.f, ft, b, eps, I, op->partials, op->ball_dev, s));
        }
        // mu^{k+1} = mu^k + sigma D (A x^{k+1} - data); without the monitors
        // the projector writes the residual itself
        if (!k.record) {
            if ((r = project_resid(op, op->x, data, nullptr, nullptr, op->q, padded))) return r;
            if ((r = filter(op, FILT_PLAIN, op->q, nullptr, nullptr, nullptr, mu, 1.f, nullptr, 0.f, fs, mun)))
                return r;
        } else {
            if ((r = project_resid(op, op->x, nullptr, nullptr, nullptr, op->q, padded))) return r;
            if ((r = filter(op, FILT_DUAL_FV, op->q, data, nullptr, nullptr, mu, 1.f, nullptr, 0.f, fs, mun)))
                return r;
            if ((r = record_monitors(op, it, M, op->x, op->q, b, nullptr, nullptr))) return r;
        }
        float* t = mup;
        mup = mu;
        mu = mun;
        mun = t;
    }
    op->mu[0] = mu;
    op->mu[1] = mup;
    op->mu[2] = mun;
    *p_final = pcur;
    if (k.state && (r = save_state(op, k.state, pcur, y, iters, tau, sigma))) return r;
    return CTPD_OK;
}

int ctpd_pd_fewview_solve(ctpd_op* op, const float* b, int32_t iters, const ctpd_params* p, float* x_out,
                          ctpd_report* rep) {
    g_errmsg[0] = 0;
    if (!op || !b || !x_out) return einval("null pointer");
    if (iters < 0) return einval("iters < 0");
    Knobs k;
    int r = read_params(p, &k);
    if (r) return r;
    Monitors M;
    if ((r = read_monitors(rep, false, &k, &M))) return r;
    const auto t0 = std::chrono::steady_clock::now();
    const size_t I = op->I;
    if ((r = reduce(op, RED_SQ_F32, b, nullptr, nullptr, I, 0))) return r;
    if ((r = read_red(op))) return r;
    if (op->red_host[1] > 0) {
        snprintf(g_errmsg, sizeof g_errmsg, "%.0f non-finite data values", op->red_host[1]);
        return CTPD_EDOMAIN;
    }
    M.bnorm2 = op->red_host[0];
    // a2: sigma tau < 1/lambda_max(A^T D(tau) A) with D(tau) = D(1)/tau, so
    // the bound is sigma lambda_max(A^T D(1) A) < 1 whatever tau is; the
    // default sigma is rho / lambda_max(A^T D(1) A).  The norm is a property
    // of the geometry, computed by the first solve on the handle.
    double sigma = k.sigma, lam1 = 0.0;
    int steps_a = 0;
    if (op->norm_fv > 0.0 && op->norm_fv_kmax == k.norm_steps) {
        lam1 = op->norm_fv;
    } else {
        if ((r = ensure_taps(op, 1.0, 0.0))) return r;
        Lanczos La;
        if ((r = setup_lambda_a(op, k.norm_steps, &La))) return r;
        if ((r = run_lanczos({&La}))) return r;
        lam1 = La.theta;
        steps_a = La.steps;
        op->norm_fv = lam1;
        op->norm_fv_kmax = k.norm_steps;
    }
    if (sigma > 0) {
        if (!(sigma * lam1 < 1.0)) {
            snprintf(g_errmsg, sizeof g_errmsg,
                     "invalid argument: sigma = %.6g violates the step-size bound of Algorithm 2: needs sigma < "
                     "1/lambda_max(A^T D(1) A) = %.6g",
                     sigma, 1.0 / lam1);
            return CTPD_EINVAL;
        }
    } else {
        sigma = k.rho / lam1;
    }
    double tau = k.tau;
    if (!(tau > 0) && (r = fewview_default_tau(op, b, sigma, &tau))) return r;
    if ((r = ensure_taps(op, tau, 0.0))) return r;
    if ((r = sync(op))) return r;
    const double setup_ms = ms_since(t0);
    const auto t1 = std::chrono::steady_clock::now();
    float* pcur = nullptr;
    if ((r = fewview_loop(op, b, nullptr, 0.0, iters, tau, sigma, k, M, &pcur))) return r;
    if ((r = finish(op, iters, false, 1.0, pcur, rep, x_out, M))) return r;
    if (rep) {
        rep->tau = tau;
        rep->sigma = sigma;
        rep->kappa = 0.0;
        rep->lambda_a = lam1 > 0 ? lam1 / tau : 0.0;
        rep->lambda_h = 0.0;
        rep->norm_steps_a = steps_a;
        rep->norm_steps_h = 0;
        rep->iters_done = iters;
        rep->setup_ms = setup_ms;
        rep->loop_ms = ms_since(t1);
    }
    return CTPD_OK;
}


// ---------------------------------------------------------------------------
// The error-tolerant few-view problem the conclusions (Sec. 5) name:
//     min psi(x)  s.t.  ||A x - b|| <= eps,  x >= 0,
// posed like Eqs. 6-7: a data-side variable y with the preconditioned
// constraint D^1/2 (A x - y) = 0 and the indicator of the ball
// B(b, eps) = {y : ||y - b|| <= eps} as its data term.  APP on the pair (x, y)
// (Eqs. 29-31 with the primal prox split into the TV prox of Eq. 17 and the
// projection onto the ball):
//     mubar = -sigma D b (k = 0, y^0 = b), 2 mu^k - mu^{k-1} (k >= 1)
//     x^{k+1} = prox(x^k - tau A^T mubar),   y^{k+1} = P_B(y^k + tau mubar)
//     mu^{k+1} = mu^k + sigma D (A x^{k+1} - y^{k+1})
// with sigma tau lambda_max(K^T D(tau) K) < 1, K = [A, -I], i.e.
// sigma lambda_max(K^T D(1) K) < 1.  eps = 0 keeps y = b bit for bit and is
// Algorithm 2.

// lambda_max(K^T D(1) K) over the float64 pair (x, y), K (x, y) = A x - y:
// (x, y) -> (A^T s, -s) with s = D(1) (A x - y); needs the taps at tau = 1.
static int setup_lambda_split(ctpd_op* op, int kmax, Lanczos* L) {
    int r = ensure_f64(op);
    if (r) return r;
    if ((r = ensure_lz(op, kmax))) return r;
    const size_t J = op->J, I = op->I, len = J + I;
    if (!op->split64) ALLOC(op->split64, 3 * len);
    double *s1 = op->sino64[4], *s2 = op->sino64[5];
    hipStream_t s = op->stream;
    L->op = op;
    L->chain = 0;
    L->per_round = 4;
    L->s = s;
    L->q = op->split64;
    L->qp = op->split64 + len;
    L->w = op->split64 + 2 * len;
    L->kmax = kmax;
    L->apply = [op, s1, s2, s, J, I](const double* in, double* out) -> int {
        HIP_TRY(launch_pad_planes<double>(in, op->pad64[0], op->pad64[1], op->n, s));
        HIP_TRY(launch_forward<double>(op->pad64[0], op->pad64[1], s1, op->views, op->n, op->m, op->nb, s));
        HIP_TRY(launch_axpby_f64(s1, in + J, -1.0, 1.0, nullptr, 0.0, I, s));   // A x - y
        HIP_TRY(launch_filter_f64(s1, s2, op->taps64, nullptr, nullptr, op->m, op->nb, s));
        HIP_TRY(launch_adjoint<double>(s2, nullptr, 1.0, 0.0, nullptr, 0.0, 1.0, out, op->views, op->n, op->m,
                                       op->nb, s));
        HIP_TRY(launch_scale_f64(out + J, s2, -1.0, I, s));
        return CTPD_OK;
    };
    return L->start(1, (int)len, 3, nullptr, 0.0);
}

int ctpd_pd_fewview_eps_solve(ctpd_op* op, const float* b, double eps, int32_t iters, const ctpd_params* p,
                              float* x_out, ctpd_report* rep) {
    g_errmsg[0] = 0;
    if (!op || !b || !x_out) return einval("null pointer");
    if (iters < 0) return einval("iters < 0");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return einval("eps must be finite and >= 0");
    Knobs k;
    int r = read_params(p, &k);
    if (r) return r;
    if (k.state && !k.state->y) return einval("the error-tolerant solve's state needs y");
    Monitors M;
    if ((r = read_monitors(rep, false, &k, &M))) return r;
    const auto t0 = std::chrono::steady_clock::now();
    const size_t I = op->I;
    if ((r = reduce(op, RED_SQ_F32, b, nullptr, nullptr, I, 0))) return r;
    if ((r = read_red(op))) return r;
    if (op->red_host[1] > 0) {
        snprintf(g_errmsg, sizeof g_errmsg, "%.0f non-finite data values", op->red_host[1]);
        return CTPD_EDOMAIN;
    }
    M.bnorm2 = op->red_host[0];
    // sigma < 1 / lambda_max(K^T D(1) K) (a property of the geometry, computed
    // by the first solve on the handle); default rho / lambda_max
    double sigma = k.sigma, lam1 = 0.0;
    int steps_a = 0;
    if (op->norm_split > 0.0 && op->norm_split_kmax == k.norm_steps) {
        lam1 = op->norm_split;
    } else {
        if ((r = ensure_taps(op, 1.0, 0.0))) return r;
        Lanczos La;
        if ((r = setup_lambda_split(op, k.norm_steps, &La))) return r;
        if ((r = run_lanczos({&La}))) return r;
        lam1 = La.theta;
        steps_a = La.steps;
        op->norm_split = lam1;
        op->norm_split_kmax = k.norm_steps;
    }
    if (sigma > 0) {
        if (!(sigma * lam1 < 1.0)) {
            snprintf(g_errmsg, sizeof g_errmsg,
                     "invalid argument: sigma = %.6g violates the step-size bound of the error-tolerant few-view "
                     "iteration: needs sigma < 1/lambda_max(K^T D(1) K) = %.6g (K = [A, -I])",
                     sigma, 1.0 / lam1);
            return CTPD_EINVAL;
        }
    } else {
        sigma = k.rho / lam1;
    }
    double tau = k.tau;
    if (!(tau > 0) && (r = fewview_default_tau(op, b, sigma, &tau))) return r;
    if ((r = ensure_taps(op, tau, 0.0))) return r;
    if (!op->ball_y) ALLOC(op->ball_y, I);
    if (!op->ball_dev) ALLOC(op->ball_dev, 2);
    if ((r = sync(op))) return r;
    const double setup_ms = ms_since(t0);
    const auto t1 = std::chrono::steady_clock::now();
    float* pcur = nullptr;
    if ((r = fewview_loop(op, b, op->ball_y, eps, iters, tau, sigma, k, M, &pcur))) return r;
    if ((r = finish(op, iters, false, 1.0, pcur, rep, x_out, M))) return r;
    if (rep) {
        rep->tau = tau;
        rep->sigma = sigma;
        rep->kappa = 0.0;
        rep->lambda_a = lam1 / tau;
        rep->lambda_h = 0.0;
        rep->norm_steps_a = steps_a;
        rep->norm_steps_h = 0;
        rep->iters_done = iters;
        rep->setup_ms = setup_ms;
        rep->loop_ms = ms_since(t1);
    }
    return CTPD_OK;
}

// ---------------------------------------------------------------------------
// Comparators (unpreconditioned first-order primal-dual methods of Sec. 4).

int ctpd_gist_lowdose_solve(ctpd_op* op, const float* b, const float* w, double beta, int32_t iters,
                            const ctpd_params* p, float* x_out, ctpd_report* rep) {
    g_errmsg[0] = 0;
    if (!op || !b || !w || !x_out) return einval("null pointer");
    if (!(beta >= 0.0) || !std::isfinite(beta)) return einval("beta must be finite and >= 0");
    if (iters < 0) return einval("iters < 0");
    Knobs k;
    int r = read_params(p, &k);
    if (r) return r;
    if ((r = no_state(k))) return r;
    if (k.sigma > 0.125) return einval("GIST dual step must be <= 1/8 (||grad||^2 <= 8)");
    Monitors M;
    if ((r = read_monitors(rep, false, &k, &M))) return r;
    const auto t0 = std::chrono::steady_clock::now();
    const size_t I = op->I, J = op->J;
    hipStream_t s = op->stream;
    if ((r = reduce(op, RED_INVW_CHECK, w, b, nullptr, I, 0))) return r;
    if ((r = read_red(op))) return r;
    if (op->red_host[1] > 0 || op->red_host[2] > 0) {
        snprintf(g_errmsg, sizeof g_errmsg, "%.0f weights <= 0 or non-finite, %.0f non-finite data",
                 op->red_host[1], op->red_host[2]);
        return CTPD_EDOMAIN;
    }
    const double kappa = op->red_host[0] / (double)I;
    // the Lipschitz constant of the data term's gradient, lambda_max(A^T W A)
    // (data-dependent): the default gamma, and the bound gamma < 2 / L a given one must meet
    double gamma = k.tau, lip = 0.0;
    int steps_a = 0;
    {
        Lanczos L;
        if ((r = setup_lambda_a(op, k.norm_steps, &L, false, w))) return r;
        if ((r = run_lanczos({&L}))) return r;
        lip = L.theta;
        steps_a = L.steps;
    }
    if (gamma > 0) {
        if (!(gamma * lip < 2.0)) {
            snprintf(g_errmsg, sizeof g_errmsg,
                     "invalid argument: GIST step gamma = %.6g needs gamma < 2/lambda_max(A^T W A) = %.6g", gamma,
                     2.0 / lip);
            return CTPD_EINVAL;
        }
    } else {
        gamma = k.rho * 2.0 / lip;
    }
    const double lam = k.sigma > 0 ? k.sigma : 0.125;
    const double radius = gamma * beta / lam;
    if ((r = monitor_bnorm(op, b, &M))) return r;
    if ((r = sync(op))) return r;
    const double setup_ms = ms_since(t0);
    const auto t1 = std::chrono::steady_clock::now();
    if (k.record && (r = ensure_cost(op, iters))) return r;
    HIP_TRY(launch_fill_f32(op->x, 0.f, J, s));
    HIP_TRY(launch_fill_f32(op->p[0], 0.f, 2 * J, s));
    float* pcur = op->p[0];
    // the dual field is kept scaled to the unit ball: v = radius * p
    const float tl = (float)(-lam * radius), ts = radius > 0 ? (float)(-1.0 / radius) : 0.f;
    for (int it = 0; it < iters; ++it) {
        // u = x - gamma A^T W (A x - b)
        if ((r = project(op, op->x, op->q))) return r;
        HIP_TRY(launch_lin3_f32(op->mubar, op->q, 1.f, b, -1.f, nullptr, 0.f, w, I, s));
        HIP_TRY(launch_adjoint<float>(op->mubar, nullptr, 1.f, 0.f, op->x, 1.f, (float)-gamma, op->z, op->views,
                                      op->n, op->m, op->nb, s));
        // y = P+(u + lam div v); v <- ball(v + grad y); x = P+(u + lam div v)
        if (radius > 0) {
            float* pf = nullptr;
            HIP_TRY(launch_tv_prox(op->z, pcur, pcur == op->p[0] ? op->p[1] : op->p[0], op->x, op->n, tl, ts, 1,
                                   &pf, s));
            pcur = pf;
        } else {
            HIP_TRY(launch_tv_finalize(op->z, pcur, op->x, op->n, 0.f, s));
        }
        if (k.record) {
            if ((r = project(op, op->x, op->q))) return r;
            if ((r = record_monitors(op, it, M, op->x, op->q, b, w, nullptr))) return r;
        }
    }
    if (rep && rep->p_out && radius > 0)   // report v itself
        HIP_TRY(launch_lin3_f32(pcur, pcur, (float)radius, nullptr, 0.f, nullptr, 0.f, nullptr, 2 * J, s));
    if ((r = finish(op, iters, true, beta, pcur, rep, x_out, M))) return r;
    if (rep) {
        rep->tau = gamma;
        rep->sigma = lam;
        rep->kappa = kappa;
        rep->lambda_a = lip;
        rep->lambda_h = 0.0;
        rep->norm_steps_a = steps_a;
        rep->norm_steps_h = 0;
        rep->iters_done = iters;
        rep->setup_ms = setup_ms;
        rep->loop_ms = ms_since(t1);
    }
    return CTPD_OK;
}

int ctpd_cp_fewview_solve(ctpd_op* op, const float* b, int32_t iters, const ctpd_params* p, float* x_out,
                          ctpd_report* rep) {
    g_errmsg[0] = 0;
    if (!op || !b || !x_out) return einval("null pointer");
    if (iters < 0) return einval("iters < 0");
    Knobs k;
    int r = read_params(p, &k);
    if (r) return r;
    if ((r = no_state(k))) return r;
    Monitors M;
    if ((r = read_monitors(rep, false, &k, &M))) return r;
    const auto t0 = std::chrono::steady_clock::now();
    const size_t I = op->I, J = op->J;
    hipStream_t s = op->stream;
    if ((r = reduce(op, RED_SQ_F32, b, nullptr, nullptr, I, 0))) return r;
    if ((r = read_red(op))) return r;
    if (op->red_host[1] > 0) {
        snprintf(g_errmsg, sizeof g_errmsg, "%.0f non-finite data values", op->red_host[1]);
        return CTPD_EDOMAIN;
    }
    M.bnorm2 = op->red_host[0];
    if (!op->xbar) ALLOC(op->xbar, J);
    // ||K||^2 <= lambda_max(A^T A) + ||grad||^2 <= lambda_max(A^T A) + 8: the defaults
    // s = t = rho / sqrt of that, and the condition s t (lambda_max(A^T A) + 8) < 1 given steps must meet
    double t = k.tau, sg = k.sigma, lata = 0.0;
    int steps_a = 0;
    if (op->norm_ata > 0.0 && op->norm_ata_kmax == k.norm_steps) {   // a property of the geometry
        lata = op->norm_ata;
    } else {
        Lanczos L;
        if ((r = setup_lambda_a(op, k.norm_steps, &L, false, nullptr))) return r;
        if ((r = run_lanczos({&L}))) return r;
        lata = L.theta;
        steps_a = L.steps;
        op->norm_ata = lata;
        op->norm_ata_kmax = k.norm_steps;
    }
    {
        const double st = k.rho / std::sqrt(lata + 8.0);
        if (!(t > 0)) t = st;
        if (!(sg > 0)) sg = st;
        if (!(sg * t * (lata + 8.0) < 1.0)) {
            snprintf(g_errmsg, sizeof g_errmsg,
                     "invalid argument: Chambolle-Pock steps s = %.6g, t = %.6g need s t (lambda_max(A^T A) + 8) < 1 "
                     "(lambda_max(A^T A) = %.6g)",
                     sg, t, lata);
            return CTPD_EINVAL;
        }
    }
    if ((r = sync(op))) return r;
    const double setup_ms = ms_since(t0);
    const auto t1 = std::chrono::steady_clock::now();
    if (k.record && (r = ensure_cost(op, iters))) return r;
    float *x = op->x, *xn = op->z, *y1 = op->mu[0];
    HIP_TRY(launch_fill_f32(x, 0.f, J, s));
    HIP_TRY(launch_fill_f32(op->xbar, 0.f, J, s));
    HIP_TRY(launch_fill_f32(op->p[0], 0.f, 2 * J, s));
    HIP_TRY(launch_fill_f32(y1, 0.f, I, s));
    const float fs = (float)sg, ft = (float)t;
    for (int it = 0; it < iters; ++it) {
        // y1 <- y1 + s (A xbar - b);  y2 <- ball(y2 + s grad xbar)
        if ((r = project(op, op->xbar, op->q))) return r;
        HIP_TRY(launch_lin3_f32(y1, y1, 1.f, op->q, fs, b, -fs, nullptr, I, s));
        HIP_TRY(launch_grad_ball(op->xbar, op->p[0], op->n, fs, s));
        // x_new = P+(x - t (A^T y1 - div y2)),  xbar = 2 x_new - x
        HIP_TRY(launch_adjoint<float>(y1, nullptr, 1.f, 0.f, x, 1.f, -ft, xn, op->views, op->n, op->m, op->nb, s));
        HIP_TRY(launch_tv_finalize(xn, op->p[0], xn, op->n, -ft, s));
        HIP_TRY(launch_lin3_f32(op->xbar, xn, 2.f, x, -1.f, nullptr, 0.f, nullptr, J, s));
        std::swap(x, xn);
        if (k.record) {
            if ((r = project(op, x, op->q))) return r;
            if ((r = record_monitors(op, it, M, x, op->q, b, nullptr, nullptr))) return r;
        }
    }
    op->x = x;
    op->z = xn;
    if ((r = finish(op, iters, false, 1.0, op->p[0], rep, x_out, M))) return r;
    if (rep) {
        rep->tau = t;
        rep->sigma = sg;
        rep->kappa = 0.0;
        rep->lambda_a = lata;
        rep->lambda_h = 0.0;
        rep->norm_steps_a = steps_a;
        rep->norm_steps_h = 0;
        rep->iters_done = iters;
        rep->setup_ms = setup_ms;
        rep->loop_ms = ms_since(t1);
    }
    return CTPD_OK;
}

}  // extern "C"
