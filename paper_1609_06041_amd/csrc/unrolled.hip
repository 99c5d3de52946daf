// Algorithm 1 unrolled for a fixed number of iterations with given step sizes,
// as a differentiable function of the data b, the TV weight beta and the steps
// tau, sigma (the filter D = D(tau) of Eq. 24 depends on tau too).  The
// forward pass runs exactly the solver's kernels and keeps the state
// (x^k, mu^k, p^k) of every iteration in a caller-owned checkpoint buffer; the
// reverse pass walks the iterations backwards, recomputing each iteration's
// intermediates (the extrapolated dual variable, z, the inner TV dual fields)
// from its checkpoint, and applies the transposed operators: A^T for A, A for
// A^T, D and dD/dtau for themselves (symmetric Toeplitz), and the TV reverse
// kernels for the prox.  Scalar adjoints are float64 sums gathered into
// separate device slots and added on the host in a fixed order.
#include <algorithm>
#include <vector>

#include "op.h"

using namespace ctpd;

namespace ctpd_host {

struct UnrolledWs {
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
    float* ps = nullptr;   // tv_cap dual fields of one outer iteration (after steps 1..n_tv)
    double* part = nullptr;    // scalar-adjoint terms: slot_cap block sums per slot
    double* sums = nullptr;    // one total per slot
    int part_cap = 0;          // block sums per slot
    std::vector<double> sums_host;
};

void free_unrolled(UnrolledWs* u) {
    if (!u) return;
    void* ptrs[] = {u->dtaps64, u->dtaps32, u->ax,   u->axt, u->zbar, u->tbar, u->prod, u->amu,  u->amu2,
                    u->amup,    u->amup2,   u->ap,   u->pba, u->pbb,  u->qbar, u->e,    u->r,    u->dr,
                    u->dm,      u->rbar,    u->az,   u->daz, u->dpaz, u->ps,   u->part, u->sums};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete u;
}

}  // namespace ctpd_host

using namespace ctpd_host;

namespace {

int ensure_unrolled(ctpd_op* op, int tv_iters, int nslots) {
    if (!op->uw) {
        op->uw = new UnrolledWs();
        UnrolledWs* u = op->uw;
        const size_t J = op->J, I = op->I, T = 2 * (size_t)op->nb - 1;
        ALLOC(u->dtaps64, T);
        ALLOC(u->dtaps32, T);
        for (float** p : {&u->ax, &u->axt, &u->zbar, &u->tbar, &u->prod}) ALLOC(*p, J);
        for (float** p : {&u->amu, &u->amu2, &u->amup, &u->amup2, &u->e, &u->r, &u->dr, &u->dm, &u->rbar, &u->az,
                          &u->daz, &u->dpaz})
            ALLOC(*p, I);
        for (float** p : {&u->ap, &u->pba, &u->pbb, &u->qbar}) ALLOC(*p, 2 * J);
    }
    UnrolledWs* u = op->uw;
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

// kappa = mean(1/w) with the validity scan (queued; read back after the
// stream is synchronised), then W^-1 and the taps of D(tau).
int prepare_begin(ctpd_op* op, const float* b, const float* w) {
    HIP_TRY(launch_reduce(RED_INVW_CHECK, w, b, nullptr, op->I, op->partials, op->red, op->stream));
    HIP_TRY(hipMemcpyAsync(op->red_host, op->red, sizeof(double) * 3, hipMemcpyDeviceToHost, op->stream));
    return CTPD_OK;
}

int prepare_end(ctpd_op* op, const float* w, double tau, double* kappa) {
    if (op->red_host[1] > 0 || op->red_host[2] > 0) {
        snprintf(g_errmsg, sizeof g_errmsg, "%.0f weights <= 0 or non-finite, %.0f non-finite data",
                 op->red_host[1], op->red_host[2]);
        return CTPD_EDOMAIN;
    }
    *kappa = op->red_host[0] / (double)op->I;
    HIP_TRY(launch_inverse_f32(op->winv, w, op->I, op->stream));
    return ensure_taps(op, tau, *kappa);
}

int check_args(ctpd_op* op, const float* b, const float* w, double beta, double tau, double sigma, int iters) {
    if (!op || !b || !w) return einval("null pointer");
    if (!(beta >= 0.0) || !std::isfinite(beta)) return einval("beta must be finite and >= 0");
    if (!(tau > 0.0) || !std::isfinite(tau)) return einval("tau must be finite and > 0");
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return einval("sigma must be finite and > 0");
    if (iters < 1) return einval("iters must be >= 1");
    return CTPD_OK;
}

struct Slots {
    size_t x, mu, p, stride;
};

Slots layout(const ctpd_op* op) {
    const size_t J = op->J, I = op->I;
    return Slots{0, J, J + I, 3 * J + I};
}

// out = c * D s with the given float32 taps
int filt(ctpd_op* op, const float* taps, const float* in, float c, float* out, const float* E0 = nullptr,
         float e0 = 0.f) {
    FilterArgs a{};
    a.in0 = in;
    a.E0 = E0;
    a.e0 = e0;
    a.c = c;
    a.mode = FILT_PLAIN;
    a.out = out;
    HIP_TRY(launch_filter_f32(a, taps, op->m, op->nb, op->stream));
    return CTPD_OK;
}

// Each problem keeps its set-up readback in its operator, so an operator may
// appear once per call.
int check_distinct(ctpd_op* const* ops, int count) {
    std::vector<ctpd_op*> v(ops, ops + count);
    std::sort(v.begin(), v.end());
    if (std::adjacent_find(v.begin(), v.end()) != v.end()) return einval("an operator appears twice");
    return CTPD_OK;
}

// The forward iterations of one problem (after prepare_end), queued on its stream.
int forward_loop(ctpd_op* op, const float* b, double beta, double tau, double sigma, int iters, const Knobs& k,
                 float* ckpt, float* x_out) {
    int r = CTPD_OK;
    const size_t J = op->J;
    const Slots L = layout(op);
    hipStream_t s = op->stream;
    auto X = [&](int i) { return ckpt + (size_t)i * L.stride + L.x; };
    auto MU = [&](int i) { return ckpt + (size_t)i * L.stride + L.mu; };
    auto P = [&](int i) { return ckpt + (size_t)i * L.stride + L.p; };
    HIP_TRY(launch_fill_f32(ckpt, 0.f, L.stride, s));
    const float fs = (float)sigma, ft = (float)tau, lam = (float)(tau * beta);
    const float tvstep = lam > 0 ? (float)(k.tv_step / (tau * beta)) : 0.f;
    for (int it = 0; it < iters; ++it) {
        float *x = X(it), *mu = MU(it), *mup = MU(it > 0 ? it - 1 : 0);
        if (it == 0)
            r = filter(op, FILT_PLAIN, b, nullptr, nullptr, nullptr, nullptr, 0.f, nullptr, 0.f, -fs, op->mubar);
        else
            r = filter(op, FILT_EXTRAP, op->winv, mu, mup, nullptr, mu, 2.f, mup, -1.f, -fs, op->mubar);
        if (r) return r;
        HIP_TRY(launch_adjoint<float>(op->mubar, nullptr, 1.f, 0.f, x, 1.f, -ft, op->z, op->views, op->n, op->m,
                                      op->nb, s));
        HIP_TRY(launch_copy_f32(op->p[0], P(it), 2 * J, s));
        float* pf = nullptr;
        if ((r = tv_prox(op, op->z, lam, k.tv_iters, tvstep, op->p[0], op->p[1], X(it + 1), &pf))) return r;
        HIP_TRY(launch_copy_f32(P(it + 1), pf, 2 * J, s));
        if ((r = project(op, X(it + 1), op->q))) return r;
        if ((r = filter(op, FILT_DUAL_LD, op->q, b, op->winv, mu, mu, 1.f, nullptr, 0.f, fs, MU(it + 1)))) return r;
    }
    HIP_TRY(launch_copy_f32(x_out, X(iters), J, s));
    return CTPD_OK;
}

enum Cat { C_SIGMA, C_TAU, C_LAM, C_STEP };

// The reverse pass of one problem (after prepare_end), queued on its stream,
// ending with the copy of the scalar terms to the host (terms: their
// categories and factors, to be combined by combine_terms after a sync).
int backward_queue(ctpd_op* op, const float* b, double beta, double tau, double sigma, double kappa, int iters,
                   const Knobs& k, const float* ckpt, const float* x_grad, float* b_grad,
                   std::vector<std::pair<int, double>>& terms) {
    int r = CTPD_OK;
    const int nt = k.tv_iters;
    const int per_iter = 2 * nt + 6;
    UnrolledWs* u = op->uw;
    if (u->dtap_tau != tau || u->dtap_kappa != kappa) {
        HIP_TRY(launch_taps(u->dtaps64, u->dtaps32, op->nb, op->m, tau, kappa, op->stream, true));
        u->dtap_tau = tau;
        u->dtap_kappa = kappa;
    }
    const size_t J = op->J, I = op->I;
    const Slots L = layout(op);
    hipStream_t s = op->stream;
    auto X = [&](int i) { return ckpt + (size_t)i * L.stride + L.x; };
    auto MU = [&](int i) { return ckpt + (size_t)i * L.stride + L.mu; };
    auto P = [&](int i) { return ckpt + (size_t)i * L.stride + L.p; };
    const float fs = (float)sigma, ft = (float)tau, lam = (float)(tau * beta);
    const float tvstep = lam > 0 ? (float)(k.tv_step / (tau * beta)) : 0.f;
    const float* taps = op->taps32;
    const float* dtaps = u->dtaps32;
    // Scalar-adjoint terms: every term gets a slot of part_cap block sums
    // (written by the kernels that produce it), reduced once at the end and
    // added up on the host by category in a fixed order.
    terms.clear();
    auto slot = [&](int cat, double factor) -> double* {
        terms.emplace_back(cat, factor);
        return u->part + (size_t)(terms.size() - 1) * u->part_cap;
    };
    auto dot = [&](int cat, double factor, const float* a, const float* bb, size_t len) -> int {
        HIP_TRY(launch_dot_partials(a, bb, len, slot(cat, factor), s));
        return CTPD_OK;
    };
    HIP_TRY(launch_fill_f64(u->part, 0.0, (size_t)u->part_cap * iters * per_iter, s));
    // adjoint state of (x^{k+1}, mu^{k+1}, mu^k as the next iteration's mu_prev, p^{k+1})
    HIP_TRY(launch_copy_f32(u->ax, x_grad, J, s));
    HIP_TRY(launch_fill_f32(u->amu, 0.f, I, s));
    HIP_TRY(launch_fill_f32(u->amup, 0.f, I, s));
    HIP_TRY(launch_fill_f32(u->ap, 0.f, 2 * J, s));
    HIP_TRY(launch_fill_f32(b_grad, 0.f, I, s));
    for (int it = iters - 1; it >= 0; --it) {
        const float *x = X(it), *mu = MU(it), *mup = MU(it > 0 ? it - 1 : 0), *x1 = X(it + 1);
        // recompute the extrapolated dual variable, z and the inner dual fields
        const float* e = b;
        if (it == 0) {
            r = filter(op, FILT_PLAIN, b, nullptr, nullptr, nullptr, nullptr, 0.f, nullptr, 0.f, -fs, op->mubar);
        } else {
            HIP_TRY(launch_lin3_f32(u->e, mu, 1.f, mup, -1.f, nullptr, 0.f, op->winv, I, s));
            e = u->e;
            r = filter(op, FILT_EXTRAP, op->winv, mu, mup, nullptr, mu, 2.f, mup, -1.f, -fs, op->mubar);
        }
        if (r) return r;
        HIP_TRY(launch_adjoint<float>(op->mubar, nullptr, 1.f, 0.f, x, 1.f, -ft, op->z, op->views, op->n, op->m,
                                      op->nb, s));
        // PS(i): dual field after inner step i (PS(0) = p^k from the checkpoint)
        auto PS = [&](int i) -> const float* { return i == 0 ? P(it) : u->ps + (size_t)(i - 1) * 2 * J; };
        if (lam > 0 && nt > 0) {
            if (nt <= tv_chunk_max()) {
                HIP_TRY(launch_tv_steps_store(op->z, P(it), u->ps, op->n, lam, tvstep, nt, s));
            } else {
                for (int i = 1; i <= nt; ++i)
                    HIP_TRY(launch_tv_steps(op->z, PS(i - 1), u->ps + (size_t)(i - 1) * 2 * J, nullptr, op->n, lam,
                                            tvstep, 1, s));
            }
        }
        if ((r = project(op, x1, op->q))) return r;
        HIP_TRY(launch_lin_mix_f32(u->r, op->q, 1.f, b, -1.f, op->winv, mu, -1.f, I, s));
        // mu^{k+1} = mu + sigma D r
        if ((r = filt(op, taps, u->r, 1.f, u->dr))) return r;
        if ((r = dot(C_SIGMA, 1.0, u->amu, u->dr, I))) return r;
        if ((r = filt(op, dtaps, u->amu, 1.f, u->dm))) return r;
        if ((r = dot(C_TAU, sigma, u->dm, u->r, I))) return r;
        if ((r = filt(op, taps, u->amu, fs, u->rbar))) return r;
        // r = A x^{k+1} - b - W^-1 mu
        HIP_TRY(launch_lin_mix_f32(u->amu2, u->amu, 1.f, u->amup, 1.f, op->winv, u->rbar, -1.f, I, s));
        HIP_TRY(launch_adjoint<float>(u->rbar, nullptr, 1.f, 0.f, u->ax, 1.f, 1.f, u->axt, op->views, op->n, op->m,
                                      op->nb, s));
        HIP_TRY(launch_lin_mix_f32(b_grad, b_grad, 1.f, u->rbar, -1.f, nullptr, nullptr, 0.f, I, s));
        // x^{k+1}, p^{k+1} = prox(z, p^k)
        if (lam > 0) {
            HIP_TRY(launch_tv_bwd_final(op->z, PS(nt), u->axt, op->n, lam, u->tbar, u->zbar, slot(C_LAM, 1.0), s));
            // the adjoint of p^{k+1} (u->ap) becomes the first qbar buffer
            for (int i = nt; i >= 1; --i) {
                HIP_TRY(launch_tv_bwd_gradproj(op->z, PS(i - 1), u->ap, u->tbar, op->n, lam, tvstep,
                                               slot(C_STEP, 1.0), s));
                HIP_TRY(launch_tv_bwd_mask(op->z, PS(i - 1), u->ap, op->n, lam, tvstep, u->tbar, u->zbar,
                                           slot(C_LAM, 1.0), s));
            }
            HIP_TRY(launch_tv_bwd_grad(u->ap, u->tbar, op->n, lam, u->pba, s));
            std::swap(u->ap, u->pba);
        } else {
            // x^{k+1} = max(0, z), p passes through unchanged
            HIP_TRY(launch_tv_bwd_final(op->z, P(it), u->axt, op->n, 0.f, u->tbar, u->zbar, slot(C_LAM, 0.0), s));
        }
        // z = x^k - tau A^T mubar
        if ((r = project(op, u->zbar, u->az))) return r;
        if ((r = dot(C_TAU, -1.0, u->az, op->mubar, I))) return r;
        if ((r = filt(op, taps, u->az, 1.f, u->daz))) return r;
        if ((r = filt(op, dtaps, u->az, 1.f, u->dpaz))) return r;
        if ((r = dot(C_SIGMA, tau, u->daz, e, I))) return r;
        if ((r = dot(C_TAU, sigma * tau, u->dpaz, e, I))) return r;
        if (it == 0) {
            HIP_TRY(launch_lin_mix_f32(b_grad, b_grad, 1.f, u->daz, (float)(sigma * tau), nullptr, nullptr, 0.f, I,
                                       s));
        } else {
            HIP_TRY(launch_lin_mix_f32(u->amu2, u->amu2, 1.f, u->az, (float)(-2.0 * tau), op->winv, u->daz,
                                       (float)(sigma * tau), I, s));
            HIP_TRY(launch_lin_mix_f32(u->amup2, u->az, ft, nullptr, 0.f, op->winv, u->daz, (float)(-sigma * tau),
                                       I, s));
        }
        std::swap(u->ax, u->zbar);
        std::swap(u->amu, u->amu2);
        std::swap(u->amup, u->amup2);
    }
    const int ns = (int)terms.size();
    HIP_TRY(launch_slot_reduce(u->part, u->part_cap, ns, u->sums, s));
    u->sums_host.assign(ns, 0.0);
    HIP_TRY(hipMemcpyAsync(u->sums_host.data(), u->sums, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
    return CTPD_OK;
}

// d/dbeta, d/dtau, d/dsigma from the scalar terms (after the sync).
void combine_terms(const UnrolledWs* u, const std::vector<std::pair<int, double>>& terms, double beta, double tau,
                   double tv_step, double* grads) {
    double g_sigma = 0.0, g_tau = 0.0, g_lam = 0.0, g_step = 0.0;
    for (size_t i = 0; i < terms.size(); ++i) {
        const double v = terms[i].second * u->sums_host[i];
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
    if (count < 1 || count > CTPD_MAX_BATCH) return einval("count must be in 1..CTPD_MAX_BATCH");
    if (!ops || !b || !w || !beta || !tau || !sigma || !ckpt || !x_out) return einval("null pointer");
    int r;
    if ((r = check_distinct(ops, count))) return r;
    for (int i = 0; i < count; ++i) {
        if ((r = check_args(ops[i], b[i], w[i], beta[i], tau[i], sigma[i], iters))) return r;
        if (!ckpt[i] || !x_out[i]) return einval("null pointer");
    }
    Knobs k;
    if ((r = read_params(p, &k))) return r;
    for (int i = 0; i < count; ++i)
        if ((r = prepare_begin(ops[i], b[i], w[i]))) return r;
    for (int i = 0; i < count; ++i) {
        if ((r = sync(ops[i]))) return r;
        double kappa = 0.0;
        if ((r = prepare_end(ops[i], w[i], tau[i], &kappa))) return r;
        if ((r = forward_loop(ops[i], b[i], beta[i], tau[i], sigma[i], iters, k, ckpt[i], x_out[i]))) return r;
    }
    return CTPD_OK;
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
    if (count < 1 || count > CTPD_MAX_BATCH) return einval("count must be in 1..CTPD_MAX_BATCH");
    if (!ops || !b || !w || !beta || !tau || !sigma || !ckpt || !x_grad || !b_grad || !grads)
        return einval("null pointer");
    int r;
    if ((r = check_distinct(ops, count))) return r;
    for (int i = 0; i < count; ++i) {
        if ((r = check_args(ops[i], b[i], w[i], beta[i], tau[i], sigma[i], iters))) return r;
        if (!ckpt[i] || !x_grad[i] || !b_grad[i]) return einval("null pointer");
    }
    Knobs k;
    if ((r = read_params(p, &k))) return r;
    const int per_iter = 2 * k.tv_iters + 6;
    for (int i = 0; i < count; ++i) {
        if ((r = ensure_unrolled(ops[i], k.tv_iters, iters * per_iter))) return r;
        if ((r = prepare_begin(ops[i], b[i], w[i]))) return r;
    }
    std::vector<std::vector<std::pair<int, double>>> terms(count);
    for (int i = 0; i < count; ++i) {
        ctpd_op* op = ops[i];
        if ((r = sync(op))) return r;
        double kappa = 0.0;
        if ((r = prepare_end(op, w[i], tau[i], &kappa))) return r;
        UnrolledWs* u = op->uw;
        if (u->dtap_tau != tau[i] || u->dtap_kappa != kappa) {
            HIP_TRY(launch_taps(u->dtaps64, u->dtaps32, op->nb, op->m, tau[i], kappa, op->stream, true));
            u->dtap_tau = tau[i];
            u->dtap_kappa = kappa;
        }
        if ((r = backward_queue(op, b[i], beta[i], tau[i], sigma[i], kappa, iters, k, ckpt[i], x_grad[i], b_grad[i],
                                terms[i])))
            return r;
    }
    for (int i = 0; i < count; ++i) {
        if ((r = sync(ops[i]))) return r;
        combine_terms(ops[i]->uw, terms[i], beta[i], tau[i], k.tv_step, grads + 3 * i);
    }
    return CTPD_OK;
}

int ctpd_unrolled_lowdose_backward(ctpd_op* op, const float* b, const float* w, double beta, double tau,
                                   double sigma, int32_t iters, const ctpd_params* p, const float* ckpt,
                                   const float* x_grad, float* b_grad, double* grads) {
    return ctpd_unrolled_lowdose_backward_many(1, &op, &b, &w, &beta, &tau, &sigma, iters, p, &ckpt, &x_grad,
                                               &b_grad, grads);
}

}  // extern "C"
