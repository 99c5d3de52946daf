// Host-side internals of libctpd shared by the translation units that hold
// the C ABI (api.hip: operator handle, single operators, solvers; batch.hip:
// batched solves): the operator handle, error helpers, step-size set-up.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <functional>
#include <vector>

#include "internal.h"

using ctpd::ViewGeom;

namespace ctpd_host {
struct UnrolledWs;
void free_unrolled(UnrolledWs* u);
}  // namespace ctpd_host

// The operator handle: geometry tables and every workspace of a solve,
// allocated once per geometry.
struct ctpd_op {
    int n = 0, m = 0, nb = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    size_t J = 0, I = 0;   // image / sinogram sizes
    size_t Jp = 0;         // padded plane size n * (n + 6)
    ViewGeom* views = nullptr;
    int* fwd_tasks = nullptr;   // the slab projector's task groups (device), spread over the chip,
    int fwd_groups = 0;         // or with fwd_groups = 0 the split form's workgroup order
    int* bat_tasks = nullptr;   // the same tasks in the fewest groups, for batched launches
    int bat_groups = 0;
    // float32 iteration state
    float* xp = nullptr;    // padded image planes for the forward projector, [n][n+6] each
    float* xTp = nullptr;
    float* x = nullptr;
    float* z = nullptr;
    float* p[2] = {nullptr, nullptr};
    float* mu[3] = {nullptr, nullptr, nullptr};
    float* mubar = nullptr;
    float* q = nullptr;
    float* sx = nullptr;   // W^-1 (mu^{k+1} - mu^k), written by the dual update for the next extrapolation
    float* winv = nullptr;
    float* xbar = nullptr;   // Chambolle-Pock extrapolated image (allocated on first use)
    // filter taps for (tap_tau, tap_kappa)
    double* taps64 = nullptr;
    float* taps32 = nullptr;
    double tap_tau = -1.0, tap_kappa = -1.0;
    // at the default low-dose tau the taps are taps1 / kappa, taps1 those at
    // kappa = 1 (a property of the geometry), and so is the symbol bound
    double* taps1 = nullptr;   // 2 nb - 1 doubles
    double* sym1 = nullptr;    // 1 + kSymBlocks doubles (bound of the symbol of taps1 in [0])
    // reductions
    double* partials = nullptr;
    double* red = nullptr;        // device, 3 * kRedSlots doubles
    double* red_host = nullptr;   // pinned host mirror
    // float64 workspaces for the operator norms (allocated on first use)
    double* img64[3] = {nullptr, nullptr, nullptr};
    double* pad64[2] = {nullptr, nullptr};
    double* sino64[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // Lanczos recurrence scalars (device + pinned host mirror) and reduction
    // partials, one set per concurrent chain; chain 1 runs on the aux stream
    double* lz[2] = {nullptr, nullptr};
    double* lz_host[2] = {nullptr, nullptr};
    double* lz_partials[2] = {nullptr, nullptr};
    int lz_cap = 0;
    hipStream_t aux = nullptr;
    hipEvent_t fork = nullptr;
    // per-iteration monitor values (device), kMonSlots slots of 3 doubles per iteration
    double* cost_dev = nullptr;
    int cost_cap = 0;
    // operator norms that depend on the geometry only (see ctpd_params.sigma):
    // kappa * lambda_max(A^T D A) at a = 2 m tau / kappa (norm_ld_a), lambda_max(A^T D(1) A)
    // for few-view, lambda_max(A^T A) (Chambolle-Pock, D = I); 0 = not yet computed
    double norm_ld = 0.0, norm_ld_a = 0.0, norm_fv = 0.0, norm_ata = 0.0;
    int norm_ld_kmax = 0, norm_fv_kmax = 0, norm_ata_kmax = 0;
    // per-view lambda_h chains (allocated on first use): scalars per view and
    // step, and the one-problem tables the shared routine runs on
    double *hv_al = nullptr, *hv_b2 = nullptr, *hv_b0 = nullptr, *hv_theta = nullptr;
    int* hv_done = nullptr;
    double* hv_maxinv = nullptr;               // device, m doubles: max 1/w per view
    double* hv_ubound = nullptr;               // device, m doubles: Ritz value + residual norm per view
    double* hv_sym = nullptr;                  // device, 1 + kSymBlocks doubles: bound of the filter's symbol
    double hv_sym_tau = -1.0, hv_sym_kappa = -1.0;   // the taps hv_sym was computed for
    int hv_cap = 0;
    ctpd::NormItem* hv_item = nullptr;        // device, 1 entry
    ctpd::NormItem* hv_item_host = nullptr;   // pinned
    ctpd::RowRef* hv_rows = nullptr;          // device, m entries
    ctpd::BlockRef* hv_filt = nullptr;        // device, filter tiles
    int hv_nfilt = 0;
    double* hv_sum = nullptr;                 // device, 3 doubles
    double* hv_sum_host = nullptr;            // pinned, two slots of 3 doubles
    hipEvent_t hv_ev[2] = {nullptr, nullptr}; // behind the copies into the two slots
    hipEvent_t hv_start_ev = nullptr;           // behind the lambda_h chains' start
    // the error-tolerant few-view solve (allocated on first use): its data-side
    // variable y, the three float64 Lanczos vectors over the pair (x, y), and
    // the ball projection's norm and scale (device)
    float* ball_y = nullptr;
    double* split64 = nullptr;   // 3 (J + I) doubles
    double* ball_dev = nullptr;  // 2 doubles
    double norm_split = 0.0;     // lambda_max(K^T D(1) K), K = [A, -I]; 0 = not yet computed
    int norm_split_kmax = 0;
    // workspaces of the unrolled solve's reverse pass (allocated on first use)
    ctpd_host::UnrolledWs* uw = nullptr;
};

namespace ctpd_host {

using namespace ctpd;

constexpr int kRedSlots = 8;
extern thread_local char g_errmsg[512];

int fail_hip(hipError_t e, const char* what);
int alloc_dev(void** p, size_t bytes);
int einval(const char* msg);

#define HIP_TRY(expr)                                         \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return fail_hip(_e, #expr);     \
    } while (0)

#define ALLOC(ptr, count)                                                          \
    do {                                                                           \
        int _r = alloc_dev((void**)&(ptr), sizeof(*(ptr)) * (size_t)(count));      \
        if (_r != CTPD_OK) return _r;                                              \
    } while (0)

std::vector<ViewGeom> make_views(int n, int m, int nb, const double* angles);
int sync(ctpd_op* op);
int ensure_taps(ctpd_op* op, double tau, double kappa);
// the taps at the default low-dose tau for this kappa (and the symbol bound
// when the per-view lambda_h buffers exist), scaled from the cached kappa = 1 set
int ensure_taps_default(ctpd_op* op, double kappa);
int ensure_sym(ctpd_op* op);
int ensure_f64(ctpd_op* op);
int reduce(ctpd_op* op, int kind, const void* a, const void* b, const void* c, size_t len, int slot);
int read_red(ctpd_op* op);
double tridiag_max(const std::vector<double>& a, const std::vector<double>& b);
int ensure_lz(ctpd_op* op, int kmax);

using ApplyFn = std::function<int(const double*, double*)>;

struct Lanczos {
    ctpd_op* op = nullptr;
    int chain = 0;
    int per_round = 8;
    hipStream_t s = nullptr;
    double *q = nullptr, *qp = nullptr, *w = nullptr;
    size_t len = 0;
    int kmax = 0, j = 0, done = 0, steps = 0;
    bool converged = false;
    double theta = 0.0, theta_prev = 0.0;
    std::vector<double> al, be;
    ApplyFn apply;

    double* AL(int i) const { return op->lz[chain] + 3 * (1 + i); }
    double* B2(int i) const { return op->lz[chain] + 3 * (1 + op->lz_cap + i); }
    bool finished() const { return converged || done >= kmax; }

    int start(int rows, int cols, uint64_t seed, const float* wgt, double inv_kappa) {
        len = (size_t)rows * cols;
        double* s0 = op->lz[chain];
        HIP_TRY(launch_start_vector(q, rows, cols, seed, wgt, inv_kappa, s));
        HIP_TRY(launch_reduce(RED_DOT_F64, q, q, nullptr, len, op->lz_partials[chain], s0, s));
        HIP_TRY(launch_normalize(q, q, s0, len, s));
        return CTPD_OK;
    }
    // queue up to n more steps and the copy-back of the scalars
    int enqueue(int n) {
        const int end = std::min(kmax, j + n);
        for (; j < end; ++j) {
            int r = apply(q, w);
            if (r) return r;
            HIP_TRY(launch_reduce(RED_DOT_F64, q, w, nullptr, len, op->lz_partials[chain], AL(j), s));
            HIP_TRY(launch_lanczos_update(w, q, j ? qp : nullptr, AL(j), j ? B2(j - 1) : nullptr, len,
                                          op->lz_partials[chain], B2(j), s));
            HIP_TRY(launch_normalize(w, w, B2(j), len, s));
            double* t = qp;
            qp = q;
            q = w;
            w = t;
        }
        HIP_TRY(hipMemcpyAsync(op->lz_host[chain], op->lz[chain], sizeof(double) * 3 * (2 * op->lz_cap + 1),
                               hipMemcpyDeviceToHost, s));
        return CTPD_OK;
    }
    // after the stream is synchronised: extend the tridiagonal matrix and test
    // the top Ritz value (relative change <= 1e-9, or an invariant subspace)
    void absorb() {
        const double* h = op->lz_host[chain];
        for (int i = done; i < j && !converged; ++i) {
            al.push_back(h[3 * (1 + i)]);
            theta = tridiag_max(al, be);
            steps = i + 1;
            const double bn = std::sqrt(std::max(h[3 * (1 + op->lz_cap + i)], 0.0));
            if ((i > 0 && std::fabs(theta - theta_prev) <= 1e-9 * std::fabs(theta)) ||
                !(bn > 1e-300 * std::max(1.0, std::fabs(theta))))
                converged = true;
            be.push_back(bn);
            theta_prev = theta;
        }
        done = j;
    }
};

int run_lanczos(const std::vector<Lanczos*>& chains);
int setup_lambda_a(ctpd_op* op, int kmax, Lanczos* L, bool filt = true, const float* wgt = nullptr);

// Sout (optional, with Sw and E0): also Sout = Sw .* (out - E0)
int filter(ctpd_op* op, int mode, const float* in0, const float* in1, const float* in2, const float* in3,
           const float* E0, float e0, const float* E1, float e1, float c, float* out, const float* Sw = nullptr,
           float* Sout = nullptr);
int project(ctpd_op* op, const float* x, float* y);
// y = A x - rb - rw .* rm (rb null: y = A x); padded: the planes of x are current
// (the TV prox wrote them), so they are not padded again
int project_resid(ctpd_op* op, const float* x, const float* rb, const float* rw, const float* rm, float* y,
                  bool padded = false);
int tv_prox(ctpd_op* op, const float* z, float lam, int n_iter, float step, float* pin, float* scratch, float* x,
            float** pout, bool planes = false);

struct Knobs {
    double tau, sigma, tv_step, rho;
    int tv_iters, norm_steps, record;
    ctpd_state* state;   // the checkpoint to start from and write back, or null
    bool resumed() const { return state && state->k > 0; }
};

// Per-iteration monitors a report asks for (float64 sums on the device).
// Slots of 3 doubles per iteration in op->cost_dev:
enum MonSlot : int {
    MON_TV = 0,      // psi(x) (Eq. 2)
    MON_DATA = 1,    // sum w (Ax - b)^2 (low-dose) or sum (Ax - b)^2 (few-view)
    MON_GAP = 2,     // sum (w (Ax - b) - mu)^2 / w  (twice the partial gap)
    MON_RES = 3,     // sum (Ax - b)^2
    MON_RMSE = 4,    // sum (x - x_ref)^2
    kMonSlots = 5,
};
struct Monitors {
    bool cost = false, gap = false, resid = false, rmse = false;
    const float* x_ref = nullptr;
    double bnorm2 = 0.0;   // ||b||^2, for resid
    bool any() const { return cost || gap || resid || rmse; }
};

int read_params(const ctpd_params* p, Knobs* k);
// CTPD_EINVAL when a checkpoint state was given (the solvers without one)
int no_state(const Knobs& k);
// the monitors rep asks for (gap_ok: the solver defines the partial gap);
// sets k->record when any is asked for
int read_monitors(const ctpd_report* rep, bool gap_ok, Knobs* k, Monitors* M);
// ||b||^2 into M->bnorm2 when resid is asked for (synchronises)
int monitor_bnorm(ctpd_op* op, const float* b, Monitors* M);
// queue the monitors of iteration `it`: x the iterate, q = A x, mu the new dual
// (low-dose: w given)
int record_monitors(ctpd_op* op, int it, const Monitors& M, const float* x, const float* q, const float* b,
                    const float* w, const float* mu);
int ensure_cost(ctpd_op* op, int iters);
double ms_since(std::chrono::steady_clock::time_point t0);
int finish(ctpd_op* op, int iters, bool lowdose, double beta, float* p_final, ctpd_report* rep, float* x_out,
           const Monitors& M);

// Set-up of Algorithm 1 (see api.hip).
constexpr double kTauMultLowdose = 0.3;   // default tau = 0.3 pi kappa / (2m)

struct LowdoseSetup {
    double kappa = 0.0, tau = 0.0, sigma = 0.0, lam_a = 0.0, lam_h = 0.0;
    double a = 0.0;         // 2 m tau / kappa: kappa * lambda_a depends on the geometry and a only
    int steps_a = 0, steps_h = 0;
    bool run_a = false;     // lambda_a from the chain (else from the handle's cache)
    Lanczos La;
};
int lowdose_setup_begin(ctpd_op* op, const float* b, const float* w, const Knobs& k, LowdoseSetup* S);

// lambda_max(W^-1/2 D W^-1/2) of each handle by per-view Lanczos chains run in
// lockstep on stream s (needs op->sino64[3] = sqrt(1/w) and the taps).  items:
// device / pinned tables of ops.size() entries; rows: every (problem, view);
// filt: the filter tiles of all problems; summary: 3 doubles per problem on
// the device, two slots of 3 per problem pinned, with an event for each slot.
// lam[i], steps[i] receive the results.  A round may still run on s after the
// return (one queued ahead that found every chain stopped: it changes nothing).
int ensure_hv(ctpd_op* op, int kmax);
// side (optional) is called once the first round is queued, with an event
// recorded on s behind the chains' start (before that round): work queued
// behind it runs beside the first round, which was dispatched first.
int lambda_h_views(const std::vector<ctpd_op*>& ops, const float* const* w, const double* kappa, int kmax,
                   hipStream_t s, ctpd::NormItem* items, ctpd::NormItem* items_host, const ctpd::RowRef* rows,
                   int nrows, const ctpd::BlockRef* filt, int nfilt, double* summary, double* summary_host,
                   const hipEvent_t* ev, double* lam, int* steps,
                   const std::function<int(hipEvent_t)>& side = nullptr, hipEvent_t side_ev = nullptr);
// lambda_a from the chain or the cache, then sigma: the default, or the given
// one checked against the bound (CTPD_EINVAL when it violates it)
int lowdose_setup_end(ctpd_op* op, const Knobs& k, LowdoseSetup* S);

// Workgroup placement of batched launches: problems go to XCDs by work
// (largest first onto the least-loaded XCD); placement 0 interleaves the XCD
// bins so that consecutive workgroups of a problem land on its own XCD (each
// XCD has its own L2), placement 1 lays the problems out one after another,
// largest first.  counts[p]: workgroups of problem p in the launch.
constexpr int kXcds = 8;
struct Placement {
    std::vector<int> order, xcd;
};
Placement plan_xcds(const std::vector<double>& work);
std::vector<ctpd::BlockRef> place_blocks(const Placement& pl, const std::vector<int>& counts, int placement);

}  // namespace ctpd_host
