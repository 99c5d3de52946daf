/*
 * ctpd.h -- C ABI of libctpd: FBP-preconditioned primal-dual (APP) TV
 * reconstruction for parallel-beam CT on AMD Instinct MI355X (gfx950).
 *
 * Method: Kudo, Yamazaki, Nemoto, Takaki, "A very fast iterative algorithm
 * for TV-regularized image reconstruction with applications to low-dose and
 * few-view CT" (arXiv 1609.06041).
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - Image x: n x n float32, row-major x[iy*n + ix], unit pixels, pixel
 *    centre (ix - (n-1)/2, iy - (n-1)/2).
 *  - Sinogram: view-major float32 [n_views][n_bins]; view v is at angle
 *    theta_v = v*pi/n_views (uniform over [0, pi)), bin u at signed distance
 *    r_u = u - (n_bins-1)/2; the ray of (v, u) is x cos + y sin = r_u.
 *  - A is Joseph's ray-driven projector: views with |cos| >= |sin| (decided
 *    from the view index: 4v <= m or 4v >= 3m) step over rows and linearly
 *    interpolate along x with step length 1/|cos|, the others step over
 *    columns with 1/|sin|; pixels outside the image are zero.
 *  - Every array argument is a DEVICE pointer to a densely packed buffer the
 *    caller allocates and owns, unless marked "host".  Inputs are never
 *    modified.  Outputs must not alias inputs.
 *  - Work is queued on the hipStream_t given to ctpd_op_create, in stream
 *    order.  project / backproject / ramp_filter / tv_prox return without
 *    waiting; the solvers wait for their own results before returning.
 *  - Return value: CTPD_OK (0) or a negative error code.  On an argument
 *    error nothing is launched and no output is written, with one
 *    exception: a step size given by the caller is checked against the
 *    convergence bound of its solver (Eq. 16 and the conditions stated with
 *    Algorithms 1 and 2) after the operator norms the bound needs have been
 *    computed on the device; a violation returns CTPD_EINVAL before any
 *    iteration runs or any output is written.  ctpd_strerror gives a message
 *    (for CTPD_EHIP it includes the HIP error of the last failure on the
 *    calling thread).
 *  - An op is not thread-safe: calls on one op must not overlap.
 */
#ifndef CTPD_H
#define CTPD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CTPD_OK 0
#define CTPD_EINVAL (-1)   /* bad argument: null pointer, size, step size, ... */
#define CTPD_EDOMAIN (-2)  /* data outside the model: w_i <= 0 or non-finite b, w */
#define CTPD_EHIP (-3)     /* a HIP runtime call failed */
#define CTPD_ENOMEM (-4)   /* device allocation failed */

/* Maximum n_bins (it bounds the LDS the filters stage their taps in). */
#define CTPD_MAX_BINS 4096
/* Maximum number of problems in one batch. */
#define CTPD_MAX_BATCH 4096
/* Maximum ctpd_params.norm_steps. */
#define CTPD_MAX_NORM_STEPS 512

typedef struct ctpd_op ctpd_op;
typedef struct ctpd_batch ctpd_batch;

/* Scan geometry (Sec. 2.1: parallel-beam, m views over [0, pi)). */
typedef struct {
    int32_t n;        /* image side, 1 <= n <= 8192 */
    int32_t n_views;  /* m >= 1 */
    int32_t n_bins;   /* 1 <= n_bins <= CTPD_MAX_BINS */
    int32_t reserved; /* 0 */
    const double* angles;  /* host array of the n_views view angles in radians, any
                              order and range (copied at creation; finite, else
                              CTPD_EINVAL), or NULL for theta_v = v pi / m.  A view
                              steps over image rows where |cos| >= |sin| (1 - 1e-12).
                              D keeps Eqs. 24 / 32 with the view count m: with
                              uneven angles it is still a valid preconditioner,
                              no longer the FBP filter of the scan. */
} ctpd_geometry;

struct ctpd_state; /* below */

/* Solver knobs.  A zero / negative value selects the default. */
typedef struct {
    double tau;          /* primal step; default: low-dose 0.3*pi*kappa/(2m), few-view
                            mean|sigma A^T D(1) b| */
    double sigma;        /* dual step; default: rho times the bound of Eq. 16 /
                            Algorithm 1 / Algorithm 2 from the operator norms.
                            A given sigma must satisfy that bound strictly:
                            low-dose sigma < min(2/lambda_h, 1/(tau lambda_A)),
                            few-view sigma lambda_max(A^T D(1) A) < 1,
                            error-tolerant few-view sigma lambda_max(K^T D(1) K) < 1
                            (K = [A, -I]); the norms are computed (or taken from
                            the handle's cache) and a violation gives CTPD_EINVAL.
                            kappa lambda_max(A^T D A) depends only on the geometry
                            and a = 2 m tau / kappa (H of Eq. 24 is
                            (1/kappa) |w| / (a + |w|)), and the few-view
                            lambda_max(A^T D(1) A) and lambda_max(K^T D(1) K) on
                            the geometry only: the handle keeps the last value of
                            each and reuses it. */
    double tv_step;      /* tau_c of the TV dual iteration, default 1/8 */
    double safety;       /* rho < 1, default 0.95 */
    int32_t tv_iters;    /* inner TV steps per outer iteration, default 10 */
    int32_t norm_steps;  /* max Lanczos steps per operator norm, default 100,
                            at most CTPD_MAX_NORM_STEPS */
    int32_t record_cost; /* 1: fill ctpd_report.cost (Eq. 1 cost, or psi for few-view).
                            Monitors (cost, gap, resid, rmse) are computed per
                            iteration in float64 on the device when requested; the
                            solver then runs the filters' fused-prologue path,
                            whose iterates equal the default path's bit for bit. */
    int32_t reserved;
    struct ctpd_state* state; /* NULL, or the checkpoint the solve starts from and
                            writes its end state into (ctpd_pd_lowdose_solve,
                            ctpd_pd_fewview_solve, ctpd_pd_fewview_eps_solve;
                            CTPD_EINVAL for the other solvers) */
} ctpd_params;

/* Checkpoint of an APP solve (Algorithms 1, 1', 2 and the error-tolerant
 * few-view solve): the iterates an iteration reads, so that K1 iterations
 * followed by K2 more from the checkpoint give the K1 + K2 iterations of one
 * solve bit for bit.  The arrays are the caller's device memory, read at the
 * start of a solve and overwritten with the state after its last iteration.
 * k == 0 starts from x = 0, mu = mu_prev = 0, p = 0 (y = b) with the step
 * sizes of the params (the arrays are not read); k > 0 resumes with the
 * state's tau and sigma (both > 0, checked against the step-size bound like
 * given ones), and the iteration after k uses the extrapolation of k >= 1. */
typedef struct ctpd_state {
    float* x;        /* [n][n] x^k */
    float* mu;       /* [n_views][n_bins] mu^k */
    float* mu_prev;  /* [n_views][n_bins] mu^{k-1} */
    float* p;        /* [2][n][n] the TV dual field (the next prox's warm start) */
    float* y;        /* [n_views][n_bins] the error-tolerant solve's y^k, else NULL */
    int32_t k;       /* iterations behind the state; the solve adds its iters */
    int32_t reserved;
    double tau, sigma;  /* the step sizes of those iterations (written by the solve) */
} ctpd_state;

/* Solver report (host struct filled by the solvers). */
typedef struct {
    double tau, sigma;   /* step sizes used */
    double kappa;        /* mean of diag(W^-1) (low-dose) */
    double lambda_a;     /* lambda_max(A^T D A) = ||D^1/2 A A^T D^T/2|| at the tau used */
    double lambda_h;     /* lambda_max(W^-1/2 D W^-1/2) = ||D^1/2 W^-1 D^T/2|| (low-dose) */
    int32_t norm_steps_a, norm_steps_h;  /* Lanczos steps taken (0: lambda_a from the handle's cache) */
    int32_t iters_done;
    int32_t reserved;
    double setup_ms;     /* host wall time of the set-up (norms, taps, defaults) */
    double loop_ms;      /* host wall time of the iterations */
    double* cost;        /* host, length >= iters, or NULL */
    float* mu_out;       /* device [n_views][n_bins] receives mu^K, or NULL */
    float* p_out;        /* device [2][n][n] receives the TV dual field, or NULL */
    /* Per-iteration convergence monitors, float64 sums on the device over the
     * iterate after each iteration k = 1..iters (host arrays of length >= iters,
     * each NULL when not wanted): */
    double* gap;         /* partial primal-dual gap f(x^k) - L(x^k, mu^k)
                            = 1/2 ||W^1/2 (A x^k - b) - W^-1/2 mu^k||^2 (Eq. 10 with the
                            theorem after it; zero at the saddle point).  Only the
                            low-dose APP solvers (Algorithm 1 and its D = I
                            ablation); CTPD_EINVAL elsewhere. */
    double* resid;       /* ||A x^k - b|| / ||b|| (the constraint of Eq. 25; all solvers) */
    double* rmse;        /* sqrt(mean((x^k - x_ref)^2)), Eq. 34 (all solvers; needs x_ref) */
    const float* x_ref;  /* device [n][n] reference image for rmse, or NULL */
} ctpd_report;

/* Create an operator for geometry *g bound to stream (a hipStream_t; NULL =
 * the null stream) on the current HIP device.  Allocates the geometry tables
 * and all iteration workspaces once.  *out receives the handle. */
int ctpd_op_create(const ctpd_geometry* g, void* stream, ctpd_op** out);

/* Release the op and its device memory (waits for its stream).  NULL is a no-op. */
void ctpd_op_destroy(ctpd_op* op);

/* y = A x (Sec. 2.1 system matrix; Eqs. 18-20 forward projection).
 * x: [n][n], y: [n_views][n_bins]. */
int ctpd_project(ctpd_op* op, const float* x, float* y);

/* x = A^T y, the exact transpose of ctpd_project (Eqs. 19, 30 backprojection).
 * y: [n_views][n_bins], x: [n][n]. */
int ctpd_backproject(ctpd_op* op, const float* y, float* x);

/* out = D s, the preconditioner of Eq. 24 (kappa > 0, smoothed ramp
 * H = |w|/(2 m tau + kappa |w|)) or Eq. 32 (kappa == 0, ramp H = |w|/(2 m tau)),
 * applied to every view as the linear convolution with the inverse DTFT of H
 * band-limited to [-pi, pi] rad/bin.  tau > 0, kappa >= 0.
 * s, out: [n_views][n_bins]. */
int ctpd_ramp_filter(ctpd_op* op, double tau, double kappa, const float* s, float* out);

/* The same D in float64 (the precision the operator norms are computed in):
 * out = D s for float64 s, out: [n_views][n_bins]. */
int ctpd_ramp_filter_f64(ctpd_op* op, double tau, double kappa, const double* s, double* out);

/* The 2*n_bins-1 filter taps h[k - (n_bins-1)], k = 0..2n_bins-2, of
 * ctpd_ramp_filter in float64, copied to the host array taps_host (blocks). */
int ctpd_filter_taps(ctpd_op* op, double tau, double kappa, double* taps_host);

/* TV prox with non-negativity (Eq. 17): approximately
 *   x = argmin_{x >= 0} lambda psi(x) + 1/2 ||x - z||^2,  psi of Eq. 2,
 * by n_iter projected-gradient steps of size tv_step/lambda on the dual field
 * p, warm-started from p_inout (updated in place), then x = max(0, z - lambda div p).
 * lambda == 0 gives x = max(0, z).  z, x: [n][n]; p_inout: [2][n][n]
 * (horizontal then vertical component, |p_j| <= 1). */
int ctpd_tv_prox(ctpd_op* op, const float* z, double lambda, int32_t n_iter, double tv_step,
                 float* p_inout, float* x);

/* Low-dose P-WLS TV reconstruction (Eq. 1), Algorithm 1 (beta > 0) or
 * Algorithm 1' (beta == 0): iters APP iterations (Eqs. 18-20) from x = 0,
 * mu = 0 with the smoothed-ramp preconditioner of Eq. 24.
 * b: [n_views][n_bins] log data; w: [n_views][n_bins] weights w_i = 1/var_i > 0;
 * x_out: [n][n].  p may be NULL (defaults); rep may be NULL.
 * Synchronises the op's stream before returning. */
int ctpd_pd_lowdose_solve(ctpd_op* op, const float* b, const float* w, double beta, int32_t iters,
                          const ctpd_params* p, float* x_out, ctpd_report* rep);

/* Few-view reconstruction min psi(x) s.t. Ax = b, x >= 0 (Eq. 25),
 * Algorithm 2: iters APP iterations (Eqs. 29-31) with the ramp of Eq. 32.
 * Arguments as for ctpd_pd_lowdose_solve without w and beta. */
int ctpd_pd_fewview_solve(ctpd_op* op, const float* b, int32_t iters, const ctpd_params* p,
                          float* x_out, ctpd_report* rep);

/* Error-tolerant few-view reconstruction, the extension the conclusions
 * (Sec. 5) name for noisy few-view data:
 *   min psi(x)  s.t.  ||A x - b|| <= eps,  x >= 0.
 * Posed like Eqs. 6-7: a data-side variable y with the preconditioned
 * constraint D^1/2 (A x - y) = 0 and the indicator of the ball
 * {y : ||y - b|| <= eps} as its data term; APP on the pair (x, y) gives
 * Eqs. 29-31 with the primal step split into the TV prox of Eq. 17 and the
 * Euclidean projection onto the ball.  Per iteration from x = 0, y = b,
 * mu = 0:
 *   mubar = -sigma D b (k = 0), 2 mu^k - mu^{k-1} (k >= 1)
 *   x = prox(x - tau A^T mubar);  y = P_ball(y + tau mubar)
 *   mu = mu + sigma D (A x - y)       (D the ramp of Eq. 32).
 * eps = 0 keeps y = b and gives Algorithm 2 (ctpd_pd_fewview_solve) bit for
 * bit at the same tau and sigma.  Step sizes: sigma < 1/lambda_max(K^T D(1) K)
 * with K = [A, -I] (Eq. 16 for the pair; D(tau) = D(1)/tau), checked when
 * given (CTPD_EINVAL), default rho / lambda_max (computed in float64 by the
 * first solve on the handle and cached); default tau as in
 * ctpd_pd_fewview_solve.  The report's lambda_a is lambda_max(K^T D(tau) K).
 * eps: finite and >= 0 (CTPD_EINVAL otherwise).  Monitors: cost (psi),
 * resid (||A x - b|| / ||b||), rmse; not gap.  Other arguments as for
 * ctpd_pd_fewview_solve. */
int ctpd_pd_fewview_eps_solve(ctpd_op* op, const float* b, double eps, int32_t iters,
                              const ctpd_params* p, float* x_out, ctpd_report* rep);

/* ---- batched solves ------------------------------------------------------
 * Many independent low-dose problems (Eq. 1) of uneven image sizes and view
 * counts solved together by Algorithm 1, each with its own set-up exactly as
 * in ctpd_pd_lowdose_solve (its own kappa, tau, taps and sigma), iterated in
 * lockstep: one launch per kernel and step covers every problem, and the
 * whole iters-iteration loop is captured once as a HIP graph and replayed on
 * later calls with the same iters / tv_iters. */

/* Create a batch of count problems with geometries geoms[0..count-1] (host
 * array), bound to stream (the caller's hipStream_t; inputs are read after
 * the work queued on it so far).  Allocates every problem's workspaces.
 * CTPD_EINVAL for count outside [1, CTPD_MAX_BATCH] or a bad geometry. */
int ctpd_batch_create(const ctpd_geometry* geoms, int32_t count, void* stream, ctpd_batch** out);

/* Release the batch (waits for its work).  NULL is a no-op. */
void ctpd_batch_destroy(ctpd_batch* batch);

/* iters iterations of Algorithm 1 on every problem.  b, w, x_out: host arrays
 * of count device pointers (problem i: b[i], w[i] [n_views][n_bins],
 * x_out[i] [n][n]); beta: host array of count values >= 0.  p applies to
 * every problem (record_cost is ignored).  reps: NULL or a host array of
 * count reports (tau, sigma, kappa, norms and step counts per problem;
 * setup_ms / loop_ms are the batch's; cost, mu_out, p_out are not used).
 * Synchronous.  Errors as for ctpd_pd_lowdose_solve (the first failing
 * problem decides). */
int ctpd_batch_lowdose_solve(ctpd_batch* batch, const float* const* b, const float* const* w,
                             const double* beta, int32_t iters, const ctpd_params* p, float* const* x_out,
                             ctpd_report* reps);

/* ---- unrolled, differentiable Algorithm 1 --------------------------------
 * x^K as a function of (b, beta, tau, sigma): exactly iters iterations of
 * Eqs. 18-20 from zero with the given step sizes (no operator norms) and
 * D = D(tau), the smoothed ramp of Eq. 24 at kappa = mean(1/w).  The forward
 * pass keeps every iteration's state in a caller-owned checkpoint buffer; the
 * reverse pass returns the gradient of <x_grad, x^K> with respect to b and
 * the three scalars. */

/* Number of floats of the checkpoint buffer for iters iterations:
 * (iters + 1) * (3 n^2 + n_views n_bins) (x^k, mu^k, p^k per iteration). */
int ctpd_unrolled_ckpt_floats(const ctpd_op* op, int32_t iters, size_t* count);

/* Forward pass.  b, w: [n_views][n_bins] (as ctpd_pd_lowdose_solve); beta >= 0,
 * tau > 0, sigma > 0, iters >= 1; p: NULL or knobs (tv_iters, tv_step are
 * used); ckpt: device buffer of ctpd_unrolled_ckpt_floats floats, written;
 * x_out: [n][n] receives x^iters.  Same arithmetic as ctpd_pd_lowdose_solve at
 * these step sizes.  Stream-ordered after one host synchronisation (kappa). */
int ctpd_unrolled_lowdose_forward(ctpd_op* op, const float* b, const float* w, double beta, double tau,
                                  double sigma, int32_t iters, const ctpd_params* p, float* ckpt, float* x_out);

/* Reverse pass for the same arguments and the checkpoints of the forward
 * pass.  x_grad: [n][n] adjoint of x^iters; b_grad: [n_views][n_bins]
 * receives d<x_grad, x^K>/db; grads (host, 3 doubles) receives the
 * derivatives with respect to beta, tau, sigma.  Synchronises the stream. */
int ctpd_unrolled_lowdose_backward(ctpd_op* op, const float* b, const float* w, double beta, double tau,
                                   double sigma, int32_t iters, const ctpd_params* p, const float* ckpt,
                                   const float* x_grad, float* b_grad, double* grads);

/* The forward / reverse passes of count independent problems in one call
 * (1 <= count <= CTPD_MAX_BATCH; every pointer array holds count entries,
 * scalars count doubles, grads 3 * count doubles laid out as (beta, tau,
 * sigma) per problem), with the arithmetic of the single calls above (which
 * are this call with count = 1).  The whole call runs on the first operator's
 * stream: every problem's pass is recorded as a list of kernel steps and each
 * step runs as one launch over all the problems, so small problems fill the
 * GPU together.  The call first synchronises the other operators' streams and
 * then once more for all the kappa reductions; the reverse pass synchronises
 * again at the end for the scalar gradients.  The operators must be distinct
 * (CTPD_EINVAL otherwise). */
int ctpd_unrolled_lowdose_forward_many(int32_t count, ctpd_op* const* ops, const float* const* b,
                                       const float* const* w, const double* beta, const double* tau,
                                       const double* sigma, int32_t iters, const ctpd_params* p,
                                       float* const* ckpt, float* const* x_out);
int ctpd_unrolled_lowdose_backward_many(int32_t count, ctpd_op* const* ops, const float* const* b,
                                        const float* const* w, const double* beta, const double* tau,
                                        const double* sigma, int32_t iters, const ctpd_params* p,
                                        const float* const* ckpt, const float* const* x_grad, float* const* b_grad,
                                        double* grads);

/* Tile shapes and workgroup placement of the batched kernels (chosen by an
 * autotuner that times ctpd_batch_time_loop over the candidates). */
typedef struct {
    int32_t placement;   /* 0: each problem's workgroups on one XCD (default); 1: problem-major order */
    int32_t tv_threads;  /* threads per 32 x 32 TV tile: 512 or 1024 (default) */
    int32_t fwd_form;    /* forward projector: 0 the slab form (default; every image side <= 634),
                            1 the gather form; both give the same bits */
    int32_t reserved;
} ctpd_batch_tiles;

/* Set / read the batch's tile choices (CTPD_EINVAL for values outside the
 * lists above).  Setting recaptures the loop graph on the next call. */
int ctpd_batch_set_tiles(ctpd_batch* batch, const ctpd_batch_tiles* tiles);
int ctpd_batch_get_tiles(const ctpd_batch* batch, ctpd_batch_tiles* tiles);

/* Replay the iters-iteration loop of the last solve's set-up reps times and
 * return the median device time per replay in *ms (HIP events).  The inputs
 * of the last solve must still be valid; results are overwritten with the
 * same values.  CTPD_EINVAL before the first solve. */
int ctpd_batch_time_loop(ctpd_batch* batch, int32_t iters, int32_t tv_iters, int32_t reps, double* ms);

/* Ablation of Algorithm 1 without its preconditioner (Sec. 3 derives D as the
 * FBP filter; here D = I): the same iteration, Eqs. 18-20, with D replaced by
 * the identity.  Step sizes from Eq. 16 with D = I: lambda_A = lambda_max(A^T A)
 * (a property of the geometry, cached per handle as for the Chambolle-Pock
 * comparator), lambda_h = lambda_max(W^-1) = max 1/w; default tau =
 * lambda_h / (2 lambda_A), where the two bounds on sigma coincide, and sigma =
 * rho min(2 / lambda_h, 1 / (tau lambda_A)).  Arguments, knobs and report as
 * ctpd_pd_lowdose_solve (norm_steps_h = 0). */
int ctpd_app_identity_lowdose_solve(ctpd_op* op, const float* b, const float* w, double beta, int32_t iters,
                                    const ctpd_params* p, float* x_out, ctpd_report* rep);

/* Comparator for the low-dose problem of Eq. 1 (Sec. 4 compares Algorithm 1
 * with it; Table 1 lists it): GIST, the Loris-Verhoeven iteration -- a
 * gradient step on the weighted data term, a projection step on the dual of
 * the TV penalty -- with x >= 0 entering as the projection of the
 * Chen-Huang-Zhang primal-dual fixed-point form.  Per iteration from x = 0,
 * v = 0:  u = x - gamma A^T W (A x - b);  y = P+(u + lam div v);
 * v = projection of (v + grad y) onto {|v_j| <= gamma beta / lam};
 * x = P+(u + lam div v).  No preconditioner.
 * Arguments as for ctpd_pd_lowdose_solve.  ctpd_params.tau is gamma (default
 * rho * 2 / lambda_max(A^T W A)), ctpd_params.sigma is lam (default and
 * maximum 1/8); the report's lambda_a is lambda_max(A^T W A) (0 when gamma
 * was given) and p_out receives v. */
int ctpd_gist_lowdose_solve(ctpd_op* op, const float* b, const float* w, double beta, int32_t iters,
                            const ctpd_params* p, float* x_out, ctpd_report* rep);

/* Comparator for the few-view problem of Eq. 25 (Sec. 4 compares Algorithm 2
 * with it; Table 1 lists it): Chambolle-Pock (theta = 1) with K = [A; grad].
 * Per iteration from zero:  y1 += s (A xbar - b);  y2 = projection of
 * (y2 + s grad xbar) onto the unit ball;  x' = P+(x - t (A^T y1 - div y2));
 * xbar = 2 x' - x.  No preconditioner.  ctpd_params.tau is t and
 * ctpd_params.sigma is s (default both rho / sqrt(lambda_max(A^T A) + 8));
 * the report's lambda_a is lambda_max(A^T A) (0 when both were given);
 * mu_out receives y1 and p_out y2.  Arguments as for ctpd_pd_fewview_solve. */
int ctpd_cp_fewview_solve(ctpd_op* op, const float* b, int32_t iters, const ctpd_params* p, float* x_out,
                          ctpd_report* rep);

/* y = A x for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same projection as ctpd_project for the scan g with uniform angles
 * theta_v = v pi / n_views (g->angles must be NULL), with no handle and no
 * allocation.  Its scratch -- the view table and the two zero-padded image
 * planes -- is one static device array of 8.7 MB that each GPU the library
 * runs on keeps until the process ends; every call on a GPU shares it, so
 * calls that overlap on one GPU (two streams, two threads) race and must be
 * serialised by the caller.  Limits: 1 <= n <= 1024, 1 <= n_views <= 4096,
 * 1 <= n_bins <= CTPD_MAX_BINS, else CTPD_EINVAL (nothing launched).
 * stream: the hipStream_t the work is queued on (NULL = the null stream);
 * x: [n][n], y: [n_views][n_bins], device.  Returns without waiting. */
int ctpd_project_noalloc(const ctpd_geometry* g, void* stream, const float* x, float* y);

/* Static message for an error code. */
const char* ctpd_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* CTPD_H */
