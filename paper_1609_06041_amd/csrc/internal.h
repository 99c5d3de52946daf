// Internal declarations shared by the HIP translation units of libctpd.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "ctpd.h"

// the LDS operand of the global-to-LDS copy builtin
typedef __attribute__((address_space(3))) void lds_void_t;

namespace ctpd {

// Per-view geometry, built on the host in float64 (see make_views in api.hip).
//
// Ray-driven form (forward projector): view v steps over t = 0..n-1 (rows when
// row != 0, else columns) and ray u samples the interpolation axis at
//     s(t, u) = s0 + u * su + t * st        (pixel-index units)
// with step length len.  Pixel-driven form (transpose): pixel (X, Y) in
// centred coordinates lies at bin coordinate  X*cs + Y*sn + (nb-1)/2, and a
// bin at distance d from it carries the hat weight max(0, len - d*len2).
struct ViewGeom {
    double su, st, s0;
    double cs, sn;
    double len, len2;
    int32_t row;
    int32_t pad;
};

// Filter prologue: how the per-view filter input s[v][j] is formed.
enum FilterMode : int {
    FILT_PLAIN = 0,    // s = in0
    FILT_EXTRAP = 1,   // s = in0 * (in1 - in2)        (W^-1 (mu^k - mu^{k-1}))
    FILT_DUAL_LD = 2,  // s = in0 - in1 - in2 * in3    (A x - b - W^-1 mu)
    FILT_DUAL_FV = 3,  // s = in0 - in1                (A x - b)
};

// out = e0 * E0 + e1 * E1 + c * (D s)   (E0 / E1 may be null); when Sout is
// set (with E0 and Sw), also Sout = Sw .* (out - E0): the dual update writes
// the next extrapolation's filter input W^-1 (mu^{k+1} - mu^k) this way.
struct FilterArgs {
    const float* in0;
    const float* in1;
    const float* in2;
    const float* in3;
    const float* E0;
    const float* E1;
    float e0, e1, c;
    int mode;
    float* out;
    const float* Sw;
    float* Sout;
};

// One problem of a batched solve: its geometry, its workspaces (the buffers of
// the problem's own operator handle), its inputs and step sizes.  Buffers with
// rotating roles are indexed by the launch's rotation argument: mu[rot] is
// mu^k, mu[(rot+1)%3] mu^{k-1}, mu[(rot+2)%3] receives mu^{k+1}.
struct BatchItem {
    int n, m, nb, lowdose;
    const ViewGeom* views;
    const float* taps;
    const float* b;
    const float* winv;
    float* x;
    float* z;
    float* q;        // the dual update's residual A x - b - W^-1 mu (written by the projector)
    float* sx;       // W^-1 (mu^{k+1} - mu^k) for the next extrapolation (written by the dual update)
    float* mubar;
    float* mu[3];
    float* p[2];
    float* xp;
    float* xTp;
    const int* tasks;   // the slab projector's task groups (of the problem's handle)
    float* x_out;
    float sigma, tau, lam, tvstep;
};

// One problem of the per-view lambda_h = lambda_max(W^-1/2 D W^-1/2) chains
// (float64).  W^-1/2 D W^-1/2 is block diagonal over views, so every view runs
// its own chain on its n_bins-vector.  The three Lanczos vectors (whole
// sinograms) rotate: v[rot] is q_j, v[(rot+1)%3] q_{j-1}, v[(rot+2)%3] receives
// the next one.  The scalars of view v at step j are al[j m + v] (alpha) and
// b2[j m + v] (beta_{j+1}^2); b0[v] is the start norm^2; theta[v] the view's top
// Ritz value; done[v] = steps once its chain has stopped (0 while running);
// summary = {max theta, views still running, max steps}.  A view also stops
// once fsym[0] * maxinv[v] -- an upper bound of its eigenvalue: the largest
// value of the filter's symbol times the view's largest 1/w -- is below the
// largest Ritz value of the problem (fsym null: no such pruning).
struct NormItem {
    int m, nb;
    const double* taps64;
    const double* rs;        // sqrt(1/w)
    const float* w;          // weights (start vector)
    double inv_kappa;
    double* v[3];
    double* al;
    double* b2;
    double* b0;
    double* theta;
    double* ubound;   // theta + the residual norm of the top Ritz pair (+inf before the first round)
    int* done;
    double* summary;
    const double* fsym;
    double* maxinv;
};

// One view (row) of one problem in the per-view chains.
struct RowRef {
    int prob, view;
};

// The problem and the block within it of one workgroup of a batched launch
// (prob < 0: an idle workgroup).
struct BlockRef {
    int prob, local;
};

// One launch of a recorded schedule for one problem (the unrolled passes):
// the step kernels read entry [prob] of a table of these through the block
// map of the step's map class, so one launch serves every problem of a call.
// active == 0 makes the problem skip the launch (the TV steps of a problem
// with beta = 0).  The fields each kind reads:
enum StepKind : int {
    SK_FILTER,     // out = fa (FilterArgs, mode fa.mode) with taps over m x nb
    SK_ADJOINT,    // out[0] = in[1] + c0 A^T in[0]
    SK_PAD,        // pad planes of in[0] into out[0] (x), out[1] (x^T)
    SK_FORWARD,    // out[0] = A x from the planes in[0], in[1]
    SK_TV,         // `steps` dual steps on in[1] (z = in[0]) into out[0]; out[1] (if set) = x;
                   // out[2] (if set) = every step's field; lam == 0: out[1] = max(0, z) only
    SK_BWD_FINAL,     // reverse of x = max(0, z - lam div p): in z, p, xbar; out tbar, zbar
    SK_BWD_GRADPROJ,  // reverse dual step, first half: in z, p_prev, tn; out[0] = qn (in place)
    SK_BWD_MASK,      // reverse dual step, second half: in z, p_prev, qbar; out tbar, zbar (+=)
    SK_BWD_GRAD,      // out[0] = in[0] + lam grad in[1]
    SK_LIN3,       // out[0] = (c0 in[0] + c1 in[1] + c2 in[2]) .* in[3]   (null operands skipped)
    SK_LINMIX,     // out[0] = c0 in[0] + c1 in[1] + c2 (in[2] .* in[3])
    SK_COPY,       // out[0] = in[0]
    SK_FILL,       // out[0] = c0
    SK_INV,        // out[0] = 1 / in[0]
    SK_DOT,        // part[block] = partial sums of in[0] . in[1] over reduce_blocks_for(len) blocks
    SK_FILL64,     // part[0 .. len) = 0
    SK_SLOTS,      // dout[k] = sum of part[k steps .. (k + 1) steps), k < len  (steps = the slot width)
};
struct UStep {
    int kind, active;
    int n, m, nb, steps;
    size_t len;
    float lam, step, c0, c1, c2;
    const float* in[4];
    float* out[3];
    double* part;
    double* dout;
    const ViewGeom* views;
    const float* taps;
    FilterArgs fa;
};
// Step launchers: one launch of kind `kind` over the table entries
// steps[0 .. P) (one per problem), nblocks workgroups described by map.
// max_nb sizes the filter's LDS.
hipError_t launch_step_filter(const UStep* steps, const BlockRef* map, int nblocks, int mode, int max_nb,
                              hipStream_t s);
hipError_t launch_step_projector(int kind, const UStep* steps, const BlockRef* map, int nblocks, hipStream_t s);
hipError_t launch_step_tv(int kind, const UStep* steps, const BlockRef* map, int nblocks, hipStream_t s);
hipError_t launch_step_vec(int kind, const UStep* steps, const BlockRef* map, int nblocks, hipStream_t s);

// ---- projector.hip -------------------------------------------------------
// pad pixels on each side of every row of the forward projector's planes
constexpr int kPlanePad = 3;
// xp / xTp: [n][n+6] row-major copies of x and its transpose with three zero
// pixels on each side of every row
template <typename T>
hipError_t launch_pad_planes(const T* x, T* xp, T* xTp, int n, hipStream_t s);
// y = len * sum_t interp(plane_t, s(t,u)); plane = xp for row views, xTp for column views
template <typename T>
hipError_t launch_forward(const T* xp, const T* xTp, T* y, const ViewGeom* views, int n, int m, int nb,
                          hipStream_t s);
// the dual-update residual straight from the projector: y = A x - rb - rw .* rm
// (rw null: y = A x - rb), with the arithmetic of the filter prologues
hipError_t launch_forward_resid(const float* xp, const float* xTp, float* y, const ViewGeom* views, int n, int m,
                                int nb, const float* rb, const float* rw, const float* rm, hipStream_t s);
// The same projection (and optional residual epilogue) in slab form, for one
// float32 problem: tasks holds ngroups groups of forward_slab_tasks_per_group()
// entries view * 64 + (64-bin block), each group of one orientation, -1 for
// none, the first entry of a group never -1.  The planes need 16 bytes of
// slack after their end.  Bit-identical to launch_forward / launch_forward_resid.
hipError_t launch_forward_slab(const float* xp, const float* xTp, float* y, const ViewGeom* views, const int* tasks,
                               int ngroups, int n, int nb, const float* rb, const float* rw, const float* rm,
                               hipStream_t s);
// the slab form when ngroups > 0 (tasks: its groups), else the split form (few
// views; tasks, when not null, its workgroup order from forward_split_order),
// else the gather form; all bit-identical
hipError_t launch_forward_auto(const float* xp, const float* xTp, float* y, const ViewGeom* views, const int* tasks,
                               int ngroups, int n, int m, int nb, const float* rb, const float* rw, const float* rm,
                               hipStream_t s);
bool forward_slab_fits(int n);
int forward_slab_tasks_per_group();
// The slab form's task groups for a geometry (host): every (view, 64-bin
// block) once, in max(min_groups, the fewest groups that hold them) groups
// (fewer when there are too few tasks to fill them), each group of one
// orientation and balanced over its SIMDs slab by slab; *dense (may be null)
// receives the fewest groups that hold them.
std::vector<int> forward_slab_schedule(const ViewGeom* hv, int m, int n, int nb, int min_groups, int* dense);
// whether a single solve should use the slab form (enough groups at their
// fullest to fill most of the chip, and a slab that fits the LDS)
bool forward_slab_preferred(int dense_groups, int n);
// the split form's workgroup order for a geometry (host): every view * nblk +
// block once, heaviest first
std::vector<int> forward_split_order(const ViewGeom* hv, int m, int n, int nb);
// floats of slack after each padded plane (the slab form copies 16-byte words)
constexpr size_t kPlaneSlack = 4;
// out = alpha * xin + beta * A^T (c1 * y1 + c2 * y2)   (xin, y2 may be null)
template <typename T>
hipError_t launch_adjoint(const T* y1, const T* y2, T c1, T c2, const T* xin, T alpha, T beta, T* out,
                          const ViewGeom* views, int n, int m, int nb, hipStream_t s);

// batched forms (grids of nblocks workgroups described by map):
//   pad planes of x, q = A x, z = x - tau A^T mubar (two: z = x - tau A^T (2 mu^k - mu^{k-1}))
hipError_t launch_pad_planes_batched(const BatchItem* items, const BlockRef* map, int nblocks, hipStream_t s);
// form: 0 the slab form (map entries (problem, task group); every problem's
// n must fit forward_slab_fits, max_n the largest), 1 the gather form (map
// entries (problem, forward_blocks_x(nb) * view + block)) -- a tuning choice
// of the batch; both give the single solve's bits.  The batch's projector
// writes the residual A x - b - W^-1 mu[rot] into q.
hipError_t launch_forward_batched(const BatchItem* items, const BlockRef* map, int nblocks, int form, int max_n,
                                  int rot, hipStream_t s);
hipError_t launch_adjoint_batched(const BatchItem* items, const BlockRef* map, int nblocks, bool two, int rot,
                                  hipStream_t s);

int adjoint_tiles(int n);       // A^T tiles per image side
int pad_tiles(int n);           // pad-plane tiles per image side
int forward_blocks_x(int nb);   // forward-projector workgroups per view

// ---- filter.hip ----------------------------------------------------------
// taps64[k], k = 0..2nb-2, for offset k - (nb-1); also written rounded to taps32.
// d_tau: the taps of dH/dtau instead of H (the filter's derivative in tau).
hipError_t launch_taps(double* taps64, float* taps32, int nb, int m, double tau, double kappa,
                       hipStream_t s, bool d_tau = false);
hipError_t launch_filter_f32(const FilterArgs& a, const float* taps32, int m, int nb, hipStream_t s);
// out = scale_in * D (scale_in .* in), elementwise scale optional (null = 1), then
// out *= scale_out (optional)
hipError_t launch_filter_f64(const double* in, double* out, const double* taps64, const double* pre,
                             const double* post, int m, int nb, hipStream_t s);

// batched filter for the solver's two uses of D (mode FILT_PLAIN: k = 0
// extrapolation; FILT_EXTRAP; FILT_DUAL_LD / FILT_DUAL_FV: dual update)
hipError_t launch_filter_batched(const BatchItem* items, const BlockRef* map, int nblocks, int mode, int rot,
                                 int max_nb, hipStream_t s);
int filter_blocks_x(int nb);
int filter_blocks_y(int m);
// float64 (norm) filter work decomposition
int norm_blocks_x(int nb);
int norm_blocks_y(int m);

// batched W^-1/2 D W^-1/2 applied to v[rot] into v[(rot+2)%3] (float64)
hipError_t launch_norm_filter_batched(const NormItem* it, const BlockRef* map, int nblocks, int rot,
                                      hipStream_t s);

// ---- tv.hip --------------------------------------------------------------
// The TV prox: n_iter dual steps on p starting from p_a (warm start), then
// x = max(0, z - lam div p).  lam > 0.  p_a and p_b are both overwritten as
// ping-pong buffers; *p_final receives the one holding the final p.  With xp
// and xTp the padded planes of x that the forward projector reads (see
// launch_pad_planes; their pad columns must already be zero) are written too.
hipError_t launch_tv_prox(const float* z, float* p_a, float* p_b, float* x, int n, float lam, float step,
                          int n_iter, float** p_final, hipStream_t s, float* xp = nullptr, float* xTp = nullptr);
// p <- projection of (p + s grad xb) onto the unit ball, pointwise (the dual
// step of Chambolle-Pock on the TV term).
hipError_t launch_grad_ball(const float* xb, float* p, int n, float s, hipStream_t st);
// batched TV prox chunk (p[src] -> p[1-src]; x written when last); threads
// per 32 x 32 tile: 512 or 1024, a tuning choice of the batch
hipError_t launch_tv_prox_batched(const BatchItem* items, const BlockRef* map, int nblocks, int src, int steps,
                                  bool last, int threads, hipStream_t s);
int tv_tiles(int n);      // TV tiles per image side
int tv_chunk_max();       // dual steps per TV launch at most
// Reverse pass of the prox: one workgroup per 64 x 4 pixels, tv_bwd_blocks(n)
// per image (each writes one block sum of its scalar-adjoint term).
int tv_bwd_blocks(int n);
hipError_t launch_tv_finalize(const float* z, const float* p, float* x, int n, float lam, hipStream_t s);

// ---- vec.hip -------------------------------------------------------------
// Deterministic float64 reductions: partial sums per block, then one block.
enum ReduceOp : int {
    RED_DOT_F64 = 0,       // sum a[i]*b[i]                    (double inputs)
    RED_INVW_CHECK = 1,    // sum 1/w[i]; counts w<=0 / non-finite w or b   (float)
    RED_ABS_F32 = 2,       // sum |a[i]|                        (float)
    RED_WRES_F32 = 3,      // sum w*(q-b)^2                     (float)
    RED_SQDIFF_F32 = 4,    // sum (q-b)^2                       (float)
    RED_SQ_F32 = 5,        // sum b^2                           (float)
    RED_DOT_F32 = 6,       // sum a[i]*b[i]                    (float)
    RED_SUM_F32 = 7,       // sum a[i]                          (float)
    RED_GAP_F32 = 8,       // sum (c (a - b) - d)^2 / c         (float; a = A x, b, c = w, d = mu)
    RED_ABS_F64 = 9,       // sum |a[i]|                        (double)
};
// Result (3 doubles: value, count1, count2) written to dev_out[0..2].
hipError_t launch_reduce(int op, const void* a, const void* b, const void* c, size_t len,
                         double* partials, double* dev_out, hipStream_t s, const void* d = nullptr);
// TV norm of x [n][n] (float), float64 sum, into dev_out[0].
hipError_t launch_tv_norm(const float* x, int n, double* partials, double* dev_out, hipStream_t s);
constexpr int kReduceBlocks = 512;

// Lanczos start vector over [rows][cols]: image bump (w null) or the sinogram
// pattern (-1)^col / (w kappa), plus counter-based noise.
hipError_t launch_start_vector(double* v, int rows, int cols, uint64_t seed, const float* w, double inv_kappa,
                               hipStream_t s);
// w <- w - alpha[0] q - sqrt(beta2[0]) qp, and beta2_out[0] = ||w||^2 (device scalars)
hipError_t launch_lanczos_update(double* w, const double* q, const double* qp, const double* alpha,
                                 const double* beta2, size_t len, double* partials, double* beta2_out,
                                 hipStream_t s);
// y = x / sqrt(sumsq[0])
hipError_t launch_normalize(double* y, const double* x, const double* sumsq, size_t len, hipStream_t s);
// y = a*x + b*y + c*z (double; z may be null)
hipError_t launch_axpby_f64(double* y, const double* x, double a, double b, const double* z, double c,
                            size_t len, hipStream_t s);
// y = a*x (double)
hipError_t launch_scale_f64(double* y, const double* x, double a, size_t len, hipStream_t s);
// out = (c0 a + c1 b + c2 c) .* w   (b, c, w may be null; out may alias a, b or c)
hipError_t launch_lin3_f32(float* out, const float* a, float c0, const float* b, float c1, const float* c, float c2,
                           const float* w, size_t len, hipStream_t s);
hipError_t launch_mul_w_f64(double* out, const double* a, const float* w, size_t len, hipStream_t s);
// out = (double) a
// Projection onto the data ball {y : ||y - b|| <= eps}: v = y + tau (c1 m1 + c2 m2)
// (m2 may be null), ball_out[0] = ||v - b||, ball_out[1] = min(1, eps / ||v - b||)
// (float64, on the device), then y = b + (v - b) ball_out[1] in place.
hipError_t launch_ball_project(float* y, const float* m1, float c1, const float* m2, float c2, float tau,
                               const float* b, double eps, size_t len, double* partials, double* ball_out,
                               hipStream_t s);
hipError_t launch_widen_f64(double* out, const float* a, size_t len, hipStream_t s);
// batched solve: zero x, p[0], mu[0], mu[1] of every problem / copy x to x_out
// (2048 elements per workgroup)
hipError_t launch_batch_init(const BatchItem* items, const BlockRef* map, int nblocks, hipStream_t s);
hipError_t launch_batch_copy_out(const BatchItem* items, const BlockRef* map, int nblocks, hipStream_t s);
// z = -sigma z per problem (the copy-out map), the first iteration's last step
hipError_t launch_batch_scale_z(const BatchItem* items, const BlockRef* map, int nblocks, hipStream_t s);
// per-view lambda_h chains over the rows of a NormItem table (one wave per row)
hipError_t launch_rows_start(const NormItem* it, const RowRef* rows, int nrows, uint64_t seed, hipStream_t s);
// before the first round: a windowed Rayleigh-quotient lower bound per view
// (theta), then the summary's symbol-bound pruning against the largest of them
// (count = problems of the table; a view stopped here records 1 step)
hipError_t launch_rows_prune(const NormItem* it, const RowRef* rows, int nrows, int count, hipStream_t s);
hipError_t launch_rows_step(const NormItem* it, const RowRef* rows, int nrows, int rot, int j, hipStream_t s);
// steps j0 .. j1-1 of every running chain in one launch (q in v[0], previous q
// in v[1] on entry and exit), each chain's Ritz step after them (as
// launch_rows_ritz: the same arithmetic) and the summary (count = problems);
// only when rows_round_fits(the largest nb of the table), which holds up to
// 1024 bins
bool rows_round_fits(int max_nb);
hipError_t launch_rows_round(const NormItem* it, const RowRef* rows, int nrows, int count, int j0, int j1,
                             int max_nb, double tol, hipStream_t s);
// upper bound of max over omega of h0 + 2 sum_k h_k cos(k omega) (taps64 as
// launch_taps writes them) into out[0]; out[1 ..] is scratch (kSymBlocks doubles)
constexpr int kSymBlocks = 64;
hipError_t launch_symbol_max(const double* taps64, int nb, double* out, hipStream_t s);
// taps64 = taps1 / kappa (and taps32 = float of it); sym_out[0] = sym1[0] / kappa when sym_out is set
hipError_t launch_taps_scale(const double* taps1, int ntap, double kappa, double* taps64, float* taps32,
                             const double* sym1, double* sym_out, hipStream_t s);
hipError_t launch_rows_ritz(const NormItem* it, const RowRef* rows, int nrows, int count, int steps, double tol,
                            hipStream_t s);
// workgroups of a float64 reduction over len elements
int reduce_blocks_for(size_t len);
// out[i] = 1/w[i] (float) or sqrt(1/w[i]) (double), computed in float64
hipError_t launch_inverse_f32(float* out, const float* w, size_t len, hipStream_t s);
// dev_out[0] = max of 1/w (float64); partials: reduce_blocks_for(len) doubles
hipError_t launch_max_inv(const float* w, size_t len, double* partials, double* dev_out, hipStream_t s);
// the taps of the identity (D = I): 1 at offset 0
hipError_t launch_identity_taps(double* taps64, float* taps32, int nb, hipStream_t s);
hipError_t launch_rsqrt_f64(double* out, const float* w, size_t len, hipStream_t s);
hipError_t launch_copy_f32(float* dst, const float* src, size_t len, hipStream_t s);
hipError_t launch_fill_f32(float* dst, float v, size_t len, hipStream_t s);
// a[0..na) = b[0..nb) = c[0..nc) = d[0..nd) = 0 in one launch
hipError_t launch_zero4_f32(float* a, size_t na, float* b, size_t nb, float* c, size_t nc, float* d, size_t nd,
                            hipStream_t s);

}  // namespace ctpd
