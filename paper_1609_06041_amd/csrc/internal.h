// Internal declarations shared by the HIP translation units of libctpd.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ctpd.h"

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

// out = e0 * E0 + e1 * E1 + c * (D s)   (E0 / E1 may be null)
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
};

// ---- projector.hip -------------------------------------------------------
// xp / xTp: [n][n+6] row-major copies of x and its transpose with three zero
// pixels on each side of every row
template <typename T>
hipError_t launch_pad_planes(const T* x, T* xp, T* xTp, int n, hipStream_t s);
// y = len * sum_t interp(plane_t, s(t,u)); plane = xp for row views, xTp for column views
template <typename T>
hipError_t launch_forward(const T* xp, const T* xTp, T* y, const ViewGeom* views, int n, int m, int nb,
                          hipStream_t s);
// out = alpha * xin + beta * A^T (c1 * y1 + c2 * y2)   (xin, y2 may be null)
template <typename T>
hipError_t launch_adjoint(const T* y1, const T* y2, T c1, T c2, const T* xin, T alpha, T beta, T* out,
                          const ViewGeom* views, int n, int m, int nb, hipStream_t s);

// ---- filter.hip ----------------------------------------------------------
// taps64[k], k = 0..2nb-2, for offset k - (nb-1); also written rounded to taps32.
hipError_t launch_taps(double* taps64, float* taps32, int nb, int m, double tau, double kappa,
                       hipStream_t s);
hipError_t launch_filter_f32(const FilterArgs& a, const float* taps32, int m, int nb, hipStream_t s);
// out = scale_in * D (scale_in .* in), elementwise scale optional (null = 1), then
// out *= scale_out (optional)
hipError_t launch_filter_f64(const double* in, double* out, const double* taps64, const double* pre,
                             const double* post, int m, int nb, hipStream_t s);

// ---- tv.hip --------------------------------------------------------------
hipError_t launch_tv_step(const float* z, const float* p_in, float* p_out, int n, float lam, float step,
                          hipStream_t s);
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
};
// Result (3 doubles: value, count1, count2) written to dev_out[0..2].
hipError_t launch_reduce(int op, const void* a, const void* b, const void* c, size_t len,
                         double* partials, double* dev_out, hipStream_t s);
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
// out[i] = f(x[i]): inverse (1/x) or sqrt(1/x)   (float in, float / double out)
hipError_t launch_inverse_f32(float* out, const float* w, size_t len, hipStream_t s);
hipError_t launch_rsqrt_f64(double* out, const float* w, size_t len, hipStream_t s);
hipError_t launch_copy_f32(float* dst, const float* src, size_t len, hipStream_t s);
hipError_t launch_fill_f32(float* dst, float v, size_t len, hipStream_t s);

}  // namespace ctpd
