// Vector utilities: deterministic float64 reductions (wave shuffles, then the
// block, then one final block in fixed order), the counter-based start
// vector of the norm computation, and small elementwise kernels.
#include "internal.h"

namespace ctpd {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sum of three per-thread values over the 256-thread block; result valid in thread 0.
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c) {
    __shared__ double red[3][4];
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = a;
        red[1][w] = b;
        red[2][w] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        b = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        c = (red[2][0] + red[2][1]) + (red[2][2] + red[2][3]);
    }
}

template <int OP>
__global__ __launch_bounds__(256) void reduce_partial_kernel(const void* __restrict__ pa, const void* __restrict__ pb,
                                                             const void* __restrict__ pc, size_t len,
                                                             double* __restrict__ partials,
                                                             const void* __restrict__ pd = nullptr) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < len; i += stride) {
        if constexpr (OP == RED_DOT_F64) {
            s0 = fma(((const double*)pa)[i], ((const double*)pb)[i], s0);
        } else if constexpr (OP == RED_INVW_CHECK) {
            const float w = ((const float*)pa)[i];
            if (w > 0.0f && isfinite(w)) s0 += 1.0 / (double)w;
            else s1 += 1.0;
            if (pb && !isfinite(((const float*)pb)[i])) s2 += 1.0;
        } else if constexpr (OP == RED_ABS_F32) {
            s0 += fabs((double)((const float*)pa)[i]);
        } else if constexpr (OP == RED_ABS_F64) {
            s0 += fabs(((const double*)pa)[i]);
        } else if constexpr (OP == RED_WRES_F32) {
            const double r = (double)((const float*)pa)[i] - (double)((const float*)pb)[i];
            s0 = fma((double)((const float*)pc)[i] * r, r, s0);
        } else if constexpr (OP == RED_SQDIFF_F32) {
            const double r = (double)((const float*)pa)[i] - (double)((const float*)pb)[i];
            s0 = fma(r, r, s0);
        } else if constexpr (OP == RED_DOT_F32) {
            s0 = fma((double)((const float*)pa)[i], (double)((const float*)pb)[i], s0);
        } else if constexpr (OP == RED_SUM_F32) {
            s0 += (double)((const float*)pa)[i];
        } else if constexpr (OP == RED_GAP_F32) {
            // (w r - mu)^2 / w = (W^1/2 r - W^-1/2 mu)^2 with r = A x - b
            const double w = (double)((const float*)pc)[i];
            const double d = w * ((double)((const float*)pa)[i] - (double)((const float*)pb)[i]) -
                             (double)((const float*)pd)[i];
            s0 += d * d / w;
        } else {   // RED_SQ_F32, counting non-finite entries
            const float v = ((const float*)pa)[i];
            if (isfinite(v)) s0 = fma((double)v, (double)v, s0);
            else s1 += 1.0;
        }
    }
    block_sum3(s0, s1, s2);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x + 0] = s0;
        partials[3 * blockIdx.x + 1] = s1;
        partials[3 * blockIdx.x + 2] = s2;
    }
}

__global__ __launch_bounds__(256) void reduce_final_kernel(const double* __restrict__ partials, int nblocks,
                                                           double* __restrict__ out) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) {
        s0 += partials[3 * b + 0];
        s1 += partials[3 * b + 1];
        s2 += partials[3 * b + 2];
    }
    block_sum3(s0, s1, s2);
    if (threadIdx.x == 0) {
        out[0] = s0;
        out[1] = s1;
        out[2] = s2;
    }
}

__host__ __device__ static inline int reduce_blocks(size_t len) {
    const size_t b = (len + 255) / 256;
    return (int)(b < (size_t)kReduceBlocks ? (b ? b : 1) : kReduceBlocks);
}

hipError_t launch_reduce(int op, const void* a, const void* b, const void* c, size_t len, double* partials,
                         double* dev_out, hipStream_t s, const void* d) {
    const int nb = reduce_blocks(len);
    switch (op) {
        case RED_GAP_F32:
            reduce_partial_kernel<RED_GAP_F32><<<nb, 256, 0, s>>>(a, b, c, len, partials, d);
            break;
        case RED_DOT_F64: reduce_partial_kernel<RED_DOT_F64><<<nb, 256, 0, s>>>(a, b, c, len, partials); break;
        case RED_INVW_CHECK: reduce_partial_kernel<RED_INVW_CHECK><<<nb, 256, 0, s>>>(a, b, c, len, partials); break;
        case RED_ABS_F32: reduce_partial_kernel<RED_ABS_F32><<<nb, 256, 0, s>>>(a, b, c, len, partials); break;
        case RED_ABS_F64: reduce_partial_kernel<RED_ABS_F64><<<nb, 256, 0, s>>>(a, b, c, len, partials); break;
        case RED_WRES_F32: reduce_partial_kernel<RED_WRES_F32><<<nb, 256, 0, s>>>(a, b, c, len, partials); break;
        case RED_SQDIFF_F32: reduce_partial_kernel<RED_SQDIFF_F32><<<nb, 256, 0, s>>>(a, b, c, len, partials); break;
        case RED_DOT_F32: reduce_partial_kernel<RED_DOT_F32><<<nb, 256, 0, s>>>(a, b, c, len, partials); break;
        case RED_SUM_F32: reduce_partial_kernel<RED_SUM_F32><<<nb, 256, 0, s>>>(a, b, c, len, partials); break;
        default: reduce_partial_kernel<RED_SQ_F32><<<nb, 256, 0, s>>>(a, b, c, len, partials); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    reduce_final_kernel<<<1, 256, 0, s>>>(partials, nb, dev_out);
    return hipGetLastError();
}

// Projection onto the data ball {y : ||y - b|| <= eps} of the error-tolerant
// few-view problem: v = y + tau mubar with mubar = c1 m1 + c2 m2 (m2 may be
// null), then y = b + (v - b) min(1, eps / ||v - b||).  Both passes form
// d = v - b with the same explicit fma, so the norm is that of the d the
// update scales; the norm and the scale are float64 and stay on the device.
__device__ __forceinline__ float ball_d(const float* __restrict__ y, const float* __restrict__ m1, float c1,
                                        const float* __restrict__ m2, float c2, float tau,
                                        const float* __restrict__ b, size_t i) {
    const float mb = m2 ? fmaf(c2, m2[i], c1 * m1[i]) : c1 * m1[i];
    return fmaf(tau, mb, y[i]) - b[i];
}

__global__ __launch_bounds__(256) void ball_partial_kernel(const float* __restrict__ y, const float* __restrict__ m1,
                                                           float c1, const float* __restrict__ m2, float c2,
                                                           float tau, const float* __restrict__ b, size_t len,
                                                           double* __restrict__ partials) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < len; i += stride) {
        const double d = ball_d(y, m1, c1, m2, c2, tau, b, i);
        s0 = fma(d, d, s0);
    }
    block_sum3(s0, s1, s2);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x + 0] = s0;
        partials[3 * blockIdx.x + 1] = 0.0;
        partials[3 * blockIdx.x + 2] = 0.0;
    }
}

// out[0] = ||v - b||, out[1] = min(1, eps / ||v - b||) (1 when v lies in the ball)
__global__ __launch_bounds__(256) void ball_scale_kernel(const double* __restrict__ partials, int nblocks, double eps,
                                                         double* __restrict__ out) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) s0 += partials[3 * b];
    block_sum3(s0, s1, s2);
    if (threadIdx.x == 0) {
        const double r = sqrt(s0);
        out[0] = r;
        out[1] = r <= eps ? 1.0 : eps / r;
    }
}

__global__ __launch_bounds__(256) void ball_apply_kernel(float* __restrict__ y, const float* __restrict__ m1, float c1,
                                                         const float* __restrict__ m2, float c2, float tau,
                                                         const float* __restrict__ b, const double* __restrict__ sc,
                                                         size_t len) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= len) return;
    const float scale = (float)sc[1];
    const float d = ball_d(y, m1, c1, m2, c2, tau, b, i);
    y[i] = fmaf(d, scale, b[i]);
}

hipError_t launch_ball_project(float* y, const float* m1, float c1, const float* m2, float c2, float tau,
                               const float* b, double eps, size_t len, double* partials, double* ball_out,
                               hipStream_t s) {
    const int nb = reduce_blocks(len);
    ball_partial_kernel<<<nb, 256, 0, s>>>(y, m1, c1, m2, c2, tau, b, len, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ball_scale_kernel<<<1, 256, 0, s>>>(partials, nb, eps, ball_out);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    ball_apply_kernel<<<(unsigned)((len + 255) / 256), 256, 0, s>>>(y, m1, c1, m2, c2, tau, b, ball_out, len);
    return hipGetLastError();
}

// TV norm (Eq. 2) of a float32 image in float64.
__global__ __launch_bounds__(256) void tv_norm_partial_kernel(const float* __restrict__ x, int n,
                                                              double* __restrict__ partials) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    const size_t len = (size_t)n * n, stride = (size_t)gridDim.x * 256;
    for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < len; idx += stride) {
        const int i = (int)(idx / n), j = (int)(idx - (size_t)i * n);
        const double xc = x[idx];
        const double g1 = (j < n - 1) ? (double)x[idx + 1] - xc : 0.0;
        const double g2 = (i < n - 1) ? (double)x[idx + n] - xc : 0.0;
        s0 += sqrt(g1 * g1 + g2 * g2);
    }
    block_sum3(s0, s1, s2);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x + 0] = s0;
        partials[3 * blockIdx.x + 1] = 0.0;
        partials[3 * blockIdx.x + 2] = 0.0;
    }
}

hipError_t launch_tv_norm(const float* x, int n, double* partials, double* dev_out, hipStream_t s) {
    const int nb = reduce_blocks((size_t)n * n);
    tv_norm_partial_kernel<<<nb, 256, 0, s>>>(x, n, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    reduce_final_kernel<<<1, 256, 0, s>>>(partials, nb, dev_out);
    return hipGetLastError();
}

// SplitMix64 (Steele, Lea, Flood 2014) as a counter-based generator.
__device__ __forceinline__ double splitmix_unit(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53;   // [0, 1)
}

// Lanczos start vectors: a shape close to the expected top eigenvector plus
// 5% counter-based noise (so no eigenvector is missed).
//   image space (n x n): Gaussian bump of width n/4 at the centre -- the
//     ramp-preconditioned A^T D A has its largest eigenvalues at the lowest
//     spatial frequencies;
//   sinogram space ([rows][cols], weights w): (-1)^u / (w kappa) -- the filter
//     response peaks at the Nyquist frequency and W^-1 favours low counts.
__global__ __launch_bounds__(256) void start_vector_kernel(double* __restrict__ v, int rows, int cols, uint64_t seed,
                                                           const float* __restrict__ w, double inv_kappa) {
    const size_t len = (size_t)rows * cols;
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= len) return;
    const int r = (int)(i / cols), c = (int)(i - (size_t)r * cols);
    double shape;
    if (w) {
        shape = ((c & 1) ? -1.0 : 1.0) * inv_kappa / (double)w[i];
    } else {
        const double h = 0.5 * (cols - 1), s = 0.25 * cols;
        const double dx = c - h, dy = r - h;
        shape = exp(-(dx * dx + dy * dy) / (2.0 * s * s));
    }
    v[i] = shape + 0.05 * (splitmix_unit(seed, i) - 0.5);
}

hipError_t launch_start_vector(double* v, int rows, int cols, uint64_t seed, const float* w, double inv_kappa,
                               hipStream_t s) {
    const size_t len = (size_t)rows * cols;
    start_vector_kernel<<<(unsigned)((len + 255) / 256), 256, 0, s>>>(v, rows, cols, seed, w, inv_kappa);
    return hipGetLastError();
}

// One Lanczos orthogonalisation with device-resident scalars:
//   w <- w - alpha q - beta qp,  beta = sqrt(beta2[0]) (qp, beta2 may be null),
// with block partial sums of w'^2 for the next beta.
__global__ __launch_bounds__(256) void lanczos_update_kernel(double* __restrict__ w, const double* __restrict__ q,
                                                             const double* __restrict__ qp,
                                                             const double* __restrict__ alpha,
                                                             const double* __restrict__ beta2, size_t len,
                                                             double* __restrict__ partials) {
    const double a = alpha[0];
    const double b = (qp && beta2) ? sqrt(beta2[0]) : 0.0;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < len; i += stride) {
        double r = w[i] - a * q[i];
        if (qp) r -= b * qp[i];
        w[i] = r;
        s0 = fma(r, r, s0);
    }
    block_sum3(s0, s1, s2);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x + 0] = s0;
        partials[3 * blockIdx.x + 1] = 0.0;
        partials[3 * blockIdx.x + 2] = 0.0;
    }
}

hipError_t launch_lanczos_update(double* w, const double* q, const double* qp, const double* alpha,
                                 const double* beta2, size_t len, double* partials, double* beta2_out,
                                 hipStream_t s) {
    const int nb = reduce_blocks(len);
    lanczos_update_kernel<<<nb, 256, 0, s>>>(w, q, qp, alpha, beta2, len, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    reduce_final_kernel<<<1, 256, 0, s>>>(partials, nb, beta2_out);
    return hipGetLastError();
}

// y = x / sqrt(sumsq[0])
__global__ __launch_bounds__(256) void normalize_kernel(double* __restrict__ y, const double* __restrict__ x,
                                                        const double* __restrict__ sumsq, size_t len) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < len) y[i] = x[i] / sqrt(sumsq[0]);
}

hipError_t launch_normalize(double* y, const double* x, const double* sumsq, size_t len, hipStream_t s) {
    normalize_kernel<<<(unsigned)((len + 255) / 256), 256, 0, s>>>(y, x, sumsq, len);
    return hipGetLastError();
}

// out = (c0 a + c1 b + c2 c) .* w   (b, c, w may be null; out may alias a, b or c)
__global__ __launch_bounds__(256) void lin3_kernel(float* out, const float* a, float c0, const float* b, float c1,
                                                   const float* c, float c2, const float* __restrict__ w,
                                                   size_t len) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= len) return;
    float r = c0 * a[i];
    if (b) r = fmaf(c1, b[i], r);
    if (c) r = fmaf(c2, c[i], r);
    if (w) r *= w[i];
    out[i] = r;
}

hipError_t launch_lin3_f32(float* out, const float* a, float c0, const float* b, float c1, const float* c, float c2,
                           const float* w, size_t len, hipStream_t s) {
    lin3_kernel<<<(unsigned)((len + 255) / 256), 256, 0, s>>>(out, a, c0, b, c1, c, c2, w, len);
    return hipGetLastError();
}

int reduce_blocks_for(size_t len) { return reduce_blocks(len); }

// out = a .* w with float weights (float64 operator applications)
__global__ __launch_bounds__(256) void mul_w_kernel(double* __restrict__ out, const double* __restrict__ a,
                                                    const float* __restrict__ w, size_t len) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < len) out[i] = a[i] * (double)w[i];
}

hipError_t launch_mul_w_f64(double* out, const double* a, const float* w, size_t len, hipStream_t s) {
    mul_w_kernel<<<(unsigned)((len + 255) / 256), 256, 0, s>>>(out, a, w, len);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void widen_kernel(double* __restrict__ out, const float* __restrict__ a, size_t len) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < len) out[i] = (double)a[i];
}

hipError_t launch_widen_f64(double* out, const float* a, size_t len, hipStream_t s) {
    widen_kernel<<<(unsigned)((len + 255) / 256), 256, 0, s>>>(out, a, len);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-view Lanczos chains for lambda_max(W^-1/2 D W^-1/2).  D acts on every
// view (row) separately and W is diagonal, so the operator is block diagonal
// and its largest eigenvalue is the largest over views: every view runs its
// own chain on its nb-vector, all views (of all problems of a table) in
// lockstep.  One workgroup per row for the Lanczos step (fixed-order
// reductions) and for the Ritz values (Sturm-sequence multisection on the
// view's tridiagonal matrix over four waves, scalars staged in LDS).  A
// stopped view's vectors are left untouched.
__device__ __forceinline__ double wave_sum_all(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

#define ROW_PROLOGUE                                                   \
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);               \
    const int lane = threadIdx.x & 63;                                 \
    if (row >= nrows) return;                                          \
    const RowRef rr = rows[row];                                       \
    const NormItem& it = items[rr.prob];                               \
    const int m = it.m, nb = it.nb, v = rr.view;                       \
    const size_t base = (size_t)v * nb;

__global__ __launch_bounds__(256) void rows_start_kernel(const NormItem* __restrict__ items,
                                                         const RowRef* __restrict__ rows, int nrows,
                                                         uint64_t seed) {
    ROW_PROLOGUE
    double* q = it.v[0] + base;
    double ss = 0.0, mi = 0.0;
    for (int u = lane; u < nb; u += 64) {
        const size_t i = base + u;
        const double iw = 1.0 / (double)it.w[i];
        const double shape = ((u & 1) ? -1.0 : 1.0) * it.inv_kappa * iw;
        const double val = shape + 0.05 * (splitmix_unit(seed, i) - 0.5);
        q[u] = val;
        ss = fma(val, val, ss);
        mi = fmax(mi, iw);
    }
    for (int off = 32; off > 0; off >>= 1) mi = fmax(mi, __shfl_xor(mi, off));
    ss = wave_sum_all(ss);
    const double inv = 1.0 / sqrt(ss);
    for (int u = lane; u < nb; u += 64) q[u] *= inv;
    if (lane == 0) {
        it.b0[v] = ss;
        it.done[v] = 0;
        it.theta[v] = 0.0;
        it.ubound[v] = HUGE_VAL;
        it.maxinv[v] = mi;
    }
    (void)m;
}

// A lower bound of each view's eigenvalue before any Lanczos step: the
// Rayleigh quotient of W_v^-1/2 D W_v^-1/2 at a vector supported on the
// kLowerWin bins around the view's largest 1/w, alternating in sign under a
// sine taper (close to the top eigenvector of a short section of the
// ramp-like Toeplitz D).  Any vector gives a valid bound; this one lands
// within a fraction of a percent of the largest view's eigenvalue on low-dose
// data, so the symbol bound can stop most views before the first round.  The
// value goes to theta[v] (each chain's running lower estimate).
constexpr int kLowerWin = 16;

__global__ __launch_bounds__(256) void rows_lower_kernel(const NormItem* __restrict__ items,
                                                         const RowRef* __restrict__ rows, int nrows) {
    ROW_PROLOGUE
    // the first bin of the largest 1/w (= smallest w)
    float wmin = 3.0e38f;
    int imin = nb;
    for (int u = lane; u < nb; u += 64) {
        const float wu = it.w[base + u];
        if (wu < wmin || (wu == wmin && u < imin)) {
            wmin = wu;
            imin = u;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const float wo = __shfl_xor(wmin, off);
        const int io = __shfl_xor(imin, off);
        if (wo < wmin || (wo == wmin && io < imin)) {
            wmin = wo;
            imin = io;
        }
    }
    const int W = min(kLowerWin, nb);
    const int lo = min(max(imin - W / 2 + 1, 0), nb - W);
    const double* h = it.taps64 + (nb - 1);
    const double* rs = it.rs + base + lo;
    double num = 0.0, den = 0.0;
    for (int e = lane; e < W * W; e += 64) {
        const int a = e / W, b = e - a * W;
        const double ua = ((a & 1) ? -1.0 : 1.0) * sin(M_PI * (a + 1) / (W + 1));
        const double ub = ((b & 1) ? -1.0 : 1.0) * sin(M_PI * (b + 1) / (W + 1));
        num = fma(ua * rs[a], h[a > b ? a - b : b - a] * (ub * rs[b]), num);
        if (a == b) den = fma(ua, ua, den);
    }
    num = wave_sum_all(num);
    den = wave_sum_all(den);
    if (lane == 0) it.theta[v] = num / den;
    (void)m;
}

// Sum over the 256-thread block, returned to every thread (fixed order).
__device__ __forceinline__ double block_allsum(double v, double* red4) {
    v = wave_sum_all(v);
    __syncthreads();   // red4 free from any previous use
    if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red4[0] + red4[1]) + (red4[2] + red4[3]);
}

// Step j after the filter has put M q into w (one workgroup per view):
// alpha = q.w;  w <- w - alpha q - beta qp;  beta'^2 = |w|^2;  w <- w / beta'.
__global__ __launch_bounds__(256) void rows_step_kernel(const NormItem* __restrict__ items,
                                                        const RowRef* __restrict__ rows, int nrows, int rot, int j) {
    __shared__ double red4[4];
    const int row = blockIdx.x;
    if (row >= nrows) return;
    const RowRef rr = rows[row];
    const NormItem& it = items[rr.prob];
    const int m = it.m, nb = it.nb, v = rr.view;
    if (it.done[v]) return;
    const size_t base = (size_t)v * nb;
    const double* q = it.v[rot] + base;
    const double* qp = it.v[(rot + 1) % 3] + base;
    double* w = it.v[(rot + 2) % 3] + base;
    double a = 0.0;
    for (int u = threadIdx.x; u < nb; u += 256) a = fma(q[u], w[u], a);
    a = block_allsum(a, red4);
    const double b = j ? sqrt(it.b2[(size_t)(j - 1) * m + v]) : 0.0;
    double ss = 0.0;
    for (int u = threadIdx.x; u < nb; u += 256) {
        double r = w[u] - a * q[u];
        if (j) r -= b * qp[u];
        w[u] = r;
        ss = fma(r, r, ss);
    }
    ss = block_allsum(ss, red4);
    if (ss > 0.0) {
        const double inv = 1.0 / sqrt(ss);
        for (int u = threadIdx.x; u < nb; u += 256) w[u] *= inv;
    }
    if (threadIdx.x == 0) {
        it.al[(size_t)j * m + v] = a;
        it.b2[(size_t)j * m + v] = ss;
    }
}

// A round of steps j0 .. j1-1 of every running view's chain in one launch,
// one 512-thread workgroup per view (nb <= kRoundMaxBins).  The view's
// operator S D S (S = W^-1/2 on the view's bins, D the nb x nb Toeplitz
// section) is applied as a dense product in float64: the mirrored taps,
// zero-extended, and u = S q sit in LDS; the eight waves split the bins k, and
// lane l accumulates the 12 consecutive outputs 12 l .. 12 l + 11 of a
// 768-output chunk, holding the 12 taps h[i - k] those outputs need in
// registers.  Going from k to k + 1 moves that window by one tap, so each k
// costs one tap read, one broadcast read of u_k and 12 FMAs.  The taps are
// stored with one unused double after every 12, which turns the lanes' stride
// of 12 doubles into 13, a stride the LDS banks serve without conflicts.  The
// wave partials are added in a fixed order (w and w + 4, then the four sums).
// The recurrence is the per-step kernel's: alpha = q.Mq, w = Mq - alpha q -
// beta qp, beta'^2 = |w|^2, q <- w / beta', with al and b2 written per step
// for the Ritz kernel.  On entry q is in v[0] and the previous q in v[1] (not
// read when j0 = 0); on exit likewise.
constexpr int kRoundWaves = 8, kRoundThreads = 64 * kRoundWaves, kRoundR = 12, kRoundChunk = 64 * kRoundR;
constexpr int kRoundMaxBins = 1024, kRoundNpt = kRoundMaxBins / kRoundThreads;

struct RoundDims {
    int Q;      // bins k per wave (a multiple of kRoundR)
    int KP;     // kRoundWaves * Q >= nb: k beyond nb meets u = 0
    int OUTP;   // outputs, a multiple of kRoundChunk
    int TP;     // LDS doubles of the padded tap array
};

__host__ __device__ inline RoundDims round_dims(int nb) {
    RoundDims d;
    d.Q = kRoundR * ((nb + kRoundWaves * kRoundR - 1) / (kRoundWaves * kRoundR));
    d.KP = kRoundWaves * d.Q;
    d.OUTP = kRoundChunk * ((nb + kRoundChunk - 1) / kRoundChunk);
    const int e = d.KP + d.OUTP;
    d.TP = e + e / kRoundR + 1;
    return d;
}

// doubles of LDS: taps, u, four wave partials of a chunk, M q, the block sums
__host__ __device__ inline size_t round_lds_doubles(int nb) {
    const RoundDims d = round_dims(nb);
    return (size_t)d.TP + d.KP + 4 * kRoundChunk + nb + kRoundWaves;
}

__device__ __forceinline__ double block_allsum8(double v, double* red8) {
    v = wave_sum_all(v);
    __syncthreads();   // red8 free from any previous use
    if ((threadIdx.x & 63) == 0) red8[threadIdx.x >> 6] = v;
    __syncthreads();
    return ((red8[0] + red8[1]) + (red8[2] + red8[3])) + ((red8[4] + red8[5]) + (red8[6] + red8[7]));
}

// acc[r] = sum over k in [kb0, kb0 + Q) of h[i_r - k] u_k for the lane's
// outputs i_r = ob + 12 lane + r.  Tap element e (0 <= e < KP + OUTP) is
// h[e - KP] at sT[e + e / 12]; output i and bin k meet element KP + i - k.
__device__ __forceinline__ void round_matvec(const double* __restrict__ sT, const double* __restrict__ su, int KP,
                                             int Q, int ob, int kb0, int lane, double (&acc)[kRoundR]) {
    const int l13 = (kRoundR + 1) * lane;
    double buf[kRoundR];   // at sub-step s the tap of output r is buf[(r - s) mod 12]
    const int c0 = KP + ob - kb0;
#pragma unroll
    for (int r = 0; r < kRoundR; ++r) {
        const int e = c0 + r;
        buf[r] = sT[e + e / kRoundR + l13];
    }
    for (int kb = kb0; kb < kb0 + Q; kb += kRoundR) {
        const int c = KP + ob - kb;
#pragma unroll
        for (int s = 0; s < kRoundR; ++s) {
            const double uk = su[kb + s];
#pragma unroll
            for (int r = 0; r < kRoundR; ++r) acc[r] = fma(buf[(r - s + kRoundR) % kRoundR], uk, acc[r]);
            // the tap entering the window at k + 1 (element c - s - 1 + 12 lane >= 0)
            const int e = c - s - 1;
            buf[(kRoundR - 1 - s) % kRoundR] = sT[e + e / kRoundR + l13];
        }
    }
}

__device__ __forceinline__ void rows_ritz_view(const NormItem& it, int v, int steps, double tol,
                                               const double* __restrict__ sal, const double* __restrict__ sbb,
                                               double* __restrict__ sb, double* __restrict__ sib,
                                               int* __restrict__ sfirst);
constexpr int kRitzMaxSteps = CTPD_MAX_NORM_STEPS;
static_assert(4 * kRitzMaxSteps <= 4 * kRoundChunk, "the Ritz step's arrays fit in the wave partials' LDS");

// Steps j0 .. j1 - 1 of a running view's chain, then its Ritz step (the
// round's workgroup computes the Ritz value, the residual norm and the stop
// of its own chain, in the LDS of the wave partials, free by then).
__global__ __launch_bounds__(kRoundThreads) void rows_round_kernel(const NormItem* __restrict__ items,
                                                                   const RowRef* __restrict__ rows, int nrows,
                                                                   int j0, int j1, double tol) {
    extern __shared__ double rsm[];
    const int row = blockIdx.x;
    if (row >= nrows) return;
    const RowRef rr = rows[row];
    const NormItem& it = items[rr.prob];
    const int m = it.m, nb = it.nb, v = rr.view;
    if (it.done[v] || nb > kRoundMaxBins) return;
    const RoundDims d = round_dims(nb);
    double* sT = rsm;
    double* su = sT + d.TP;
    double* sp = su + d.KP;
    double* sy = sp + 4 * kRoundChunk;
    double* red8 = sy + nb;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const size_t base = (size_t)v * nb;
    for (int e = tid; e < d.KP + d.OUTP; e += kRoundThreads) {
        const int o = e - d.KP;
        sT[e + e / kRoundR] = (o > -nb && o < nb) ? it.taps64[nb - 1 + o] : 0.0;
    }
    for (int k = nb + tid; k < d.KP; k += kRoundThreads) su[k] = 0.0;
    double q[kRoundNpt], qp[kRoundNpt], sc[kRoundNpt];
#pragma unroll
    for (int r = 0; r < kRoundNpt; ++r) {
        const int i = tid + kRoundThreads * r;
        const bool in = i < nb;
        q[r] = in ? it.v[0][base + i] : 0.0;
        qp[r] = (in && j0 > 0) ? it.v[1][base + i] : 0.0;
        sc[r] = in ? it.rs[base + i] : 0.0;
    }
    double bprev = j0 > 0 ? it.b2[(size_t)(j0 - 1) * m + v] : 0.0;
    for (int j = j0; j < j1; ++j) {
#pragma unroll
        for (int r = 0; r < kRoundNpt; ++r) {
            const int i = tid + kRoundThreads * r;
            if (i < nb) su[i] = sc[r] * q[r];
        }
        __syncthreads();   // u (and on the first step the taps) complete; the previous step's sy read
        for (int ob = 0; ob < nb; ob += kRoundChunk) {
            double acc[kRoundR];
#pragma unroll
            for (int r = 0; r < kRoundR; ++r) acc[r] = 0.0;
            round_matvec(sT, su, d.KP, d.Q, ob, wv * d.Q, lane, acc);
            if (wv >= 4) {
#pragma unroll
                for (int r = 0; r < kRoundR; ++r) sp[(wv - 4) * kRoundChunk + r * 64 + lane] = acc[r];
            }
            __syncthreads();
            if (wv < 4) {
#pragma unroll
                for (int r = 0; r < kRoundR; ++r) {
                    double* p = sp + wv * kRoundChunk + r * 64 + lane;
                    *p = acc[r] + *p;
                }
            }
            __syncthreads();
            // slot r * 64 + l holds output ob + 12 l + r
            for (int t = tid; t < kRoundChunk; t += kRoundThreads) {
                const int i = ob + kRoundR * (t & 63) + (t >> 6);
                if (i < nb)
                    sy[i] = (sp[t] + sp[kRoundChunk + t]) + (sp[2 * kRoundChunk + t] + sp[3 * kRoundChunk + t]);
            }
            __syncthreads();   // sy complete; sp free for the next chunk
        }
        double y[kRoundNpt];
        double a = 0.0;
#pragma unroll
        for (int r = 0; r < kRoundNpt; ++r) {
            const int i = tid + kRoundThreads * r;
            y[r] = i < nb ? sc[r] * sy[i] : 0.0;
            a = fma(q[r], y[r], a);
        }
        a = block_allsum8(a, red8);
        const double b = j ? sqrt(bprev) : 0.0;
        double ss = 0.0;
#pragma unroll
        for (int r = 0; r < kRoundNpt; ++r) {
            double t = y[r] - a * q[r];
            if (j) t -= b * qp[r];
            y[r] = t;
            ss = fma(t, t, ss);
        }
        ss = block_allsum8(ss, red8);
        const double inv = ss > 0.0 ? 1.0 / sqrt(ss) : 1.0;
#pragma unroll
        for (int r = 0; r < kRoundNpt; ++r) {
            qp[r] = q[r];
            q[r] = ss > 0.0 ? y[r] * inv : y[r];
        }
        if (tid == 0) {
            it.al[(size_t)j * m + v] = a;
            it.b2[(size_t)j * m + v] = ss;
        }
        bprev = ss;
    }
#pragma unroll
    for (int r = 0; r < kRoundNpt; ++r) {
        const int i = tid + kRoundThreads * r;
        if (i < nb) {
            it.v[0][base + i] = q[r];
            it.v[1][base + i] = qp[r];
        }
    }
    // the Ritz step after j1 steps (thread 0's scalars of this round are
    // visible to the workgroup after the barrier)
    __syncthreads();
    double* sal = sp;
    double* sbb = sp + kRitzMaxSteps;
    for (int i = tid; i < j1; i += kRoundThreads) {
        sal[i] = it.al[(size_t)i * m + v];
        sbb[i] = it.b2[(size_t)i * m + v];
    }
    __syncthreads();
    rows_ritz_view(it, v, j1, tol, sal, sbb, sp + 2 * kRitzMaxSteps, sp + 3 * kRitzMaxSteps,
                   reinterpret_cast<int*>(red8));
}

// b / d for the Sturm recurrence: the reciprocal instruction refined by one
// Newton step (a few dependent instructions instead of the division's
// sequence; the counts only need the sign of each pivot)
__device__ __forceinline__ double sturm_quot(double b, double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    return b * r;
}

// Largest eigenvalues of the leading k x k and (k-1) x (k-1) sections of the
// tridiagonal matrix (alpha_i, sqrt(b2_i)) of a view, by multisection over the
// kRitzWaves waves of a workgroup: each round every lane counts (Sturm
// sequence) the eigenvalues below its own shift of each bracket (256 shifts),
// and each bracket shrinks to the interval between the last shift with fewer
// eigenvalues below than the section's size and the first with all of them
// (257x per round), until its width is 1e-12 of its magnitude -- far below
// the 1e-7 change that stops a chain.  The two sections' sequences are
// interleaved in one loop, so their dependent chains overlap.  th1 is NaN for
// k = 1.  Every thread of the workgroup calls it and gets the same results; a
// workgroup of more than kRitzWaves waves gives the same results too (its
// further waves only join the barriers).
constexpr int kRitzWaves = 4, kRitzThreads = 64 * kRitzWaves, kRitzShifts = kRitzThreads;

__device__ void rows_tridiag_max2(const double* __restrict__ al, const double* __restrict__ bb,
                                  const double* __restrict__ sb, int k, int* __restrict__ sfirst, double* th,
                                  double* th1) {
    // al[i]: alpha_i; bb[i]: beta_{i+1}^2 (couples i and i+1); sb[i] = sqrt(bb[i]); all in LDS
    const int k1 = k - 1;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    double lo = al[0], hi = al[0], lo1 = al[0], hi1 = al[0];
    for (int i = 0; i < k; ++i) {
        const double left = i > 0 ? sb[i - 1] : 0.0;
        const double r = left + (i < k - 1 ? sb[i] : 0.0);
        lo = fmin(lo, al[i] - r);
        hi = fmax(hi, al[i] + r);
        if (i < k1) {
            const double r1 = left + (i < k1 - 1 ? sb[i] : 0.0);
            lo1 = fmin(lo1, al[i] - r1);
            hi1 = fmax(hi1, al[i] + r1);
        }
    }
    if (!isfinite(lo) || !isfinite(hi)) {
        *th = hi;
        *th1 = k1 > 0 ? hi1 : NAN;
        return;
    }
    auto open = [](double l, double h) { return h - l > 1e-12 * fmax(fabs(l), fabs(h)); };
    // shift j (1 .. 256) of the bracket [l, h]; the bracket update reuses the
    // same expression, so its new ends are shifts that were tested
    auto shift = [](double l, double h, int j) {
        return l + (h - l) * ((double)j * (1.0 / (double)(kRitzShifts + 1)));
    };
    bool go = open(lo, hi), go1 = k1 > 0 && isfinite(lo1) && isfinite(hi1) && open(lo1, hi1);
    for (int round = 0; round < 40 && (go || go1); ++round) {
        const double x = shift(lo, hi, t + 1), x1 = shift(lo1, hi1, t + 1);
        int cnt = 0, cnt1 = 0;
        double d = 1.0, d1 = 1.0;
        // the recurrence scalars of 8 steps are read ahead of their dependent chain
        for (int i0 = 0; i0 < (wv < kRitzWaves ? k : 0); i0 += 8) {
            double A[8], B[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + u;
                A[u] = i < k ? al[i] : 0.0;
                B[u] = (i > 0 && i < k) ? bb[i - 1] : 0.0;
            }
            // branch-free (selects), so the two chains interleave; B = 0 at i = 0
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = i0 + u;
                const double dn = A[u] - x - sturm_quot(B[u], d);
                const double dn1 = A[u] - x1 - sturm_quot(B[u], d1);
                const bool on = i < k, on1 = i < k1;
                d = on ? (dn == 0.0 ? -1e-300 : dn) : d;
                d1 = on1 ? (dn1 == 0.0 ? -1e-300 : dn1) : d1;
                cnt += (on && d < 0.0) ? 1 : 0;
                cnt1 += (on1 && d1 < 0.0) ? 1 : 0;
            }
        }
        // the first shift (over the workgroup) that lies above every eigenvalue
        const unsigned long long above = __ballot(cnt == k), above1 = __ballot(cnt1 == k1);
        if (lane == 0 && wv < kRitzWaves) {
            sfirst[wv] = above ? wv * 64 + __ffsll((long long)above) - 1 : kRitzShifts;
            sfirst[kRitzWaves + wv] = above1 ? wv * 64 + __ffsll((long long)above1) - 1 : kRitzShifts;
        }
        __syncthreads();
        int f = kRitzShifts, f1 = kRitzShifts;
#pragma unroll
        for (int w = 0; w < kRitzWaves; ++w) {
            f = min(f, sfirst[w]);
            f1 = min(f1, sfirst[kRitzWaves + w]);
        }
        __syncthreads();   // sfirst free for the next round
        if (go) {
            const double nhi = f < kRitzShifts ? shift(lo, hi, f + 1) : hi;
            const double nlo = f > 0 ? shift(lo, hi, f) : lo;
            lo = nlo;
            hi = nhi;
            go = open(lo, hi);
        }
        if (go1) {
            const double nhi = f1 < kRitzShifts ? shift(lo1, hi1, f1 + 1) : hi1;
            const double nlo = f1 > 0 ? shift(lo1, hi1, f1) : lo1;
            lo1 = nlo;
            hi1 = nhi;
            go1 = open(lo1, hi1);
        }
    }
    *th = hi;
    *th1 = k1 > 0 ? hi1 : NAN;
}

constexpr int kRitzMax = CTPD_MAX_NORM_STEPS;   // steps a per-view chain can take

// Residual norm ||B q - th q|| of the Ritz pair (th, q = Q_k x / ||x||) of a
// chain after k steps, x the eigenvector of the tridiagonal T_k for th.  x is
// taken by the three-term recurrence of T_k x = th x run upwards from
// x_{k-1} = 1 (for the top Ritz value the components grow upwards, so the
// recurrence is stable in that direction); what the first row then misses,
// d0 = (th - alpha_0) x_0 - beta_1 x_1, is the error of th.  From
// B Q_k = Q_k T_k + beta_k q_k e_{k-1}^T, B q - th q = (d0 Q_k e_0 +
// beta_k x_{k-1} q_k) / ||x||, so the norm is at most (|d0| + beta_k) / ||x||,
// and B has an eigenvalue within that distance of th.  sb[i] = sqrt(bb[i]),
// sib[i] = 1 / sb[i]; bn = beta_k.  +inf when the recurrence does not stay
// finite.
__device__ double ritz_residual(const double* __restrict__ sal, const double* __restrict__ sb,
                                const double* __restrict__ sib, int k, double th, double bn) {
    double x = 1.0, xn = 0.0, nrm = 1.0, last = 1.0;   // x_i, x_{i+1}, sum x^2, x_{k-1}
    for (int i = k - 1; i >= 1; --i) {
        const double xp = ((th - sal[i]) * x - (i + 1 < k ? sb[i] * xn : 0.0)) * sib[i - 1];
        xn = x;
        x = xp;
        nrm = fma(xp, xp, nrm);
        if (fabs(x) > 1e100) {   // rescale, exactly (a power of two)
            const double f = 0x1p-332;
            x *= f;
            xn *= f;
            last *= f;
            nrm *= f * f;
        }
    }
    const double d0 = (th - sal[0]) * x - (k > 1 ? sb[0] * xn : 0.0);
    const double r = (fabs(d0) + bn * last) / sqrt(nrm);
    return isfinite(r) ? r : HUGE_VAL;
}

// After `steps` steps: a running view's top Ritz value and that value plus
// its residual norm; the view stops when the Ritz value changed by <= tol
// relative over the last step or its Krylov space is exhausted (beta ~ 0).
// sal / sbb hold the view's recurrence scalars (steps of each), sb / sib room
// for as many; every thread of the workgroup calls it.
__device__ __forceinline__ void rows_ritz_view(const NormItem& it, int v, int steps, double tol,
                                               const double* __restrict__ sal, const double* __restrict__ sbb,
                                               double* __restrict__ sb, double* __restrict__ sib,
                                               int* __restrict__ sfirst) {
    for (int i = threadIdx.x; i < steps; i += blockDim.x) {
        sb[i] = sqrt(fmax(sbb[i], 0.0));
        sib[i] = 1.0 / sb[i];
    }
    __syncthreads();
    double th, th1;
    rows_tridiag_max2(sal, sbb, sb, steps, sfirst, &th, &th1);
    const double bn = sb[steps - 1];
    bool stop = !(bn > 1e-300 * fmax(1.0, fabs(th))) || !isfinite(th);
    if (!stop && steps > 1) stop = fabs(th - th1) <= tol * fabs(th);
    if (threadIdx.x == 0) {
        it.theta[v] = th;
        it.ubound[v] = stop ? HUGE_VAL : th + ritz_residual(sal, sb, sib, steps, th, bn);
        if (stop) it.done[v] = steps;
    }
}

// The Ritz step of the per-step form (rows past the round kernel's size):
// one workgroup of kRitzWaves waves per view.
__global__ __launch_bounds__(kRitzThreads) void rows_ritz_kernel(const NormItem* __restrict__ items,
                                                                 const RowRef* __restrict__ rows, int nrows,
                                                                 int steps, double tol) {
    __shared__ double sal[kRitzMax], sbb[kRitzMax], sb[kRitzMax], sib[kRitzMax];
    __shared__ int sfirst[2 * kRitzWaves];
    const int row = blockIdx.x;
    if (row >= nrows) return;
    const RowRef rr = rows[row];
    const NormItem& it = items[rr.prob];
    const int v = rr.view, m = it.m;
    if (it.done[v]) return;   // uniform over the workgroup
    // the view's recurrence scalars into LDS (strided by m in HBM; read once)
    for (int i = threadIdx.x; i < steps; i += kRitzThreads) {
        sal[i] = it.al[(size_t)i * m + v];
        sbb[i] = it.b2[(size_t)i * m + v];
    }
    __syncthreads();
    rows_ritz_view(it, v, steps, tol, sal, sbb, sb, sib, sfirst);
}

// one workgroup per problem: {max theta, running views, max steps}, after
// stopping the views whose eigenvalue lies below the largest Ritz value (a
// lower bound of the problem's lambda_h; the margin covers the rounding of
// the Ritz values): those whose symbol bound is below it, and those whose Ritz
// value plus residual norm is -- B_v then has an eigenvalue below it next to
// the Ritz value, and that eigenvalue is taken for the top one, the reading
// the stopping rule of a converged chain rests on as well.
__global__ __launch_bounds__(256) void rows_summary_kernel(const NormItem* __restrict__ items, int steps) {
    const NormItem& it = items[blockIdx.x];
    __shared__ double r0[256], r1[256], r2[256];
    double mx = -1e300;
    for (int v = threadIdx.x; v < it.m; v += 256) {
        const double th = it.theta[v];
        if (isfinite(th)) mx = fmax(mx, th);
    }
    r0[threadIdx.x] = mx;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) r0[threadIdx.x] = fmax(r0[threadIdx.x], r0[threadIdx.x + off]);
        __syncthreads();
    }
    mx = r0[0];
    __syncthreads();
    const double cut = it.fsym ? mx * (1.0 - 1e-9) : -1e300;
    double run = 0.0, st = 0.0;
    for (int v = threadIdx.x; v < it.m; v += 256) {
        if (!it.done[v] && it.fsym && (it.fsym[0] * it.maxinv[v] < cut || it.ubound[v] < cut)) it.done[v] = steps;
        if (!it.done[v]) run += 1.0;
        st = fmax(st, (double)it.done[v]);
    }
    r0[threadIdx.x] = mx;
    r1[threadIdx.x] = run;
    r2[threadIdx.x] = st;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            r0[threadIdx.x] = fmax(r0[threadIdx.x], r0[threadIdx.x + off]);
            r1[threadIdx.x] += r1[threadIdx.x + off];
            r2[threadIdx.x] = fmax(r2[threadIdx.x], r2[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        it.summary[0] = r0[0];
        it.summary[1] = r1[0];
        it.summary[2] = r2[0];
    }
}

#undef ROW_PROLOGUE

hipError_t launch_rows_start(const NormItem* it, const RowRef* rows, int nrows, uint64_t seed, hipStream_t s) {
    rows_start_kernel<<<(nrows + 3) / 4, 256, 0, s>>>(it, rows, nrows, seed);
    return hipGetLastError();
}

hipError_t launch_rows_prune(const NormItem* it, const RowRef* rows, int nrows, int count, hipStream_t s) {
    rows_lower_kernel<<<(nrows + 3) / 4, 256, 0, s>>>(it, rows, nrows);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    rows_summary_kernel<<<count, 256, 0, s>>>(it, 1);
    return hipGetLastError();
}

hipError_t launch_rows_step(const NormItem* it, const RowRef* rows, int nrows, int rot, int j, hipStream_t s) {
    rows_step_kernel<<<nrows, 256, 0, s>>>(it, rows, nrows, rot, j);
    return hipGetLastError();
}

bool rows_round_fits(int max_nb) {
    return max_nb <= kRoundMaxBins && round_lds_doubles(max_nb) * sizeof(double) <= 65536;
}

hipError_t launch_rows_round(const NormItem* it, const RowRef* rows, int nrows, int count, int j0, int j1,
                             int max_nb, double tol, hipStream_t s) {
    if (!rows_round_fits(max_nb)) return hipErrorInvalidValue;
    rows_round_kernel<<<nrows, kRoundThreads, round_lds_doubles(max_nb) * sizeof(double), s>>>(it, rows, nrows, j0,
                                                                                                j1, tol);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    rows_summary_kernel<<<count, 256, 0, s>>>(it, j1);
    return hipGetLastError();
}

hipError_t launch_rows_ritz(const NormItem* it, const RowRef* rows, int nrows, int count, int steps, double tol,
                            hipStream_t s) {
    rows_ritz_kernel<<<nrows, kRitzThreads, 0, s>>>(it, rows, nrows, steps, tol);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    rows_summary_kernel<<<count, 256, 0, s>>>(it, steps);
    return hipGetLastError();
}

// Batched solve start / end, 2048 elements per workgroup of the problem's
// virtual concatenation [x | p0 | mu0 | mu1] (init: zeroed) or [x] (copy-out).
__global__ __launch_bounds__(256) void batch_init_kernel(const BatchItem* __restrict__ items,
                                                         const BlockRef* __restrict__ map) {
    const BlockRef e = map[blockIdx.x];
    if (e.prob < 0) return;
    const BatchItem& it = items[e.prob];
    const size_t J = (size_t)it.n * it.n, I = (size_t)it.m * it.nb;
    for (int r = 0; r < 8; ++r) {
        size_t i = (size_t)e.local * 2048 + r * 256 + threadIdx.x;
        if (i < J) {
            it.x[i] = 0.f;
            continue;
        }
        i -= J;
        if (i < 2 * J) {
            it.p[0][i] = 0.f;
            continue;
        }
        i -= 2 * J;
        if (i < I) {
            it.mu[0][i] = 0.f;
            continue;
        }
        i -= I;
        if (i < I) it.mu[1][i] = 0.f;
    }
}

__global__ __launch_bounds__(256) void batch_copy_out_kernel(const BatchItem* __restrict__ items,
                                                             const BlockRef* __restrict__ map) {
    const BlockRef e = map[blockIdx.x];
    if (e.prob < 0) return;
    const BatchItem& it = items[e.prob];
    const size_t J = (size_t)it.n * it.n;
    for (int r = 0; r < 8; ++r) {
        const size_t i = (size_t)e.local * 2048 + r * 256 + threadIdx.x;
        if (i < J) it.x_out[i] = it.x[i];
    }
}

// the first iteration's z = -sigma (x - tau A^T D b), in place (the copy-out map)
__global__ __launch_bounds__(256) void batch_scale_z_kernel(const BatchItem* __restrict__ items,
                                                            const BlockRef* __restrict__ map) {
    const BlockRef e = map[blockIdx.x];
    if (e.prob < 0) return;
    const BatchItem& it = items[e.prob];
    const size_t J = (size_t)it.n * it.n;
    const float c = -it.sigma;
    for (int r = 0; r < 8; ++r) {
        const size_t i = (size_t)e.local * 2048 + r * 256 + threadIdx.x;
        if (i < J) it.z[i] = c * it.z[i];
    }
}

hipError_t launch_batch_scale_z(const BatchItem* items, const BlockRef* map, int nblocks, hipStream_t s) {
    batch_scale_z_kernel<<<nblocks, 256, 0, s>>>(items, map);
    return hipGetLastError();
}

hipError_t launch_batch_init(const BatchItem* items, const BlockRef* map, int nblocks, hipStream_t s) {
    batch_init_kernel<<<nblocks, 256, 0, s>>>(items, map);
    return hipGetLastError();
}

hipError_t launch_batch_copy_out(const BatchItem* items, const BlockRef* map, int nblocks, hipStream_t s) {
    batch_copy_out_kernel<<<nblocks, 256, 0, s>>>(items, map);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void axpby_kernel(double* __restrict__ y, const double* __restrict__ x, double a,
                                                    double b, const double* __restrict__ z, double c, size_t len) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= len) return;
    double r = a * x[i] + b * y[i];
    if (z) r += c * z[i];
    y[i] = r;
}

hipError_t launch_axpby_f64(double* y, const double* x, double a, double b, const double* z, double c,
                            size_t len, hipStream_t s) {
    axpby_kernel<<<(unsigned)((len + 255) / 256), 256, 0, s>>>(y, x, a, b, z, c, len);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void scale_kernel(double* __restrict__ y, const double* __restrict__ x, double a,
                                                    size_t len) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < len) y[i] = a * x[i];
}

hipError_t launch_scale_f64(double* y, const double* x, double a, size_t len, hipStream_t s) {
    scale_kernel<<<(unsigned)((len + 255) / 256), 256, 0, s>>>(y, x, a, len);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void inverse_kernel(float* __restrict__ out, const float* __restrict__ w,
                                                      size_t len) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < len) out[i] = (float)(1.0 / (double)w[i]);
}

hipError_t launch_inverse_f32(float* out, const float* w, size_t len, hipStream_t s) {
    inverse_kernel<<<(unsigned)((len + 255) / 256), 256, 0, s>>>(out, w, len);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void rsqrt_kernel(double* __restrict__ out, const float* __restrict__ w,
                                                    size_t len) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < len) out[i] = sqrt(1.0 / (double)w[i]);
}

hipError_t launch_rsqrt_f64(double* out, const float* w, size_t len, hipStream_t s) {
    rsqrt_kernel<<<(unsigned)((len + 255) / 256), 256, 0, s>>>(out, w, len);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void copy_kernel(float* __restrict__ dst, const float* __restrict__ src,
                                                   size_t len) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < len) dst[i] = src[i];
}

hipError_t launch_copy_f32(float* dst, const float* src, size_t len, hipStream_t s) {
    if (len == 0) return hipSuccess;
    copy_kernel<<<(unsigned)((len + 255) / 256), 256, 0, s>>>(dst, src, len);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_kernel(float* __restrict__ dst, float v, size_t len) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < len) dst[i] = v;
}

hipError_t launch_fill_f32(float* dst, float v, size_t len, hipStream_t s) {
    if (len == 0) return hipSuccess;
    fill_kernel<<<(unsigned)((len + 255) / 256), 256, 0, s>>>(dst, v, len);
    return hipGetLastError();
}

// Zero four buffers in one launch.  Buffer q owns the index span span[q]
// (its length rounded up to a multiple of 4, spans laid end to end); a thread
// clears 4 consecutive elements of one buffer, never past its length n[q].
struct Zero4 {
    float* p[4];
    size_t n[4], span[4];
};

__global__ __launch_bounds__(256) void zero4_kernel(Zero4 z) {
    size_t i = ((size_t)blockIdx.x * 256 + threadIdx.x) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (i < z.span[q]) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (i + e < z.n[q]) z.p[q][i + e] = 0.f;
            return;
        }
        i -= z.span[q];
    }
}

hipError_t launch_zero4_f32(float* a, size_t na, float* b, size_t nb, float* c, size_t nc, float* d, size_t nd,
                            hipStream_t s) {
    Zero4 z{{a, b, c, d}, {na, nb, nc, nd}, {}};
    size_t total = 0;
    for (int q = 0; q < 4; ++q) {
        z.span[q] = (z.n[q] + 3) / 4 * 4;
        total += z.span[q];
    }
    if (total == 0) return hipSuccess;
    zero4_kernel<<<(unsigned)((total / 4 + 255) / 256), 256, 0, s>>>(z);
    return hipGetLastError();
}

// Recorded elementwise / reduction steps (one table entry per problem).
// Elementwise kinds: 256 elements per workgroup.  SK_DOT: the problem's
// reduce_blocks(len) workgroups stride over len, as launch_dot_partials.
// SK_SLOTS: one workgroup per slot.
__global__ __launch_bounds__(256) void step_vec_kernel(const UStep* __restrict__ steps,
                                                       const BlockRef* __restrict__ map) {
    const BlockRef e = map[blockIdx.x];
    if (e.prob < 0) return;
    const UStep& st = steps[e.prob];
    if (!st.active) return;
    const int kind = st.kind;
    if (kind == SK_DOT) {
        const size_t stride = (size_t)reduce_blocks(st.len) * 256;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (size_t i = (size_t)e.local * 256 + threadIdx.x; i < st.len; i += stride)
            s0 = fma((double)st.in[0][i], (double)st.in[1][i], s0);
        block_sum3(s0, s1, s2);
        if (threadIdx.x == 0) st.part[e.local] = s0;
        return;
    }
    if (kind == SK_SLOTS) {
        const double* p = st.part + (size_t)e.local * st.steps;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int b = threadIdx.x; b < st.steps; b += 256) s0 += p[b];
        block_sum3(s0, s1, s2);
        if (threadIdx.x == 0) st.dout[e.local] = s0;
        return;
    }
    const size_t i = (size_t)e.local * 256 + threadIdx.x;
    if (i >= st.len) return;
    switch (kind) {
        case SK_LIN3: {
            float r = st.c0 * st.in[0][i];
            if (st.in[1]) r = fmaf(st.c1, st.in[1][i], r);
            if (st.in[2]) r = fmaf(st.c2, st.in[2][i], r);
            if (st.in[3]) r *= st.in[3][i];
            st.out[0][i] = r;
            break;
        }
        case SK_LINMIX: {
            float r = st.c0 * st.in[0][i];
            if (st.in[1]) r = fmaf(st.c1, st.in[1][i], r);
            if (st.in[2]) r = fmaf(st.c2, st.in[3] ? st.in[2][i] * st.in[3][i] : st.in[2][i], r);
            st.out[0][i] = r;
            break;
        }
        case SK_COPY: st.out[0][i] = st.in[0][i]; break;
        case SK_FILL: st.out[0][i] = st.c0; break;
        case SK_INV: st.out[0][i] = (float)(1.0 / (double)st.in[0][i]); break;
        case SK_FILL64: st.part[i] = 0.0; break;
        default: break;
    }
}

hipError_t launch_step_vec(int kind, const UStep* steps, const BlockRef* map, int nblocks, hipStream_t s) {
    (void)kind;
    step_vec_kernel<<<nblocks, 256, 0, s>>>(steps, map);
    return hipGetLastError();
}

// out[0] = max over i of 1/w[i] (float64), two passes of fixed order.
__global__ __launch_bounds__(256) void max_inv_partial_kernel(const float* __restrict__ w, size_t len,
                                                              double* __restrict__ partial) {
    __shared__ double red[4];
    double mx = 0.0;
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < len; i += stride) mx = fmax(mx, 1.0 / (double)w[i]);
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ __launch_bounds__(256) void max_final_kernel(const double* __restrict__ partial, int n,
                                                        double* __restrict__ out) {
    __shared__ double red[4];
    double mx = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) mx = fmax(mx, partial[i]);
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

hipError_t launch_max_inv(const float* w, size_t len, double* partials, double* dev_out, hipStream_t s) {
    const int nb = reduce_blocks(len);
    max_inv_partial_kernel<<<nb, 256, 0, s>>>(w, len, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    max_final_kernel<<<1, 256, 0, s>>>(partials, nb, dev_out);
    return hipGetLastError();
}

// taps of D = I: 1 at offset 0, 0 elsewhere
__global__ __launch_bounds__(256) void identity_taps_kernel(double* __restrict__ taps64, float* __restrict__ taps32,
                                                            int ntap) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < ntap) {
        const double v = (i == ntap / 2) ? 1.0 : 0.0;
        taps64[i] = v;
        taps32[i] = (float)v;
    }
}

hipError_t launch_identity_taps(double* taps64, float* taps32, int nb, hipStream_t s) {
    const int ntap = 2 * nb - 1;
    identity_taps_kernel<<<(ntap + 255) / 256, 256, 0, s>>>(taps64, taps32, ntap);
    return hipGetLastError();
}

}  // namespace ctpd
