// TV prox with non-negativity (Eq. 17, the prox of Eqs. 19 and 30), solved on
// the dual field p by projected gradient steps (Chambolle's projection with
// the constraint x >= 0 inside):
//     x~ = max(0, z - lam div p)
//     p  <- (p - step grad x~) / max(1, |p - step grad x~|),  step = tau_c / lam
// and finally x = max(0, z - lam div p).  grad is the forward difference of
// Eq. 2's h_j, v_j (zero on the last column / row), div its negative adjoint.
//
// The step kernel is a 5-point stencil: every lane forms x~ at its pixel and
// at its right and lower neighbours directly from z and p (reads hit L1/L2),
// so one launch is one dual step, with p double-buffered.
#include "internal.h"

namespace ctpd {

__device__ __forceinline__ float div_p(const float* __restrict__ p1, const float* __restrict__ p2, int i, int j,
                                       int n) {
    const size_t idx = (size_t)i * n + j;
    float d = 0.0f;
    if (j < n - 1) d += p1[idx];
    if (j > 0) d -= p1[idx - 1];
    if (i < n - 1) d += p2[idx];
    if (i > 0) d -= p2[idx - n];
    return d;
}

__device__ __forceinline__ float xtilde(const float* __restrict__ z, const float* __restrict__ p1,
                                        const float* __restrict__ p2, int i, int j, int n, float lam) {
    return fmaxf(0.0f, z[(size_t)i * n + j] - lam * div_p(p1, p2, i, j, n));
}

__global__ __launch_bounds__(256) void tv_step_kernel(const float* __restrict__ z, const float* __restrict__ p_in,
                                                      float* __restrict__ p_out, int n, float lam, float step) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= n || j >= n) return;
    const size_t nn = (size_t)n * n;
    const float* __restrict__ p1 = p_in;
    const float* __restrict__ p2 = p_in + nn;
    const float xc = xtilde(z, p1, p2, i, j, n, lam);
    const float g1 = (j < n - 1) ? xtilde(z, p1, p2, i, j + 1, n, lam) - xc : 0.0f;
    const float g2 = (i < n - 1) ? xtilde(z, p1, p2, i + 1, j, n, lam) - xc : 0.0f;
    const size_t idx = (size_t)i * n + j;
    const float q1 = p1[idx] - step * g1;
    const float q2 = p2[idx] - step * g2;
    const float s = fmaxf(1.0f, sqrtf(q1 * q1 + q2 * q2));
    p_out[idx] = q1 / s;
    p_out[nn + idx] = q2 / s;
}

__global__ __launch_bounds__(256) void tv_finalize_kernel(const float* __restrict__ z, const float* __restrict__ p,
                                                          float* __restrict__ x, int n, float lam) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= n || j >= n) return;
    const size_t nn = (size_t)n * n;
    x[(size_t)i * n + j] = (lam == 0.0f) ? fmaxf(0.0f, z[(size_t)i * n + j]) : xtilde(z, p, p + nn, i, j, n, lam);
}

hipError_t launch_tv_step(const float* z, const float* p_in, float* p_out, int n, float lam, float step,
                          hipStream_t s) {
    dim3 grid((n + 63) / 64, (n + 3) / 4);
    tv_step_kernel<<<grid, 256, 0, s>>>(z, p_in, p_out, n, lam, step);
    return hipGetLastError();
}

hipError_t launch_tv_finalize(const float* z, const float* p, float* x, int n, float lam, hipStream_t s) {
    dim3 grid((n + 63) / 64, (n + 3) / 4);
    tv_finalize_kernel<<<grid, 256, 0, s>>>(z, p, x, n, lam);
    return hipGetLastError();
}

}  // namespace ctpd
