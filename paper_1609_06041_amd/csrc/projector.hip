// Joseph ray-driven forward projector A and its exact transpose A^T
// (Sec. 2.1 system matrix; the dominant per-iteration operations of
// Eqs. 18-20 and 29-31).
//
// Both kernels are gathers (no atomics), so results are deterministic.
// Sample positions are computed in float64: in float32 a position of ~500
// pixels carries ~3e-5 pixel of rounding, which alone would exceed a 1e-5
// relative error on non-smooth images; the float64 position costs a few
// full-rate DP instructions per sample on CDNA.
#include "internal.h"

namespace ctpd {

// ---------------------------------------------------------------------------
// Transpose (column views read the image along columns; keeping a transposed
// copy makes their taps contiguous and the wave's loads coalesced).
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T* __restrict__ in, T* __restrict__ out, int n) {
    __shared__ T tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int iy = by + r, ix = bx + tx;
        if (iy < n && ix < n) tile[r][tx] = in[(size_t)iy * n + ix];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int ox = bx + r, oy = by + tx;   // out[ox][oy] = in[oy][ox]
        if (ox < n && oy < n) out[(size_t)ox * n + oy] = tile[tx][r];
    }
}

template <typename T>
hipError_t launch_transpose(const T* in, T* out, int n, hipStream_t s) {
    dim3 grid((n + 31) / 32, (n + 31) / 32);
    transpose_kernel<T><<<grid, 256, 0, s>>>(in, out, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Forward projection: one lane per ray (v, u).  Consecutive lanes are
// consecutive bins of one view, so at each step the wave reads a short
// contiguous run of one image row (row views) or one row of the transposed
// image (column views).
template <typename T>
__global__ __launch_bounds__(256) void forward_kernel(const T* __restrict__ x, const T* __restrict__ xT,
                                                      T* __restrict__ y, const ViewGeom* __restrict__ views,
                                                      int n, int nb) {
    const int v = blockIdx.y;
    const int u = blockIdx.x * 256 + threadIdx.x;
    if (u >= nb) return;
    const ViewGeom g = views[v];
    const T* __restrict__ plane = g.row ? x : xT;
    const double base = fma((double)u, g.su, g.s0);
    // Steps whose sample lies in (-1, n) touch the image; outside both taps are zero.
    int t0 = 0, t1 = n - 1;
    if (g.st != 0.0) {
        const double ta = (-1.0 - base) / g.st, tb = ((double)n - base) / g.st;
        const double lo = fmin(fmax(fmin(ta, tb) - 1.0, 0.0), (double)n);
        const double hi = fmax(fmin(fmax(ta, tb) + 1.0, (double)(n - 1)), -1.0);
        t0 = (int)floor(lo);
        t1 = (int)ceil(hi);
    } else if (!(base > -1.0 && base < (double)n)) {
        t1 = -1;
    }
    T acc = T(0);
    for (int t = t0; t <= t1; ++t) {
        const double s = fma((double)t, g.st, base);
        const double fl = floor(s);
        const int k = (int)fl;
        const T f = (T)(s - fl);
        const T* __restrict__ row = plane + (size_t)t * n;
        const T a = (k >= 0 && k < n) ? row[k] : T(0);
        const T b = (k >= -1 && k < n - 1) ? row[k + 1] : T(0);
        acc += a + f * (b - a);
    }
    y[(size_t)v * nb + u] = acc * (T)g.len;
}

template <typename T>
hipError_t launch_forward(const T* x, const T* xT, T* y, const ViewGeom* views, int n, int m, int nb,
                          hipStream_t s) {
    dim3 grid((nb + 255) / 256, m);
    forward_kernel<T><<<grid, 256, 0, s>>>(x, xT, y, views, n, nb);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Transpose of the forward projector as a pixel-driven gather.  For pixel
// (X, Y) and view v the Joseph weights of A are the hat function
// max(0, 1 - |u - t|/s_v)/s_v of the distance between bin u and the pixel's
// bin coordinate t = X cos + Y sin + (nb-1)/2, with s_v = |cos| (row views)
// or |sin| (column views) <= 1, so at most the bins floor(t), floor(t)+1 carry
// weight.  out = alpha * xin + beta * A^T (c1 y1 + c2 y2).
template <typename T, bool TWO>
__global__ __launch_bounds__(256) void adjoint_kernel(const T* __restrict__ y1, const T* __restrict__ y2, T c1,
                                                      T c2, const T* __restrict__ xin, T alpha, T beta,
                                                      T* __restrict__ out, const ViewGeom* __restrict__ views,
                                                      int n, int m, int nb) {
    const int ix = blockIdx.x * 16 + (threadIdx.x & 15);
    const int iy = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (ix >= n || iy >= n) return;
    const double c = 0.5 * (double)(n - 1), cd = 0.5 * (double)(nb - 1);
    const double X = (double)ix - c, Y = (double)iy - c;
    T acc = T(0);
    for (int v = 0; v < m; ++v) {
        const ViewGeom g = views[v];
        const double t = fma(X, g.cs, fma(Y, g.sn, cd));
        const double fl = floor(t);
        const int u0 = (int)fl;
        const T f = (T)(t - fl);
        const T len = (T)g.len, len2 = (T)g.len2;
        const T w0 = fmax(T(0), len - f * len2);
        const T w1 = fmax(T(0), len - (T(1) - f) * len2);
        const size_t rb = (size_t)v * nb;
        T a = T(0), b = T(0);
        if (u0 >= 0 && u0 < nb) a = TWO ? c1 * y1[rb + u0] + c2 * y2[rb + u0] : y1[rb + u0];
        if (u0 >= -1 && u0 < nb - 1) b = TWO ? c1 * y1[rb + u0 + 1] + c2 * y2[rb + u0 + 1] : y1[rb + u0 + 1];
        acc += w0 * a + w1 * b;
    }
    const size_t idx = (size_t)iy * n + ix;
    T r = beta * acc;
    if (xin) r += alpha * xin[idx];
    out[idx] = r;
}

template <typename T>
hipError_t launch_adjoint(const T* y1, const T* y2, T c1, T c2, const T* xin, T alpha, T beta, T* out,
                          const ViewGeom* views, int n, int m, int nb, hipStream_t s) {
    dim3 grid((n + 15) / 16, (n + 15) / 16);
    if (y2)
        adjoint_kernel<T, true><<<grid, 256, 0, s>>>(y1, y2, c1, c2, xin, alpha, beta, out, views, n, m, nb);
    else
        adjoint_kernel<T, false><<<grid, 256, 0, s>>>(y1, y2, c1, c2, xin, alpha, beta, out, views, n, m, nb);
    return hipGetLastError();
}

template hipError_t launch_transpose<float>(const float*, float*, int, hipStream_t);
template hipError_t launch_transpose<double>(const double*, double*, int, hipStream_t);
template hipError_t launch_forward<float>(const float*, const float*, float*, const ViewGeom*, int, int, int,
                                          hipStream_t);
template hipError_t launch_forward<double>(const double*, const double*, double*, const ViewGeom*, int, int,
                                           int, hipStream_t);
template hipError_t launch_adjoint<float>(const float*, const float*, float, float, const float*, float, float,
                                          float*, const ViewGeom*, int, int, int, hipStream_t);
template hipError_t launch_adjoint<double>(const double*, const double*, double, double, const double*, double,
                                           double, double*, const ViewGeom*, int, int, int, hipStream_t);

}  // namespace ctpd
