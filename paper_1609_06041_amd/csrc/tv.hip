// TV prox with non-negativity (Eq. 17, the prox of Eqs. 19 and 30), solved on
// the dual field p by projected gradient steps (Chambolle's projection with
// the constraint x >= 0 inside):
//     x~ = max(0, z - lam div p)
//     p  <- (p - step grad x~) / max(1, |p - step grad x~|),  step = tau_c / lam
// and finally x = max(0, z - lam div p).  grad is the forward difference of
// Eq. 2's h_j, v_j (zero on the last column / row), div its negative adjoint.
//
// The prox kernel blocks the dual steps in time: a workgroup owns a 32 x 32
// tile, stages z and p on the tile plus a halo of (steps + 1) pixels in LDS,
// and runs up to kTvChunk steps there (one step reads p one pixel away in
// each direction, so the valid region shrinks by one pixel per step and the
// halo is what is used up), then writes p and, on the last chunk, x for the
// tile.  Chunks ping-pong p between two global buffers.
#include <utility>

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

constexpr int kTvTile = 32;
constexpr int kTvChunk = 10;
constexpr int kTvMaxW = kTvTile + 2 * (kTvChunk + 1);

// One workgroup = 16 waves (four per SIMD, to hide the LDS latency of the
// dependent stencil reads); a wave sweeps one 64-wide LDS row at a time.
constexpr int kTvThreads = 1024;

// ps_store (optional): the dual field after every step t = 1..steps is also
// written to ps_store + (t - 1) * 2 n^2 (the interior stays valid: the halo
// is one pixel wider than the steps taken).
template <int THREADS>
__device__ __forceinline__ void tv_prox_body(const float* __restrict__ z, const float* __restrict__ p_in,
                                             float* __restrict__ p_out, float* __restrict__ x, int n, float lam,
                                             float step, int steps, int bxi, int byi,
                                             float* __restrict__ ps_store = nullptr) {
    __shared__ float sz[kTvMaxW * kTvMaxW], sx[kTvMaxW * kTvMaxW];
    __shared__ float s1[kTvMaxW * kTvMaxW], s2[kTvMaxW * kTvMaxW];
    const int H = steps + 1, W = kTvTile + 2 * H;
    const int i0 = byi * kTvTile - H, j0 = bxi * kTvTile - H;
    const int c = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const size_t nn = (size_t)n * n;
    const int j = j0 + c;
    const bool colin = c < W;
    const bool jin = colin && j >= 0 && j < n;
    for (int r = ty; r < W; r += (THREADS / 64)) {
        const int i = i0 + r;
        if (!colin) continue;
        const int o = r * W + c;
        float zz = 0.f, a1 = 0.f, a2 = 0.f;
        if (jin && i >= 0 && i < n) {
            const size_t g = (size_t)i * n + j;
            zz = z[g];
            a1 = p_in[g];
            a2 = p_in[nn + g];
        }
        sz[o] = zz;
        s1[o] = a1;
        s2[o] = a2;
    }
    __syncthreads();
    // x~ at LDS cell (r, c) with the masked divergence of the global pixel (i, j)
    auto xt_at = [&](int r, int i) -> float {
        const int o = r * W + c;
        float d = 0.f;
        if (j < n - 1) d += s1[o];
        if (j > 0 && c > 0) d -= s1[o - 1];
        if (i < n - 1) d += s2[o];
        if (i > 0 && r > 0) d -= s2[o - W];
        return fmaxf(0.f, sz[o] - lam * d);
    };
    for (int t = 1; t <= steps; ++t) {
        // cells whose new p is still needed: rows / columns [t, W - t)
        for (int r = t - 1 + ty; r < W - t + 1; r += (THREADS / 64)) {
            if (!colin) continue;
            sx[r * W + c] = xt_at(r, i0 + r);
        }
        __syncthreads();
        for (int r = t + ty; r < W - t; r += (THREADS / 64)) {
            const int i = i0 + r;
            if (!(jin && c >= t && c < W - t && i >= 0 && i < n)) continue;
            const int o = r * W + c;
            const float xc = sx[o];
            const float g1 = (j < n - 1) ? sx[o + 1] - xc : 0.f;
            const float g2 = (i < n - 1) ? sx[o + W] - xc : 0.f;
            const float q1 = s1[o] - step * g1, q2 = s2[o] - step * g2;
            const float sc = fmaxf(1.f, sqrtf(q1 * q1 + q2 * q2));
            s1[o] = q1 / sc;
            s2[o] = q2 / sc;
        }
        __syncthreads();
        if (ps_store) {
            float* dst = ps_store + (size_t)(t - 1) * 2 * nn;
            for (int r = H + ty; r < H + kTvTile; r += (THREADS / 64)) {
                const int i = i0 + r;
                if (!(jin && c >= H && c < H + kTvTile && i < n)) continue;
                const size_t g = (size_t)i * n + j;
                dst[g] = s1[r * W + c];
                dst[nn + g] = s2[r * W + c];
            }
        }
    }
    for (int r = H + ty; r < H + kTvTile; r += (THREADS / 64)) {
        const int i = i0 + r;
        if (!(jin && c >= H && c < H + kTvTile && i < n)) continue;
        const int o = r * W + c;
        const size_t g = (size_t)i * n + j;
        p_out[g] = s1[o];
        p_out[nn + g] = s2[o];
        if (x) x[g] = xt_at(r, i);
    }
}

// x may alias z (each pixel reads only its own z)
__global__ __launch_bounds__(256) void tv_finalize_kernel(const float* z, const float* __restrict__ p, float* x, int n,
                                                          float lam) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= n || j >= n) return;
    const size_t nn = (size_t)n * n;
    x[(size_t)i * n + j] = (lam == 0.0f) ? fmaxf(0.0f, z[(size_t)i * n + j]) : xtilde(z, p, p + nn, i, j, n, lam);
}

__global__ __launch_bounds__(kTvThreads) void tv_prox_kernel(const float* __restrict__ z,
                                                             const float* __restrict__ p_in,
                                                             float* __restrict__ p_out, float* __restrict__ x, int n,
                                                             float lam, float step, int steps) {
    tv_prox_body<kTvThreads>(z, p_in, p_out, x, n, lam, step, steps, blockIdx.x, blockIdx.y);
}

// Batched TV prox chunk: p[src] -> p[1 - src] for every problem, x written on
// the last chunk; a problem with lam == 0 (beta = 0) takes x = max(0, z).
// THREADS (512 or 1024 per 32 x 32 tile) is a tuning choice of the batch.
template <int THREADS>
__global__ __launch_bounds__(THREADS) void tv_prox_batched(const BatchItem* __restrict__ items,
                                                           const BlockRef* __restrict__ map, int src, int steps,
                                                           int last) {
    const BlockRef e = map[blockIdx.x];
    if (e.prob < 0) return;
    const BatchItem& it = items[e.prob];
    const int gx = (it.n + kTvTile - 1) / kTvTile;
    const int bxi = e.local % gx, byi = e.local / gx;
    if (it.lam > 0.f) {
        tv_prox_body<THREADS>(it.z, it.p[src], it.p[1 - src], last ? it.x : nullptr, it.n, it.lam, it.tvstep, steps,
                              bxi, byi);
    } else if (last) {
        const int c = threadIdx.x & 63, ty = threadIdx.x >> 6;
        const int j = bxi * kTvTile + c;
        for (int r = ty; r < kTvTile; r += THREADS / 64) {
            const int i = byi * kTvTile + r;
            if (c < kTvTile && i < it.n && j < it.n) {
                const size_t g = (size_t)i * it.n + j;
                it.x[g] = fmaxf(0.f, it.z[g]);
            }
        }
    }
}

hipError_t launch_tv_prox_batched(const BatchItem* items, const BlockRef* map, int nblocks, int src, int steps,
                                  bool last, int threads, hipStream_t s) {
    if (threads == 512)
        tv_prox_batched<512><<<nblocks, 512, 0, s>>>(items, map, src, steps, last ? 1 : 0);
    else
        tv_prox_batched<1024><<<nblocks, 1024, 0, s>>>(items, map, src, steps, last ? 1 : 0);
    return hipGetLastError();
}

int tv_tiles(int n) { return (n + kTvTile - 1) / kTvTile; }
int tv_chunk_max() { return kTvChunk; }

__global__ __launch_bounds__(256) void grad_ball_kernel(const float* __restrict__ xb, float* __restrict__ p, int n,
                                                        float sg) {
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= n || j >= n) return;
    const size_t nn = (size_t)n * n, idx = (size_t)i * n + j;
    const float xc = xb[idx];
    const float g1 = (j < n - 1) ? xb[idx + 1] - xc : 0.f;
    const float g2 = (i < n - 1) ? xb[idx + n] - xc : 0.f;
    const float q1 = fmaf(sg, g1, p[idx]), q2 = fmaf(sg, g2, p[nn + idx]);
    const float sc = fmaxf(1.f, sqrtf(q1 * q1 + q2 * q2));
    p[idx] = q1 / sc;
    p[nn + idx] = q2 / sc;
}

hipError_t launch_grad_ball(const float* xb, float* p, int n, float sg, hipStream_t s) {
    dim3 grid((n + 63) / 64, (n + 3) / 4);
    grad_ball_kernel<<<grid, 256, 0, s>>>(xb, p, n, sg);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reverse pass of the prox (for the unrolled solve's gradient).  One forward
// dual step maps p to p' = P(q), q = p - step grad x~, x~ = max(0, z - lam div p),
// P the pointwise projection onto the unit ball.  Given the adjoint pbar of
// p', the reverse step is
//   qbar = J_P(q) pbar        (J_P = I inside the ball, (I - q^ q^T)/|q| outside)
//   t    = [z - lam div p > 0] * step * div qbar      (adjoint of x~ through grad)
//   pbar_prev = qbar + lam grad t,   zbar += t,
// and the scalar adjoints collect -t . div p (for lam) and -qbar . grad x~ (for
// step).  Each kernel recomputes what it needs from z and the stored p.
__device__ __forceinline__ float tv_div(const float* __restrict__ p1, const float* __restrict__ p2, int i, int j,
                                        int n, size_t idx) {
    float d = 0.0f;
    if (j < n - 1) d += p1[idx];
    if (j > 0) d -= p1[idx - 1];
    if (i < n - 1) d += p2[idx];
    if (i > 0) d -= p2[idx - n];
    return d;
}

// Sum of one value per thread over the 256-thread block, written by thread 0
// to out (fixed order).
__device__ __forceinline__ void block_sum_to(float v, double* out) {
    __shared__ double red[4];
    double d = (double)v;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = d;
    __syncthreads();
    if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
}

// One pixel per thread, 64 x 4 per workgroup (block (bx, by) of a grid gx
// blocks wide); out-of-range threads take part in the block sums with zero.
#define TV_PIXEL                                              \
    const int j = bx * 64 + (threadIdx.x & 63);               \
    const int i = by * 4 + (threadIdx.x >> 6);                \
    const bool in = i < n && j < n;                           \
    const size_t nn = (size_t)n * n, idx = in ? (size_t)i * n + j : 0;
#define TV_SLOT (partial + by * gx + bx)

// x = max(0, z - lam div p): t = mask * xbar; tbar = t, zbar = t; sum -t.div p
__device__ __forceinline__ void tv_bwd_final_body(const float* __restrict__ z, const float* __restrict__ p,
                                                  const float* __restrict__ xbar, int n, float lam,
                                                  float* __restrict__ tbar, float* __restrict__ zbar,
                                                  double* __restrict__ partial, int bx, int by, int gx) {
    TV_PIXEL
    float v = 0.0f;
    if (in) {
        const float d = tv_div(p, p + nn, i, j, n, idx);
        const float t = (z[idx] - lam * d > 0.0f) ? xbar[idx] : 0.0f;
        tbar[idx] = t;
        zbar[idx] = t;
        v = -t * d;
    }
    block_sum_to(v, TV_SLOT);
}

// Reverse of one dual step, first half: pbar = qn + lam grad tn (the adjoint of
// the step's output p), then qbar = J_P(q) pbar written over qn; sum -qbar.grad x~.
__device__ __forceinline__ void tv_bwd_gradproj_body(const float* __restrict__ z, const float* __restrict__ pp,
                                                     float* qn, const float* __restrict__ tn, int n, float lam,
                                                     float step, double* __restrict__ partial, int bx, int by,
                                                     int gx) {
    TV_PIXEL
    float v = 0.0f;
    if (in) {
        const float tc = tn[idx];
        const float b1 = qn[idx] + lam * ((j < n - 1) ? tn[idx + 1] - tc : 0.0f);
        const float b2 = qn[nn + idx] + lam * ((i < n - 1) ? tn[idx + n] - tc : 0.0f);
        const float* p1 = pp;
        const float* p2 = pp + nn;
        const float xc = fmaxf(0.0f, z[idx] - lam * tv_div(p1, p2, i, j, n, idx));
        const float g1 =
            (j < n - 1) ? fmaxf(0.0f, z[idx + 1] - lam * tv_div(p1, p2, i, j + 1, n, idx + 1)) - xc : 0.0f;
        const float g2 =
            (i < n - 1) ? fmaxf(0.0f, z[idx + n] - lam * tv_div(p1, p2, i + 1, j, n, idx + n)) - xc : 0.0f;
        const float q1 = p1[idx] - step * g1, q2 = p2[idx] - step * g2;
        const float nq = sqrtf(q1 * q1 + q2 * q2);
        float r1 = b1, r2 = b2;
        if (nq > 1.0f) {
            const float u1 = q1 / nq, u2 = q2 / nq;
            const float dp = u1 * b1 + u2 * b2;
            r1 = (b1 - u1 * dp) / nq;
            r2 = (b2 - u2 * dp) / nq;
        }
        qn[idx] = r1;
        qn[nn + idx] = r2;
        v = -(r1 * g1 + r2 * g2);
    }
    block_sum_to(v, TV_SLOT);
}

// Second half: t = mask * step * div qbar; tbar = t, zbar += t; sum -t.div p.
__device__ __forceinline__ void tv_bwd_mask_body(const float* __restrict__ z, const float* __restrict__ pp,
                                                 const float* __restrict__ qbar, int n, float lam, float step,
                                                 float* __restrict__ tbar, float* __restrict__ zbar,
                                                 double* __restrict__ partial, int bx, int by, int gx) {
    TV_PIXEL
    float v = 0.0f;
    if (in) {
        const float d = tv_div(pp, pp + nn, i, j, n, idx);
        const float xtb = step * tv_div(qbar, qbar + nn, i, j, n, idx);
        const float t = (z[idx] - lam * d > 0.0f) ? xtb : 0.0f;
        tbar[idx] = t;
        zbar[idx] += t;
        v = -t * d;
    }
    block_sum_to(v, TV_SLOT);
}

// pbar = qbar + lam grad tbar (the adjoint of the warm-start dual field)
__device__ __forceinline__ void tv_bwd_grad_body(const float* __restrict__ qbar, const float* __restrict__ tbar,
                                                 int n, float lam, float* __restrict__ pbar, int bx, int by) {
    TV_PIXEL
    if (!in) return;
    const float tc = tbar[idx];
    const float g1 = (j < n - 1) ? tbar[idx + 1] - tc : 0.0f;
    const float g2 = (i < n - 1) ? tbar[idx + n] - tc : 0.0f;
    pbar[idx] = qbar[idx] + lam * g1;
    pbar[nn + idx] = qbar[nn + idx] + lam * g2;
}

#undef TV_SLOT
#undef TV_PIXEL

// Recorded steps (one table entry per problem): TV prox chunks and the
// reverse kernels.  A TV step of a problem with lam == 0 only writes
// x = max(0, z) (when out[1] is set) and leaves the dual field alone.
__global__ __launch_bounds__(kTvThreads) void step_tv_kernel(const UStep* __restrict__ steps,
                                                             const BlockRef* __restrict__ map) {
    const BlockRef e = map[blockIdx.x];
    if (e.prob < 0) return;
    const UStep& st = steps[e.prob];
    if (!st.active) return;
    const int gx = (st.n + kTvTile - 1) / kTvTile;
    const int bxi = e.local % gx, byi = e.local / gx;
    if (st.lam > 0.f) {
        tv_prox_body<kTvThreads>(st.in[0], st.in[1], st.out[0], st.out[1], st.n, st.lam, st.step, st.steps, bxi, byi,
                                 st.out[2]);
    } else if (st.out[1]) {
        const int c = threadIdx.x & 63, ty = threadIdx.x >> 6;
        const int j = bxi * kTvTile + c;
        for (int r = ty; r < kTvTile; r += kTvThreads / 64) {
            const int i = byi * kTvTile + r;
            if (c < kTvTile && i < st.n && j < st.n) {
                const size_t g = (size_t)i * st.n + j;
                st.out[1][g] = fmaxf(0.f, st.in[0][g]);
            }
        }
    }
}

__global__ __launch_bounds__(256) void step_tv_bwd_kernel(const UStep* __restrict__ steps,
                                                          const BlockRef* __restrict__ map) {
    const BlockRef e = map[blockIdx.x];
    if (e.prob < 0) return;
    const UStep& st = steps[e.prob];
    if (!st.active) return;
    const int gx = (st.n + 63) / 64;
    const int bx = e.local % gx, by = e.local / gx;
    switch (st.kind) {
        case SK_BWD_FINAL:
            tv_bwd_final_body(st.in[0], st.in[1], st.in[2], st.n, st.lam, st.out[0], st.out[1], st.part, bx, by, gx);
            break;
        case SK_BWD_GRADPROJ:
            tv_bwd_gradproj_body(st.in[0], st.in[1], st.out[0], st.in[2], st.n, st.lam, st.step, st.part, bx, by,
                                 gx);
            break;
        case SK_BWD_MASK:
            tv_bwd_mask_body(st.in[0], st.in[1], st.in[2], st.n, st.lam, st.step, st.out[0], st.out[1], st.part, bx,
                             by, gx);
            break;
        default: tv_bwd_grad_body(st.in[0], st.in[1], st.n, st.lam, st.out[0], bx, by); break;
    }
}

hipError_t launch_step_tv(int kind, const UStep* steps, const BlockRef* map, int nblocks, hipStream_t s) {
    switch (kind) {
        case SK_TV: step_tv_kernel<<<nblocks, kTvThreads, 0, s>>>(steps, map); break;
        case SK_BWD_FINAL:
        case SK_BWD_GRADPROJ:
        case SK_BWD_MASK:
        case SK_BWD_GRAD: step_tv_bwd_kernel<<<nblocks, 256, 0, s>>>(steps, map); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int tv_bwd_blocks(int n) { return ((n + 63) / 64) * ((n + 3) / 4); }

hipError_t launch_tv_prox(const float* z, float* p_a, float* p_b, float* x, int n, float lam, float step,
                          int n_iter, float** p_final, hipStream_t s) {
    dim3 grid((n + kTvTile - 1) / kTvTile, (n + kTvTile - 1) / kTvTile);
    float* src = p_a;
    float* dst = p_b;
    int left = n_iter;
    do {
        const int k = left < kTvChunk ? left : kTvChunk;
        left -= k;
        tv_prox_kernel<<<grid, kTvThreads, 0, s>>>(z, src, dst, left == 0 ? x : nullptr, n, lam, step, k);
        std::swap(src, dst);
    } while (left > 0);
    *p_final = src;
    return hipGetLastError();
}

hipError_t launch_tv_finalize(const float* z, const float* p, float* x, int n, float lam, hipStream_t s) {
    dim3 grid((n + 63) / 64, (n + 3) / 4);
    tv_finalize_kernel<<<grid, 256, 0, s>>>(z, p, x, n, lam);
    return hipGetLastError();
}

}  // namespace ctpd
