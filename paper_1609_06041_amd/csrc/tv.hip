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

// One workgroup = 16 waves.  Lane c of every wave is window column c (the
// window is at most 64 columns wide) and wave w owns the window rows
// [w R, w R + R): a thread keeps z and p of its R rows in registers.  The
// left neighbour of p1 and the right neighbour of x~ come from the adjacent
// lane (DPP wave shifts), vertical neighbours from the thread's own rows;
// only the edge rows of a strip pass through LDS.  Every step each wave
// publishes the first row of its p (p1, p2) and the last row of its p2, one
// barrier later reads its neighbours' rows, evaluates x~ on its rows and on
// the row below the strip, and updates its p.  The exchange buffer has two
// parities, so step t + 1 can publish while a slower wave still reads step t.
// Cells outside the image or outside the shrinking valid region are updated
// too (a kept cell never reads them: the image-edge masks drop neighbours
// outside the image, and the halo covers the window edge); a wave whose rows
// all lie outside the valid region of a step skips that step's arithmetic.
// Every multiply-add is an explicit fmaf, so the 512- and 1024-thread forms
// (and every caller) round alike.
constexpr int kTvThreads = 1024;

// Lane c receives lane c - 1 (lane 0 receives 0), and lane c + 1 (lane 63
// receives 0): DPP wave_shr:1 and wave_shl:1.  Every lane of the wave must be
// active at the call.
__device__ __forceinline__ float from_left_lane(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float from_right_lane(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}

// ps_store (optional): the dual field after every step t = 1..steps is also
// written to ps_store + (t - 1) * 2 n^2 (the interior stays valid: the halo
// is one pixel wider than the steps taken).
template <int THREADS>
__device__ __forceinline__ void tv_prox_body(const float* __restrict__ z, const float* __restrict__ p_in,
                                             float* __restrict__ p_out, float* __restrict__ x, int n, float lam,
                                             float step, int steps, int bxi, int byi,
                                             float* __restrict__ ps_store = nullptr, float* __restrict__ xp = nullptr,
                                             float* __restrict__ xTp = nullptr) {
    constexpr int NW = THREADS / 64;
    constexpr int R = (kTvMaxW + NW - 1) / NW;
    // [parity][first-row p1, first-row p2, last-row p2][slot][lane]: wave w
    // writes slot w of the first rows and slot w + 1 of the last row, so slot
    // NW of the first rows and slot 0 of the last row stay zero.
    __shared__ float ex[2][3][NW + 1][64];
    const int H = steps + 1, W = kTvTile + 2 * H;
    const int i0 = byi * kTvTile - H, j0 = bxi * kTvTile - H;
    const int c = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int rb = w * R;
    const bool active = rb < W;
    const int j = j0 + c;
    const bool jin = c < W && j >= 0 && j < n;
    const bool right = j < n - 1, left = j > 0;
    const bool cout = jin && c >= H && c < H + kTvTile;
    const size_t nn = (size_t)n * n;

    float zr[R + 1], p1[R], p2[R];
#pragma unroll
    for (int k = 0; k <= R; ++k) {
        const int r = rb + k, i = i0 + r;
        const bool in = active && jin && r < W && i >= 0 && i < n;
        const size_t g = in ? (size_t)i * n + j : 0;
        zr[k] = in ? z[g] : 0.f;
        if (k < R) {
            p1[k] = in ? p_in[g] : 0.f;
            p2[k] = in ? p_in[nn + g] : 0.f;
        }
    }
    for (int q = 0; q < 2; ++q) {
        if (w == 0) ex[q][2][0][c] = 0.f;
        if (w == NW - 1) {
            ex[q][0][NW][c] = 0.f;
            ex[q][1][NW][c] = 0.f;
        }
        if (!active) {
            ex[q][0][w][c] = 0.f;
            ex[q][1][w][c] = 0.f;
            ex[q][2][w + 1][c] = 0.f;
        }
    }

    // x~ on the strip's rows and the row below it, from p and the rows the
    // neighbouring waves published (pb1/pb2: first row below, pa2: last p2 above)
    auto xtilde_rows = [&](float pb1, float pb2, float pa2, float (&xt)[R + 1]) {
#pragma unroll
        for (int k = 0; k <= R; ++k) {
            const float a1 = k < R ? p1[k] : pb1, a2 = k < R ? p2[k] : pb2;
            const float up2 = k == 0 ? pa2 : p2[k - 1];
            const float l1 = from_left_lane(a1);
            const int r = rb + k, i = i0 + r;
            const float d = ((right ? a1 : 0.f) - (left ? l1 : 0.f)) + (i < n - 1 ? a2 : 0.f) -
                            (i > 0 && r > 0 ? up2 : 0.f);
            xt[k] = fmaxf(0.f, fmaf(-lam, d, zr[k]));
        }
    };

    for (int t = 1; t <= steps; ++t) {
        const int par = t & 1;
        if (active) {
            ex[par][0][w][c] = p1[0];
            ex[par][1][w][c] = p2[0];
            ex[par][2][w + 1][c] = p2[R - 1];
        }
        __syncthreads();
        // rows whose p is still needed after step t: [t, W - t)
        if (active && rb + R > t && rb < W - t) {
            float xt[R + 1];
            xtilde_rows(ex[par][0][w + 1][c], ex[par][1][w + 1][c], ex[par][2][w][c], xt);
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int i = i0 + rb + k;
                const float xr = from_right_lane(xt[k]);
                const float g1 = right ? xr - xt[k] : 0.f;
                const float g2 = (i < n - 1) ? xt[k + 1] - xt[k] : 0.f;
                const float q1 = fmaf(-step, g1, p1[k]), q2 = fmaf(-step, g2, p2[k]);
                const float s2 = fmaf(q1, q1, q2 * q2);
                const float f = s2 > 1.f ? __builtin_amdgcn_rsqf(s2) : 1.f;
                p1[k] = q1 * f;
                p2[k] = q2 * f;
            }
            if (ps_store) {
                float* dst = ps_store + (size_t)(t - 1) * 2 * nn;
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int r = rb + k, i = i0 + r;
                    if (cout && r >= H && r < H + kTvTile && i < n) {
                        const size_t g = (size_t)i * n + j;
                        dst[g] = p1[k];
                        dst[nn + g] = p2[k];
                    }
                }
            }
        }
    }
    const int par = (steps + 1) & 1;
    if (active) ex[par][2][w + 1][c] = p2[R - 1];
    __syncthreads();
    // with xp / xTp the forward projector's padded planes of x are written too
    // (pitch n + 6, three pixels of pad on each side, pads left alone): xp
    // straight, xTp through a tile in LDS so that its rows are stored whole
    __shared__ float tileT[kTvTile][kTvTile + 1];
    const bool planes = x && xp;
    const int P = n + 2 * kPlanePad;
    if (active && rb + R > H && rb < H + kTvTile) {
        float xt[R + 1];
        if (x) xtilde_rows(0.f, 0.f, ex[par][2][w][c], xt);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int r = rb + k, i = i0 + r;
            if (cout && r >= H && r < H + kTvTile && i < n) {
                const size_t g = (size_t)i * n + j;
                p_out[g] = p1[k];
                p_out[nn + g] = p2[k];
                if (x) x[g] = xt[k];
                if (planes) {
                    xp[(size_t)i * P + j + kPlanePad] = xt[k];
                    tileT[c - H][r - H] = xt[k];
                }
            }
        }
    }
    if (planes) {
        __syncthreads();
        // xTp row j0 + a holds column j0 + a of x: tile element (a, b) is x[i0 + b][j0 + a]
        for (int e = threadIdx.x; e < kTvTile * kTvTile; e += THREADS) {
            const int a = e / kTvTile, b = e % kTvTile;
            const int jj = bxi * kTvTile + a, ii = byi * kTvTile + b;
            if (jj < n && ii < n) xTp[(size_t)jj * P + ii + kPlanePad] = tileT[a][b];
        }
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
                                                             float lam, float step, int steps,
                                                             float* __restrict__ xp, float* __restrict__ xTp) {
    tv_prox_body<kTvThreads>(z, p_in, p_out, x, n, lam, step, steps, blockIdx.x, blockIdx.y, nullptr, xp, xTp);
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
                          int n_iter, float** p_final, hipStream_t s, float* xp, float* xTp) {
    dim3 grid((n + kTvTile - 1) / kTvTile, (n + kTvTile - 1) / kTvTile);
    float* src = p_a;
    float* dst = p_b;
    int left = n_iter;
    do {
        const int k = left < kTvChunk ? left : kTvChunk;
        left -= k;
        tv_prox_kernel<<<grid, kTvThreads, 0, s>>>(z, src, dst, left == 0 ? x : nullptr, n, lam, step, k, xp, xTp);
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
