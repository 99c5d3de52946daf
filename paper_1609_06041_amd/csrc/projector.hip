// Joseph ray-driven forward projector A and its exact transpose A^T
// (Sec. 2.1 system matrix; the dominant per-iteration operations of
// Eqs. 18-20 and 29-31).
//
// Both kernels are gathers (no atomics), so results are deterministic.
// Sample positions are computed in float64: in float32 a position of ~500
// pixels carries ~3e-5 pixel of rounding, which alone would exceed a 1e-5
// relative error on non-smooth images; the float64 position costs a few
// full-rate DP instructions per sample on CDNA.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <set>
#include <tuple>
#include <utility>
#include <vector>

#include "internal.h"

namespace ctpd {

// ---------------------------------------------------------------------------
// Padded planes.  Row views read image rows, column views read image columns;
// the forward projector reads both from row-major copies padded with FP_PAD
// zero pixels on each side of every row, so taps outside the image need no
// test:  xp[t][k + FP_PAD] = x[t][k],  xTp[t][k + FP_PAD] = x[k][t],
// pitch n + 2 FP_PAD.
constexpr int FP_PAD = kPlanePad;

// Kernel bodies take their block coordinates as arguments so that the single
// launches and the batched launches (one flattened grid over many problems)
// share them.
template <typename T>
__device__ __forceinline__ void pad_planes_body(const T* __restrict__ in, T* __restrict__ xp, T* __restrict__ xTp,
                                                int n, int bxi, int byi) {
    __shared__ T tile[32][33];
    const int bx = bxi * 32, by = byi * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    const int P = n + 2 * FP_PAD;
    for (int r = ty; r < 32; r += 8) {
        const int iy = by + r, ix = bx + tx;
        T val = T(0);
        if (iy < n && ix < n) val = in[(size_t)iy * n + ix];
        tile[r][tx] = val;
        if (iy < n && ix < n) xp[(size_t)iy * P + ix + FP_PAD] = val;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int ox = bx + r, oy = by + tx;   // xT[ox][oy] = x[oy][ox]
        if (ox < n && oy < n) xTp[(size_t)ox * P + oy + FP_PAD] = tile[tx][r];
    }
    // zero pads: the blocks of the first block column write the pad columns of their rows
    if (bxi == 0) {
        for (int e = threadIdx.x; e < 32 * 2 * FP_PAD; e += 256) {
            const int r = by + e / (2 * FP_PAD), q = e % (2 * FP_PAD);
            const int col = q < FP_PAD ? q : n + q;
            if (r < n) {
                xp[(size_t)r * P + col] = T(0);
                xTp[(size_t)r * P + col] = T(0);
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void pad_planes_kernel(const T* __restrict__ in, T* __restrict__ xp,
                                                         T* __restrict__ xTp, int n) {
    pad_planes_body<T>(in, xp, xTp, n, blockIdx.x, blockIdx.y);
}

template <typename T>
hipError_t launch_pad_planes(const T* x, T* xp, T* xTp, int n, hipStream_t s) {
    dim3 grid((n + 31) / 32, (n + 31) / 32);
    pad_planes_kernel<T><<<grid, 256, 0, s>>>(x, xp, xTp, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Forward projection: one lane per ray (v, u).  A wave holds the rays of 64
// consecutive bins of one view and steps through the union of their step
// ranges together (the row offset is then a scalar); a lane outside its own
// range clamps its column into the zero pad (one unsigned min: negative
// columns wrap to the right pad) and so adds exact zeros.
//
// Positions are 32.32 fixed point, biased by FP_PAD so that the integer part
// is the padded column, and are defined per segment of FW_SEG rows: at row t
// of the segment that starts at row s0 the position is
//     S + (t - s0) d   (mod 2^64),   S = round((s0 st + base + FP_PAD) 2^32),
// d = round(st 2^32), with S and d from float64 -- exact integer arithmetic,
// so every form computes the same positions whatever order it visits the rows
// in (rounding of d adds at most FW_SEG 2^-33 pixel).  A ray's sum is formed
// per segment in row order from zero, and the segment sums are added in
// segment order; segments with no step of the wave's range are skipped, and
// out-of-range steps add exact zeros.  The gather, split and slab forms below
// all follow this, so their results are equal bit for bit.
typedef float v2f_t __attribute__((ext_vector_type(2)));
typedef double v2d_t __attribute__((ext_vector_type(2)));

constexpr int FW_SEG = 32;

__device__ __forceinline__ unsigned long long seg_position(double base, double st, int s0) {
    return (unsigned long long)llrint((fma((double)s0, st, base) + FP_PAD) * 4294967296.0);
}

__device__ __forceinline__ void load_taps(const __amdgpu_buffer_rsrc_t& rs, unsigned voff, int soff, float& a,
                                          float& b) {
    const v2f_t ab = __builtin_bit_cast(v2f_t, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
    a = ab.x;
    b = ab.y;
}

__device__ __forceinline__ void load_taps(const __amdgpu_buffer_rsrc_t& rs, unsigned voff, int soff, double& a,
                                          double& b) {
    const v2d_t ab = __builtin_bit_cast(v2d_t, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
    a = ab.x;
    b = ab.y;
}

// Buffer resource word 3 for raw (untyped) buffers on CDNA.
constexpr int kBufferRsrcWord3 = 0x00020000;
constexpr int FW_BATCH = 8;

// Ray u of view g: its sample position at step 0 (base; rays past the last
// bin reuse the last bin's) and the steps [t0, t1] whose sample lies within
// one step of (-1, n), as the union over the wave (wave-uniform; empty when
// t0 > t1).
__device__ __forceinline__ void wave_ray_span(const ViewGeom& g, int u, int n, int nb, double& base, int& t0,
                                              int& t1) {
    base = fma((double)min(u, nb - 1), g.su, g.s0);
    t0 = n;
    t1 = -1;
    if (u < nb) {
        if (g.st != 0.0) {
            const double ta = (-1.0 - base) / g.st, tb = ((double)n - base) / g.st;
            const double lo = fmin(fmax(fmin(ta, tb), -1.0), (double)n);
            const double hi = fmin(fmax(fmax(ta, tb), -1.0), (double)n);
            t0 = max(0, (int)floor(lo));
            t1 = min(n - 1, (int)ceil(hi));
        } else if (base > -1.0 && base < (double)n) {
            t0 = 0;
            t1 = n - 1;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        t0 = min(t0, __shfl_xor(t0, off));
        t1 = max(t1, __shfl_xor(t1, off));
    }
    t0 = __builtin_amdgcn_readfirstlane(t0);
    t1 = __builtin_amdgcn_readfirstlane(t1);
}

// Steps [ta, tb] of one segment through raw buffer loads of both taps (8
// bytes, 16 for float64) of the padded plane; acc_a sums the left taps and
// acc_d the low position word times (right - left).
template <typename T, int FB>
__device__ __forceinline__ void gather_segment(const __amdgpu_buffer_rsrc_t& rs, unsigned long long sfix,
                                               unsigned long long dfix, int ta, int tb, int rowstride,
                                               unsigned cmax, T& acc_a, T& acc_d) {
    int rowb = ta * rowstride, t = ta;
    for (; t + FB - 1 <= tb; t += FB) {
        unsigned off[FB];
        T lf[FB], a[FB], b[FB];
#pragma unroll
        for (int q = 0; q < FB; ++q) {
            off[q] = min((unsigned)(sfix >> 32), cmax) * (unsigned)sizeof(T);
            lf[q] = (T)(unsigned)sfix;
            sfix += dfix;
        }
#pragma unroll
        for (int q = 0; q < FB; ++q) load_taps(rs, off[q], rowb + q * rowstride, a[q], b[q]);
#pragma unroll
        for (int q = 0; q < FB; ++q) {
            acc_a += a[q];
            acc_d = fma(lf[q], b[q] - a[q], acc_d);
        }
        rowb += FB * rowstride;
    }
    for (; t <= tb; ++t) {
        T a, b;
        load_taps(rs, min((unsigned)(sfix >> 32), cmax) * (unsigned)sizeof(T), rowb, a, b);
        acc_a += a;
        acc_d = fma((T)(unsigned)sfix, b - a, acc_d);
        sfix += dfix;
        rowb += rowstride;
    }
}

// The ray's value len (acc_a + acc_d 2^-32), or with rb the residual
// value - rb - rw .* rm (rw null: value - rb), the arithmetic of the filter prologues.
template <typename T>
__device__ __forceinline__ T ray_value(T acc_a, T acc_d, double len, size_t idx, const T* __restrict__ rb,
                                       const T* __restrict__ rw, const T* __restrict__ rm) {
    T q = (acc_a + acc_d * (T)2.3283064365386962890625e-10) * (T)len;
    if (rb) q = rw ? fma(-rw[idx], rm[idx], q - rb[idx]) : q - rb[idx];
    return q;
}

// Gather form: 256 consecutive bins of one view per workgroup.
template <typename T, int FB = FW_BATCH>
__device__ __forceinline__ void forward_body(const T* __restrict__ xp, const T* __restrict__ xTp, T* __restrict__ y,
                                             const ViewGeom* __restrict__ views, int n, int nb, int bxi, int v,
                                             const T* __restrict__ rb = nullptr, const T* __restrict__ rw = nullptr,
                                             const T* __restrict__ rm = nullptr) {
    const int u = bxi * 256 + threadIdx.x;
    const ViewGeom g = views[v];
    const int P = n + 2 * FP_PAD;
    double base;
    int t0, t1;
    wave_ray_span(g, u, n, nb, base, t0, t1);
    const unsigned long long dfix = (unsigned long long)llrint(g.st * 4294967296.0);
    const unsigned cmax = (unsigned)(P - 2);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(g.row ? xp : xTp), (short)0, (int)((size_t)n * P * sizeof(T)), kBufferRsrcWord3);
    T tot_a = T(0), tot_d = T(0);
    for (int s0 = t0 - t0 % FW_SEG; s0 <= t1; s0 += FW_SEG) {
        const int ta = max(t0, s0), tb = min(t1, s0 + FW_SEG - 1);
        T acc_a = T(0), acc_d = T(0);
        gather_segment<T, FB>(rs, seg_position(base, g.st, s0) + (unsigned long long)(ta - s0) * dfix, dfix, ta, tb,
                              P * (int)sizeof(T), cmax, acc_a, acc_d);
        tot_a += acc_a;
        tot_d += acc_d;
    }
    if (u < nb) {
        const size_t idx = (size_t)v * nb + u;
        y[idx] = ray_value<T>(tot_a, tot_d, g.len, idx, rb, rw, rm);
    }
}

__global__ __launch_bounds__(256) void forward_resid_kernel(const float* __restrict__ xp,
                                                            const float* __restrict__ xTp, float* __restrict__ y,
                                                            const ViewGeom* __restrict__ views, int n, int nb,
                                                            const float* __restrict__ rb,
                                                            const float* __restrict__ rw,
                                                            const float* __restrict__ rm) {
    forward_body<float>(xp, xTp, y, views, n, nb, blockIdx.x, blockIdx.y, rb, rw, rm);
}

hipError_t launch_forward_resid(const float* xp, const float* xTp, float* y, const ViewGeom* views, int n, int m,
                                int nb, const float* rb, const float* rw, const float* rm, hipStream_t s) {
    dim3 grid((nb + 255) / 256, m);
    forward_resid_kernel<<<grid, 256, 0, s>>>(xp, xTp, y, views, n, nb, rb, rw, rm);
    return hipGetLastError();
}

// Split form, for scans with few views: a workgroup of kSplitWaves waves takes
// one (view, 64-bin block); wave w forms the sums of segments w, w + W, ...,
// and wave 0 adds them in segment order.  The work of a few-view scan is then
// spread over m * nblk * W waves instead of m * nblk.
constexpr int kSplitWaves = 16, kSplitFB = 4, kSplitMaxSeg = 64;

__global__ __launch_bounds__(64 * kSplitWaves) void forward_split_kernel(
    const float* __restrict__ xp, const float* __restrict__ xTp, float* __restrict__ y,
    const ViewGeom* __restrict__ views, const int* __restrict__ order, int n, int nb, int nblk,
    const float* __restrict__ rb, const float* __restrict__ rw, const float* __restrict__ rm) {
    __shared__ float part[2][kSplitMaxSeg][64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int task = order ? order[blockIdx.x] : (int)blockIdx.x;
    const int v = task / nblk, blk = task - v * nblk;
    const int u = blk * 64 + lane;
    const ViewGeom g = views[v];
    const int P = n + 2 * FP_PAD;
    double base;
    int t0, t1;
    wave_ray_span(g, u, n, nb, base, t0, t1);
    const unsigned long long dfix = (unsigned long long)llrint(g.st * 4294967296.0);
    const unsigned cmax = (unsigned)(P - 2);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(g.row ? xp : xTp), (short)0, (int)((size_t)n * P * sizeof(float)), kBufferRsrcWord3);
    const int ns = (n + FW_SEG - 1) / FW_SEG;
    for (int sg = wv; sg < ns; sg += kSplitWaves) {
        const int s0 = sg * FW_SEG;
        const int ta = max(t0, s0), tb = min(t1, s0 + FW_SEG - 1);
        float acc_a = 0.f, acc_d = 0.f;
        if (ta <= tb)
            gather_segment<float, kSplitFB>(rs, seg_position(base, g.st, s0) + (unsigned long long)(ta - s0) * dfix,
                                            dfix, ta, tb, P * (int)sizeof(float), cmax, acc_a, acc_d);
        part[0][sg][lane] = acc_a;
        part[1][sg][lane] = acc_d;
    }
    __syncthreads();
    if (wv == 0 && u < nb) {
        // segments outside the range hold zeros: adding them changes no bit
        float tot_a = 0.f, tot_d = 0.f;
        const int sa = t0 / FW_SEG, sb = t1 < 0 ? -1 : t1 / FW_SEG;
        for (int sg = sa; sg <= sb; ++sg) {
            tot_a += part[0][sg][lane];
            tot_d += part[1][sg][lane];
        }
        const size_t idx = (size_t)v * nb + u;
        y[idx] = ray_value<float>(tot_a, tot_d, g.len, idx, rb, rw, rm);
    }
}

// Slab form (float32, one problem, scans with many views).  A workgroup of
// 12 waves takes 36 (view, 64-bin block) tasks of views of one orientation,
// three per wave, and streams that orientation's padded plane through LDS in
// slabs of FW_SEG rows (one segment each): the next slab is copied straight
// from global memory into the other half of a double buffer (16 bytes a lane,
// no registers) while the current one is read.  Each wave steps its three
// rays together over the union of their row ranges within the slab, so every
// step issues three independent pairs of LDS reads.  The plane needs 16 bytes
// of slack after its end (the copy moves whole 16-byte words).
constexpr int kSlabWaves = 12, kSlabThreads = 64 * kSlabWaves, kSlabTPW = 3, kSlabTasks = kSlabWaves * kSlabTPW;
constexpr int kSlabFB = 2;
constexpr size_t kSlabMaxLds = 160 * 1024;

size_t forward_slab_lds(int n) { return (size_t)2 * FW_SEG * (n + 2 * FP_PAD) * sizeof(float); }
bool forward_slab_fits(int n) { return forward_slab_lds(n) <= kSlabMaxLds; }
int forward_slab_tasks_per_group() { return kSlabTasks; }

// tk: the group's kSlabTasks task entries
__device__ __forceinline__ void forward_slab_body(const float* __restrict__ xp, const float* __restrict__ xTp,
                                                  float* __restrict__ y, const ViewGeom* __restrict__ views,
                                                  const int* __restrict__ tk, int n, int nb,
                                                  const float* __restrict__ rb, const float* __restrict__ rw,
                                                  const float* __restrict__ rm) {
    constexpr int R = FW_SEG, J = kSlabTPW, FB = kSlabFB;
    extern __shared__ __align__(16) float slabs[];
    const int P = n + 2 * FP_PAD;
    const int SL = R * P;   // floats per buffer, a multiple of 4
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const float* plane = views[tk[0] >> 6].row ? xp : xTp;
    const unsigned cmax = (unsigned)(P - 2);
    unsigned long long dfix[J];
    double bs[J], sts[J];
    float tot_a[J], tot_d[J];
    int vv[J], uu[J];
    int tu0 = n, tu1 = -1;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int e = tk[wv + kSlabWaves * j];
        const int v = e >= 0 ? e >> 6 : -1;
        const int u = e >= 0 ? (e & 63) * 64 + lane : nb;
        vv[j] = v;
        uu[j] = u;
        tot_a[j] = tot_d[j] = 0.f;
        double base = -1000.0, st = 0.0;   // a missing task reads the pad
        int t0 = n, t1 = -1;
        if (v >= 0) {
            const ViewGeom g = views[v];
            st = g.st;
            wave_ray_span(g, u, n, nb, base, t0, t1);
        }
        bs[j] = base;
        sts[j] = st;
        dfix[j] = (unsigned long long)llrint(st * 4294967296.0);
        tu0 = min(tu0, t0);
        tu1 = max(tu1, t1);
    }
    // rows [r0, r0 + R) of the plane into buffer b, 16 bytes a lane
    auto copy = [&](int r0, int b) {
        const int cnt4 = (min(R, n - r0) * P + 3) / 4;
        const float* src = plane + (size_t)r0 * P;
        for (int i0 = wv * 64; i0 < cnt4; i0 += kSlabThreads) {
            if (i0 + lane < cnt4)
                __builtin_amdgcn_global_load_lds((const void*)(src + 4 * (i0 + lane)),
                                                 (lds_void_t*)(slabs + b * SL + 4 * i0), 16, 0, 0);
        }
    };
    copy(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    int buf = 0;
    for (int r0 = 0; r0 < n; r0 += R) {
        if (r0 + R < n) copy(r0 + R, buf ^ 1);
        const float* slab = slabs + buf * SL;
        const int ta = max(tu0, r0), tb = min(tu1, min(n, r0 + R) - 1);
        if (ta <= tb) {
            unsigned long long sfix[J];
            float acc_a[J], acc_d[J];
#pragma unroll
            for (int j = 0; j < J; ++j) {
                sfix[j] = seg_position(bs[j], sts[j], r0) + (unsigned long long)(ta - r0) * dfix[j];
                acc_a[j] = acc_d[j] = 0.f;
            }
            int t = ta;
            for (; t + FB - 1 <= tb; t += FB) {
                unsigned off[FB][J];
                float lf[FB][J], a[FB][J], b[FB][J];
#pragma unroll
                for (int q = 0; q < FB; ++q)
#pragma unroll
                    for (int j = 0; j < J; ++j) {
                        off[q][j] = min((unsigned)(sfix[j] >> 32), cmax) + (unsigned)((t - r0 + q) * P);
                        lf[q][j] = (float)(unsigned)sfix[j];
                        sfix[j] += dfix[j];
                    }
#pragma unroll
                for (int q = 0; q < FB; ++q)
#pragma unroll
                    for (int j = 0; j < J; ++j) {
                        a[q][j] = slab[off[q][j]];
                        b[q][j] = slab[off[q][j] + 1];
                    }
#pragma unroll
                for (int q = 0; q < FB; ++q)
#pragma unroll
                    for (int j = 0; j < J; ++j) {
                        acc_a[j] += a[q][j];
                        acc_d[j] = fma(lf[q][j], b[q][j] - a[q][j], acc_d[j]);
                    }
            }
            for (; t <= tb; ++t) {
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    const unsigned off = min((unsigned)(sfix[j] >> 32), cmax) + (unsigned)((t - r0) * P);
                    const float a = slab[off], b = slab[off + 1];
                    acc_a[j] += a;
                    acc_d[j] = fma((float)(unsigned)sfix[j], b - a, acc_d[j]);
                    sfix[j] += dfix[j];
                }
            }
#pragma unroll
            for (int j = 0; j < J; ++j) {
                tot_a[j] += acc_a[j];
                tot_d[j] += acc_d[j];
            }
        }
        // the next slab has landed and every wave is done with this one
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
        if (vv[j] >= 0 && uu[j] < nb) {
            const size_t idx = (size_t)vv[j] * nb + uu[j];
            y[idx] = ray_value<float>(tot_a[j], tot_d[j], views[vv[j]].len, idx, rb, rw, rm);
        }
    }
}

__global__ __launch_bounds__(kSlabThreads) void forward_slab_kernel(const float* __restrict__ xp,
                                                                    const float* __restrict__ xTp,
                                                                    float* __restrict__ y,
                                                                    const ViewGeom* __restrict__ views,
                                                                    const int* __restrict__ tasks, int n, int nb,
                                                                    const float* __restrict__ rb,
                                                                    const float* __restrict__ rw,
                                                                    const float* __restrict__ rm) {
    forward_slab_body(xp, xTp, y, views, tasks + (size_t)blockIdx.x * kSlabTasks, n, nb, rb, rw, rm);
}

// The batch's slab projector: one workgroup per (problem, task group), the
// residual A x - b - W^-1 mu[rot] into q.
__global__ __launch_bounds__(kSlabThreads) void forward_slab_batched(const BatchItem* __restrict__ items,
                                                                     const BlockRef* __restrict__ map, int rot) {
    const BlockRef e = map[blockIdx.x];
    if (e.prob < 0) return;
    const BatchItem& it = items[e.prob];
    forward_slab_body(it.xp, it.xTp, it.q, it.views, it.tasks + (size_t)e.local * kSlabTasks, it.n, it.nb, it.b,
                      it.lowdose ? it.winv : nullptr, it.mu[rot]);
}

// lift the dynamic LDS limit of the slab kernels to the chip's 160 KB, once
static hipError_t slab_lds_attributes() {
    static std::once_flag once;
    static hipError_t attr = hipSuccess;
    std::call_once(once, [] {
        attr = hipFuncSetAttribute((const void*)forward_slab_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)kSlabMaxLds);
        if (attr == hipSuccess)
            attr = hipFuncSetAttribute((const void*)forward_slab_batched, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kSlabMaxLds);
    });
    return attr;
}

hipError_t launch_forward_slab(const float* xp, const float* xTp, float* y, const ViewGeom* views, const int* tasks,
                               int ngroups, int n, int nb, const float* rb, const float* rw, const float* rm,
                               hipStream_t s) {
    const hipError_t attr = slab_lds_attributes();
    if (attr != hipSuccess) return attr;
    forward_slab_kernel<<<ngroups, kSlabThreads, forward_slab_lds(n), s>>>(xp, xTp, y, views, tasks, n, nb, rb, rw,
                                                                        rm);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Task schedule of the slab form (host).  A group's waves meet at a barrier
// after every slab, so per slab a group takes as long as its busiest SIMD
// (waves wv, wv + 4 and wv + 8 share SIMD wv mod 4), and a wave as long as
// the union of its three rays' step ranges within the slab.  The tasks of
// one orientation are sorted by step range and cut into triples of near-equal
// ranges (one wave each); the triples are dealt, heaviest first, to the SIMD
// slot whose per-slab load then peaks lowest (ties: the less loaded, then the
// first), so that a SIMD holds e.g. one full-range wave beside a prefix and a
// suffix wave of complementary lengths.  The orientations share
// max(min_groups, the fewest groups that hold them) groups in proportion to
// their work.  Which wave computes a ray changes none of its bits.
constexpr int kSlabMinGroups = 150, kSlabSimds = 4, kSlabSlots = kSlabWaves / kSlabSimds;
static_assert(kSlabWaves % kSlabSimds == 0, "waves per SIMD");

// host copy of wave_ray_span over the 64 rays of block b (a cost estimate
// only).  With st != 0 both ends of a ray's range are monotone in u, so the
// first and last ray of the block bound the union.
static void slab_task_span(const ViewGeom& g, int b, int n, int nb, int& t0, int& t1) {
    t0 = n;
    t1 = -1;
    auto ray = [&](int u) {
        const double base = std::fma((double)u, g.su, g.s0);
        if (g.st != 0.0) {
            const double ta = (-1.0 - base) / g.st, tb = ((double)n - base) / g.st;
            const double lo = std::fmin(std::fmax(std::fmin(ta, tb), -1.0), (double)n);
            const double hi = std::fmin(std::fmax(std::fmax(ta, tb), -1.0), (double)n);
            t0 = std::min(t0, std::max(0, (int)std::floor(lo)));
            t1 = std::max(t1, std::min(n - 1, (int)std::ceil(hi)));
        } else if (base > -1.0 && base < (double)n) {
            t0 = 0;
            t1 = n - 1;
        }
    };
    const int ua = b * 64, ue = std::min(b * 64 + 63, nb - 1);
    if (g.st != 0.0) {
        ray(ua);
        ray(ue);
    } else {
        for (int u = ua; u <= ue; ++u) ray(u);
    }
}

std::vector<int> forward_slab_schedule(const ViewGeom* hv, int m, int n, int nb, int min_groups, int* dense) {
    constexpr int W = kSlabWaves, J = kSlabTPW;
    const int nblk = (nb + 63) / 64, ns = (n + FW_SEG - 1) / FW_SEG;
    struct Job {
        int task[J];
        long total;
        std::vector<int> load;   // steps per slab, times J
    };
    std::vector<Job> jobs[2];
    double work[2] = {0.0, 0.0};
    for (int o = 0; o < 2; ++o) {
        struct Span { int id, t0, t1; };
        std::vector<Span> ts;
        for (int v = 0; v < m; ++v)
            if (hv[v].row == 1 - o)   // row views first
                for (int b = 0; b < nblk; ++b) {
                    Span sp{v * 64 + b, 0, 0};
                    slab_task_span(hv[v], b, n, nb, sp.t0, sp.t1);
                    ts.push_back(sp);
                }
        std::stable_sort(ts.begin(), ts.end(), [](const Span& a, const Span& b) {
            const bool ea = a.t1 < a.t0, eb = b.t1 < b.t0;
            if (ea != eb) return eb;
            return a.t0 != b.t0 ? a.t0 < b.t0 : a.t1 < b.t1;
        });
        for (size_t i = 0; i < ts.size(); i += J) {
            Job jb;
            int t0 = n, t1 = -1;
            for (int j = 0; j < J; ++j) {
                const bool has = i + j < ts.size();
                jb.task[j] = has ? ts[i + j].id : -1;
                if (has && ts[i + j].t1 >= ts[i + j].t0) {
                    t0 = std::min(t0, ts[i + j].t0);
                    t1 = std::max(t1, ts[i + j].t1);
                }
            }
            jb.load.assign(ns, 0);
            jb.total = 0;
            for (int s = 0; s < ns; ++s) {
                const int a = std::max(t0, s * FW_SEG), b = std::min(t1, s * FW_SEG + FW_SEG - 1);
                jb.load[s] = b >= a ? J * (b - a + 1) : 0;
                jb.total += jb.load[s];
            }
            work[o] += (double)jb.total;
            jobs[o].push_back(std::move(jb));
        }
    }
    int need[2], G[2];
    for (int o = 0; o < 2; ++o) need[o] = ((int)jobs[o].size() + W - 1) / W;
    if (dense) *dense = need[0] + need[1];
    const int total = std::max(min_groups, need[0] + need[1]);
    if (!need[0] || !need[1]) {
        G[0] = need[0] ? total : 0;
        G[1] = need[1] ? total : 0;
    } else {
        const double share = work[0] + work[1] > 0.0 ? work[0] / (work[0] + work[1]) : 0.5;
        G[0] = std::min(std::max((int)std::lround(share * total), need[0]), total - need[1]);
        G[1] = total - G[0];
    }
    std::vector<int> out;
    int ng[2] = {0, 0};   // groups emitted per orientation
    for (int o = 0; o < 2; ++o) {
        if (!G[o]) continue;
        const int B = G[o] * kSlabSimds;
        std::vector<int> order(jobs[o].size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return jobs[o][a].total > jobs[o][b].total; });
        std::vector<int> load((size_t)B * ns, 0), cnt(B, 0), slot((size_t)B * kSlabSlots, -1), peak(B, 0);
        std::vector<long> tot(B, 0);
        // open bins ordered by (own peak, total, index): a bin's new peak is at least
        // its own, so the scan stops at the first bin whose own peak exceeds the best
        std::set<std::tuple<int, long, int>> open;
        int next_empty = 0;
        for (int q : order) {
            const Job& jb = jobs[o][q];
            int best = -1;
            if (next_empty < B) {
                best = next_empty++;   // an empty bin: the lowest possible peak and total
            } else {
                int best_peak = 0;
                long best_tot = 0;
                for (const auto& e : open) {
                    const int k = std::get<2>(e);
                    if (best >= 0 && std::get<0>(e) > best_peak) break;
                    int pk = 0;
                    for (int s = 0; s < ns; ++s) pk = std::max(pk, load[(size_t)k * ns + s] + jb.load[s]);
                    if (best < 0 || pk < best_peak || (pk == best_peak && (tot[k] < best_tot ||
                                                                           (tot[k] == best_tot && k < best)))) {
                        best = k;
                        best_peak = pk;
                        best_tot = tot[k];
                    }
                }
                open.erase({peak[best], tot[best], best});
            }
            for (int s = 0; s < ns; ++s) {
                load[(size_t)best * ns + s] += jb.load[s];
                peak[best] = std::max(peak[best], load[(size_t)best * ns + s]);
            }
            tot[best] += jb.total;
            slot[(size_t)best * kSlabSlots + cnt[best]++] = q;
            if (cnt[best] < kSlabSlots) open.insert({peak[best], tot[best], best});
        }
        // SIMD slot c of SIMD k is wave k + 4 c; an empty bin takes the next
        // job before any other bin does, so a group is empty exactly when its
        // SIMD 0 bin is, and then so are the groups after it
        for (int g = 0; g < G[o]; ++g) {
            if (cnt[g * kSlabSimds] == 0) break;
            const size_t base = out.size();
            out.resize(base + (size_t)W * J, -1);
            for (int k = 0; k < kSlabSimds; ++k)
                for (int c = 0; c < kSlabSlots; ++c) {
                    const int q = slot[(size_t)(g * kSlabSimds + k) * kSlabSlots + c];
                    if (q < 0) continue;
                    const int wv = k + kSlabSimds * c;
                    for (int j = 0; j < J; ++j) out[base + wv + (size_t)W * j] = jobs[o][q].task[j];
                }
            ++ng[o];
        }
    }
    // Workgroup b runs on XCD b mod 8: groups of orientation 0 go to
    // positions b mod 8 < 4 and those of orientation 1 to the others (either
    // taking the other's positions once it has none left), so each padded
    // plane is pulled into four XCDs' L2 instead of all eight.  Which
    // workgroup runs a group changes no ray's sum.
    const size_t GS = (size_t)W * J;
    std::vector<int> xcd(out.size());
    int i0 = 0, i1 = 0;
    for (int b = 0; b < ng[0] + ng[1]; ++b) {
        const bool first = (b & 7) < 4;
        const int g = ((first && i0 < ng[0]) || i1 >= ng[1]) ? i0++ : ng[0] + i1++;
        std::copy(out.begin() + (size_t)g * GS, out.begin() + (size_t)(g + 1) * GS, xcd.begin() + (size_t)b * GS);
    }
    return xcd;
}

// The split form's workgroup order: the (view, block) tasks by decreasing step
// range.  The first workgroups of a launch take one compute unit each and the
// rest double up behind them, so the heavy tasks go first and the light ones
// (blocks at the detector's edges) share compute units with them.
std::vector<int> forward_split_order(const ViewGeom* hv, int m, int n, int nb) {
    const int nblk = (nb + 63) / 64;
    std::vector<std::pair<int, int>> w;
    w.reserve((size_t)m * nblk);
    for (int v = 0; v < m; ++v)
        for (int b = 0; b < nblk; ++b) {
            int t0, t1;
            slab_task_span(hv[v], b, n, nb, t0, t1);
            w.push_back({-std::max(0, t1 - t0 + 1), v * nblk + b});
        }
    std::stable_sort(w.begin(), w.end());
    std::vector<int> out(w.size());
    for (size_t i = 0; i < w.size(); ++i) out[i] = w[i].second;
    return out;
}

bool forward_slab_preferred(int dense_groups, int n) {
    return dense_groups >= kSlabMinGroups && forward_slab_fits(n);
}

// The form for the geometry (all three give the same bits): the slab form
// when it was preferred for the geometry (ngroups > 0), else the split form,
// else the gather form (images beyond the split form's segment table).
hipError_t launch_forward_auto(const float* xp, const float* xTp, float* y, const ViewGeom* views, const int* tasks,
                               int ngroups, int n, int m, int nb, const float* rb, const float* rw, const float* rm,
                               hipStream_t s) {
    if (tasks && ngroups > 0)
        return launch_forward_slab(xp, xTp, y, views, tasks, ngroups, n, nb, rb, rw, rm, s);
    if (n <= kSplitMaxSeg * FW_SEG) {
        const int nblk = (nb + 63) / 64;
        forward_split_kernel<<<m * nblk, 64 * kSplitWaves, 0, s>>>(xp, xTp, y, views, tasks, n, nb, nblk, rb, rw,
                                                                 rm);
        return hipGetLastError();
    }
    return launch_forward_resid(xp, xTp, y, views, n, m, nb, rb, rw, rm, s);
}

template <typename T>
__global__ __launch_bounds__(256) void forward_kernel(const T* __restrict__ xp, const T* __restrict__ xTp,
                                                      T* __restrict__ y, const ViewGeom* __restrict__ views,
                                                      int n, int nb) {
    forward_body<T>(xp, xTp, y, views, n, nb, blockIdx.x, blockIdx.y);
}

template <typename T>
hipError_t launch_forward(const T* xp, const T* xTp, T* y, const ViewGeom* views, int n, int m, int nb,
                          hipStream_t s) {
    dim3 grid((nb + 255) / 256, m);
    forward_kernel<T><<<grid, 256, 0, s>>>(xp, xTp, y, views, n, nb);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Transpose of the forward projector as a pixel-driven gather.  For pixel
// (X, Y) and view v the Joseph weights of A are the hat function
// max(0, 1 - |u - t|/s_v)/s_v of the distance between bin u and the pixel's
// bin coordinate t = X cos + Y sin + (nb-1)/2, with s_v = |cos| (row views)
// or |sin| (column views) <= 1, so only bins floor(t), floor(t)+1 carry
// weight.  out = alpha * xin + beta * A^T (c1 y1 + c2 y2).
//
// Workgroup: a 32 x 32 pixel tile, G view streams of SL lanes; stream h
// takes the views h, h+G, h+2G, ... in chunks of VC and its lane (tx, ty)
// owns the pixels (x0 + tx, y0 + ty + RS j), j = 0..PJ-1.  For each chunk
// of views the stream stages, per view, the 48 bins starting one below the
// tile's lowest bin coordinate (the tile spans at most 31 sqrt(2) + 2 bins),
// zero outside the detector, so the inner loop reads LDS without bounds
// tests.  The next chunk's bins are loaded into registers while the current
// chunk is used.  The streams are summed through LDS at the end in a fixed
// order (deterministic).  Per view the stream also tabulates the bin
// positions of the tile's first row and the row increments, so a lane's
// positions take only 64-bit adds.  The inner loop reads from LDS 8 bytes
// of taps per (pixel, view) plus the view's 32 bytes of tables per lane,
// which the PJ pixels of a lane share (with 4 pixels a lane those reads
// bound the loop; with 16 the VALU work and latency do).
constexpr int AT_T = 32;
constexpr int AT_THREADS = 1024;   // 16 waves: a 512^2 image has one tile per CU
constexpr int AT_W = 48;

// Stream layouts.  Stream h takes every G-th view, so with few views the
// sixteen streams of the float layout hold a view or two each and the
// per-tile costs (staging the windows, the stream reduction) dominate: float
// scans with fewer than kAtFewViews views use eight streams of eight pixels
// a lane (32 views at 512^2: 10.0 -> 7.4 us per call; 720 views keep the
// sixteen streams, 62 against 67 us).  Every launch (single, batched, the
// unrolled steps) picks the layout by the same rule, so their results stay
// equal bit for bit.
struct AtF16 {
    static constexpr int G = 16;   // view streams per tile, one wave each
    static constexpr int PJ = 16;  // pixels per lane, one column
    static constexpr int VC = 8;   // views per chunk
    static constexpr int VQ = 1;   // views per inner pass
};
struct AtF8 {
    static constexpr int G = 8;
    static constexpr int PJ = 8;
    static constexpr int VC = 8;
    static constexpr int VQ = 1;
};
struct AtD8 {
    static constexpr int G = 8;
    static constexpr int PJ = 8;
    static constexpr int VC = 8;
    static constexpr int VQ = 2;
};
constexpr int kAtFewViews = 128;
__host__ __device__ inline bool at_few_views(int m) { return m < kAtFewViews; }

template <typename T, typename CFG>
struct AtLds {
    static constexpr int RS = AT_T / CFG::PJ;
    // the staged bins, each already multiplied by its view's len (first, at
    // LDS offset zero, so the per-view bases fold into the read instructions'
    // offsets)
    T win[CFG::G][CFG::VC][AT_W];
    // per view of the staged chunk, in 32.32 fixed point relative to the
    // window: colt[i][tx] = t of pixel (x0 + tx, y0), rowt[i][r] = r * (the
    // per-row increment), r = 0..RS -- so a lane's positions are
    // colt[tx] + rowt[ty] + j rowt[RS] (adds only)
    long long colt[CFG::G][CFG::VC][AT_T];
    long long rowt[CFG::G][CFG::VC][RS + 1];
    // the hat weights over len: 1 - f prate (left bin) and poff + f prate
    // (right bin), f the 32-bit fraction, prate = len2 / (len 2^32), poff = 1 - len2 / len
    T prate[CFG::G][CFG::VC], poff[CFG::G][CFG::VC];
};
// LDS of a float launch that may take either layout
constexpr size_t kAtFloatLds = sizeof(AtLds<float, AtF16>) > sizeof(AtLds<float, AtF8>)
                                   ? sizeof(AtLds<float, AtF16>)
                                   : sizeof(AtLds<float, AtF8>);

struct TileBox {
    double xlo, xhi, ylo, yhi, cd;
};

// A hat weight over len: at most 1 by construction, so clamping to [0, 1]
// is max(0, w); in float the clamp is the fma's output modifier.
__device__ __forceinline__ float hat_clamp(float w) { return __builtin_amdgcn_fmed3f(w, 0.f, 1.f); }
__device__ __forceinline__ double hat_clamp(double w) { return fmax(0.0, w); }

// First staged bin of view g for the tile (one below floor of the lowest t).
__device__ __forceinline__ int window_base(const ViewGeom& g, const TileBox& b) {
    const double tmin = b.cd + (g.cs >= 0.0 ? b.xlo * g.cs : b.xhi * g.cs) + (g.sn >= 0.0 ? b.ylo * g.sn : b.yhi * g.sn);
    return (int)floor(tmin) - 1;
}

// smem: the launch's LDS block for the layout's tables (AtLds<T, CFG>)
template <typename T, bool TWO, typename CFG>
__device__ __forceinline__ void adjoint_body(const T* __restrict__ y1, const T* __restrict__ y2, T c1, T c2,
                                             const T* __restrict__ xin, T alpha, T beta, T* __restrict__ out,
                                             const ViewGeom* __restrict__ views, int n, int m, int nb, int bxi,
                                             int byi, void* smem) {
    constexpr int G = CFG::G, PJ = CFG::PJ, VC = CFG::VC, VQ = CFG::VQ;
    constexpr int RS = AT_T / PJ;          // lane rows per stream
    constexpr int SL = AT_T * RS;          // lanes per stream
    constexpr int PER = VC * AT_W / SL;    // staged bins per lane and chunk
    static_assert(SL * G == AT_THREADS && SL % 64 == 0, "whole waves per stream");
    static_assert(PER * SL == VC * AT_W && VC % VQ == 0 && VC * AT_T % SL == 0, "chunk shape");
    using Lds = AtLds<T, CFG>;
    Lds& sh = *reinterpret_cast<Lds*>(smem);
    auto& win = sh.win;
    auto& colt = sh.colt;
    auto& rowt = sh.rowt;
    auto& prate = sh.prate;
    auto& poff = sh.poff;
    // h is the same on every lane of a wave: keep it (and the LDS bases built
    // from it) in scalar registers
    const int tid = threadIdx.x, h = __builtin_amdgcn_readfirstlane(tid / SL), l = tid % SL;
    const int tx = l % AT_T, ty = l / AT_T;
    const int x0 = bxi * AT_T, y0 = byi * AT_T;
    const double c = 0.5 * (double)(n - 1);
    const TileBox box{x0 - c, x0 + (AT_T - 1) - c, y0 - c, y0 + (AT_T - 1) - c, 0.5 * (double)(nb - 1)};
    // step st of stream h holds the views (st VC + i) G + h, i = 0..VC-1, so
    // every stream has work even when the view count is small
    const int nsteps = (m + VC * G - 1) / (VC * G);
    const double two32 = 4294967296.0;

    // Per view of a chunk, lane i < VC of every wave computes the view's
    // values once (window base, len, the 32.32 position of the tile's first
    // pixel, the column and row increments, the weight constants); the other
    // lanes take them by lane shuffles.
    const int lw = threadIdx.x & 63;
    T stg[PER];
    long long pv_t0 = 0, pv_dc = 0, pv_dr = 0;
    T pv_rate = T(0), pv_off = T(0);
    auto fetch = [&](int st) {
        int wb = 0;
        T len = T(0);
        pv_t0 = 3ll << 31;   // past the last view: position 1.5 in a zero window
        pv_dc = pv_dr = 0;
        pv_rate = pv_off = T(0);
        const int vl = (st * VC + lw) * G + h;
        if (lw < VC && vl < m) {
            const ViewGeom g = views[vl];
            wb = window_base(g, box);
            len = (T)g.len;
            const double t0 = fma(box.xlo, g.cs, fma(box.ylo, g.sn, box.cd)) - (double)wb;
            pv_t0 = llrint(t0 * two32);
            pv_dc = llrint(g.cs * two32);
            pv_dr = llrint(g.sn * two32);
            if (g.len > 0.0) {
                const double q = g.len2 / g.len;
                pv_rate = (T)(q / two32);
                pv_off = (T)(1.0 - q);
            }
        }
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int e = l + SL * r;
            const int i = e / AT_W, k = e - i * AT_W;
            const int v = (st * VC + i) * G + h;
            const int u = __shfl(wb, i) + k;
            const T lv = __shfl(len, i);
            T val = T(0);
            if (v < m && u >= 0 && u < nb) {
                const size_t idx = (size_t)v * nb + u;
                val = (TWO ? c1 * y1[idx] + c2 * y2[idx] : y1[idx]) * lv;
            }
            stg[r] = val;
        }
    };
    // The tables of the chunk's views (the weights absorb the 2^-32 of the
    // fraction through prate).
    auto commit = [&](int st) {
#pragma unroll
        for (int r = 0; r < PER; ++r) {
            const int e = l + SL * r;
            const int i = e / AT_W;
            win[h][i][e - i * AT_W] = stg[r];
        }
#pragma unroll
        for (int q = 0; q < VC * AT_T / SL; ++q) {
            const int e = l + SL * q;
            const int i = e / AT_T, cx = e % AT_T;
            colt[h][i][cx] = __shfl(pv_t0, i) + (long long)cx * __shfl(pv_dc, i);
        }
        for (int e0 = 0; e0 < VC * (RS + 2); e0 += SL) {
            const int e = e0 + l;
            // every lane of the wave takes part in the shuffles
            const int i = e < VC * (RS + 1) ? e / (RS + 1) : min(e - VC * (RS + 1), VC - 1);
            const long long dr = __shfl(pv_dr, i);
            const T rate = __shfl(pv_rate, i), off = __shfl(pv_off, i);
            if (e < VC * (RS + 1))
                rowt[h][i][e - (RS + 1) * i] = (long long)(e - (RS + 1) * i) * dr;
            else if (e < VC * (RS + 2)) {
                prate[h][i] = rate;
                poff[h][i] = off;
            }
        }
        (void)st;
    };

    T acc[PJ];
#pragma unroll
    for (int j = 0; j < PJ; ++j) acc[j] = T(0);
    fetch(0);
    commit(0);
    __syncthreads();
    for (int st = 0; st < nsteps; ++st) {
        fetch(st + 1);
        // the step's live views (uniform over the wave); a dead slot in the
        // last pass has a zero window
        const int rem = m - h - st * VC * G;
        const int nlive = rem <= 0 ? 0 : min(VC, (rem + G - 1) / G);
        {
            // VQ views x PJ pixels per pass: all VQ PJ tap-pair reads are independent
#pragma unroll 1
            for (int i = 0; i < nlive; i += VQ) {
                unsigned k[VQ][PJ];
                T f[VQ][PJ], a[VQ][PJ], b[VQ][PJ], rate[VQ], off[VQ];
#pragma unroll
                for (int q = 0; q < VQ; ++q) {
                    unsigned long long tj = (unsigned long long)(colt[h][i + q][tx] + rowt[h][i + q][ty]);
                    const unsigned long long dr = (unsigned long long)rowt[h][i + q][RS];
                    rate[q] = prate[h][i + q];
                    off[q] = poff[h][i + q];
#pragma unroll
                    for (int j = 0; j < PJ; ++j) {
                        // t >= 1 - rounding > 0, so the high word is floor(t)
                        k[q][j] = (unsigned)(tj >> 32);
                        f[q][j] = (T)(unsigned)tj;
                        tj += dr;
                    }
                }
#pragma unroll
                for (int q = 0; q < VQ; ++q)
#pragma unroll
                    for (int j = 0; j < PJ; ++j) {
                        a[q][j] = win[h][i + q][k[q][j]];
                        b[q][j] = win[h][i + q][k[q][j] + 1];
                    }
#pragma unroll
                for (int q = 0; q < VQ; ++q)
#pragma unroll
                    for (int j = 0; j < PJ; ++j) {
                        const T w0 = hat_clamp(fma(-f[q][j], rate[q], T(1)));
                        const T w1 = hat_clamp(fma(f[q][j], rate[q], off[q]));
                        acc[j] = fma(w0, a[q][j], fma(w1, b[q][j], acc[j]));
                    }
            }
        }
        __syncthreads();
        commit(st + 1);
        __syncthreads();
    }
    // sum the streams through LDS (reusing the staging and position tables)
    // as a fixed-order tree: at each level stream h < half adds stream h + half
    T* red = reinterpret_cast<T*>(&sh);
    constexpr int TP = AT_T * AT_T;
    static_assert((G / 2) * TP * sizeof(T) <= sizeof(sh.win) + sizeof(sh.colt), "reduction buffer");
    static_assert((G & (G - 1)) == 0, "power-of-two stream count");
    const int pix0 = ty * AT_T + tx, pstep = RS * AT_T;
#pragma unroll
    for (int half = G / 2; half >= 1; half /= 2) {
        if (h >= half && h < 2 * half) {
#pragma unroll
            for (int j = 0; j < PJ; ++j) red[(h - half) * TP + pix0 + pstep * j] = acc[j];
        }
        __syncthreads();
        if (h < half) {
#pragma unroll
            for (int j = 0; j < PJ; ++j) acc[j] += red[h * TP + pix0 + pstep * j];
        }
        __syncthreads();
    }
    if (h == 0) {
        const int ix = x0 + tx;
#pragma unroll
        for (int j = 0; j < PJ; ++j) {
            const int iy = y0 + ty + RS * j;
            if (ix < n && iy < n) {
                const size_t idx = (size_t)iy * n + ix;
                T r = beta * acc[j];
                if (xin) r += alpha * xin[idx];
                out[idx] = r;
            }
        }
    }
}

template <typename T, bool TWO, typename CFG>
__global__ __launch_bounds__(AT_THREADS) void adjoint_kernel(const T* __restrict__ y1, const T* __restrict__ y2, T c1,
                                                      T c2, const T* __restrict__ xin, T alpha, T beta,
                                                      T* __restrict__ out, const ViewGeom* __restrict__ views,
                                                      int n, int m, int nb) {
    __shared__ __align__(16) unsigned char smem[sizeof(AtLds<T, CFG>)];
    adjoint_body<T, TWO, CFG>(y1, y2, c1, c2, xin, alpha, beta, out, views, n, m, nb, blockIdx.x, blockIdx.y, smem);
}

template <typename T, typename CFG>
static void launch_adjoint_cfg(const T* y1, const T* y2, T c1, T c2, const T* xin, T alpha, T beta, T* out,
                               const ViewGeom* views, int n, int m, int nb, hipStream_t s) {
    dim3 grid((n + AT_T - 1) / AT_T, (n + AT_T - 1) / AT_T);
    if (y2)
        adjoint_kernel<T, true, CFG><<<grid, AT_THREADS, 0, s>>>(y1, y2, c1, c2, xin, alpha, beta, out, views, n, m,
                                                                 nb);
    else
        adjoint_kernel<T, false, CFG><<<grid, AT_THREADS, 0, s>>>(y1, y2, c1, c2, xin, alpha, beta, out, views, n,
                                                                  m, nb);
}

template <typename T>
hipError_t launch_adjoint(const T* y1, const T* y2, T c1, T c2, const T* xin, T alpha, T beta, T* out,
                          const ViewGeom* views, int n, int m, int nb, hipStream_t s) {
    if constexpr (sizeof(T) == 8)
        launch_adjoint_cfg<T, AtD8>(y1, y2, c1, c2, xin, alpha, beta, out, views, n, m, nb, s);
    else if (at_few_views(m))
        launch_adjoint_cfg<T, AtF8>(y1, y2, c1, c2, xin, alpha, beta, out, views, n, m, nb, s);
    else
        launch_adjoint_cfg<T, AtF16>(y1, y2, c1, c2, xin, alpha, beta, out, views, n, m, nb, s);
    return hipGetLastError();
}

// the float body in the layout the view count picks (batched and step launches)
template <bool TWO>
__device__ __forceinline__ void adjoint_body_f32(const float* __restrict__ y1, const float* __restrict__ y2, float c1,
                                                 float c2, const float* __restrict__ xin, float alpha, float beta,
                                                 float* __restrict__ out, const ViewGeom* __restrict__ views, int n,
                                                 int m, int nb, int bxi, int byi, void* smem) {
    if (at_few_views(m))
        adjoint_body<float, TWO, AtF8>(y1, y2, c1, c2, xin, alpha, beta, out, views, n, m, nb, bxi, byi, smem);
    else
        adjoint_body<float, TWO, AtF16>(y1, y2, c1, c2, xin, alpha, beta, out, views, n, m, nb, bxi, byi, smem);
}

// ---------------------------------------------------------------------------
// Batched launches: one flattened grid over all problems of a batch; the
// block map gives each workgroup its problem and its block within it.
__global__ __launch_bounds__(256) void pad_planes_batched(const BatchItem* __restrict__ items,
                                                          const BlockRef* __restrict__ map) {
    const BlockRef e = map[blockIdx.x];
    if (e.prob < 0) return;
    const BatchItem& it = items[e.prob];
    const int gx = (it.n + 31) / 32;
    pad_planes_body<float>(it.x, it.xp, it.xTp, it.n, e.local % gx, e.local / gx);
}

template <int FB>
__global__ __launch_bounds__(256) void forward_batched(const BatchItem* __restrict__ items,
                                                       const BlockRef* __restrict__ map, int rot) {
    const BlockRef e = map[blockIdx.x];
    if (e.prob < 0) return;
    const BatchItem& it = items[e.prob];
    const int gx = (it.nb + 255) / 256;
    forward_body<float, FB>(it.xp, it.xTp, it.q, it.views, it.n, it.nb, e.local % gx, e.local / gx, it.b,
                            it.lowdose ? it.winv : nullptr, it.mu[rot]);
}

// z = x - tau A^T mubar  (mode 0), or z = x - tau A^T (2 mu - mu_prev)  (mode 1, few-view k >= 1)
template <bool TWO>
__global__ __launch_bounds__(AT_THREADS) void adjoint_batched(const BatchItem* __restrict__ items,
                                                       const BlockRef* __restrict__ map, int rot) {
    const BlockRef e = map[blockIdx.x];
    if (e.prob < 0) return;
    const BatchItem& it = items[e.prob];
    const int gx = (it.n + AT_T - 1) / AT_T;
    const float* y1 = TWO ? it.mu[rot] : it.mubar;
    const float* y2 = TWO ? it.mu[(rot + 1) % 3] : nullptr;
    __shared__ __align__(16) unsigned char smem[kAtFloatLds];
    adjoint_body_f32<TWO>(y1, y2, 2.f, -1.f, it.x, 1.f, -it.tau, it.z, it.views, it.n, it.m, it.nb, e.local % gx,
                          e.local / gx, smem);
}

hipError_t launch_pad_planes_batched(const BatchItem* items, const BlockRef* map, int nblocks, hipStream_t s) {
    pad_planes_batched<<<nblocks, 256, 0, s>>>(items, map);
    return hipGetLastError();
}

hipError_t launch_forward_batched(const BatchItem* items, const BlockRef* map, int nblocks, int form, int max_n,
                                  int rot, hipStream_t s) {
    if (form == 0) {
        const hipError_t attr = slab_lds_attributes();
        if (attr != hipSuccess) return attr;
        forward_slab_batched<<<nblocks, kSlabThreads, forward_slab_lds(max_n), s>>>(items, map, rot);
    } else {
        forward_batched<FW_BATCH><<<nblocks, 256, 0, s>>>(items, map, rot);
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_batched(const BatchItem* items, const BlockRef* map, int nblocks, bool two, int rot,
                                  hipStream_t s) {
    if (two)
        adjoint_batched<true><<<nblocks, AT_THREADS, 0, s>>>(items, map, rot);
    else
        adjoint_batched<false><<<nblocks, AT_THREADS, 0, s>>>(items, map, rot);
    return hipGetLastError();
}

// Recorded steps (one table entry per problem): pad planes, A, A^T.
__global__ __launch_bounds__(256) void step_pad_kernel(const UStep* __restrict__ steps,
                                                       const BlockRef* __restrict__ map) {
    const BlockRef e = map[blockIdx.x];
    if (e.prob < 0) return;
    const UStep& st = steps[e.prob];
    if (!st.active) return;
    const int gx = (st.n + 31) / 32;
    pad_planes_body<float>(st.in[0], st.out[0], st.out[1], st.n, e.local % gx, e.local / gx);
}

__global__ __launch_bounds__(256) void step_forward_kernel(const UStep* __restrict__ steps,
                                                           const BlockRef* __restrict__ map) {
    const BlockRef e = map[blockIdx.x];
    if (e.prob < 0) return;
    const UStep& st = steps[e.prob];
    if (!st.active) return;
    const int gx = (st.nb + 255) / 256;
    forward_body<float>(st.in[0], st.in[1], st.out[0], st.views, st.n, st.nb, e.local % gx, e.local / gx);
}

__global__ __launch_bounds__(AT_THREADS) void step_adjoint_kernel(const UStep* __restrict__ steps,
                                                           const BlockRef* __restrict__ map) {
    const BlockRef e = map[blockIdx.x];
    if (e.prob < 0) return;
    const UStep& st = steps[e.prob];
    if (!st.active) return;
    const int gx = (st.n + AT_T - 1) / AT_T;
    __shared__ __align__(16) unsigned char smem[kAtFloatLds];
    adjoint_body_f32<false>(st.in[0], nullptr, 1.f, 0.f, st.in[1], 1.f, st.c0, st.out[0], st.views, st.n, st.m, st.nb,
                            e.local % gx, e.local / gx, smem);
}

hipError_t launch_step_projector(int kind, const UStep* steps, const BlockRef* map, int nblocks, hipStream_t s) {
    switch (kind) {
        case SK_PAD: step_pad_kernel<<<nblocks, 256, 0, s>>>(steps, map); break;
        case SK_FORWARD: step_forward_kernel<<<nblocks, 256, 0, s>>>(steps, map); break;
        case SK_ADJOINT: step_adjoint_kernel<<<nblocks, AT_THREADS, 0, s>>>(steps, map); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int adjoint_tiles(int n) { return (n + AT_T - 1) / AT_T; }
int pad_tiles(int n) { return (n + 31) / 32; }
int forward_blocks_x(int nb) { return (nb + 255) / 256; }

template hipError_t launch_pad_planes<float>(const float*, float*, float*, int, hipStream_t);
template hipError_t launch_pad_planes<double>(const double*, double*, double*, int, hipStream_t);
template hipError_t launch_forward<float>(const float*, const float*, float*, const ViewGeom*, int, int, int,
                                          hipStream_t);
template hipError_t launch_forward<double>(const double*, const double*, double*, const ViewGeom*, int, int,
                                           int, hipStream_t);
template hipError_t launch_adjoint<float>(const float*, const float*, float, float, const float*, float, float,
                                          float*, const ViewGeom*, int, int, int, hipStream_t);
template hipError_t launch_adjoint<double>(const double*, const double*, double, double, const double*, double,
                                           double, double*, const ViewGeom*, int, int, int, hipStream_t);

}  // namespace ctpd
