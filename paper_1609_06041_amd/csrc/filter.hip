// The preconditioner D of Eqs. 24 and 32: per view, the linear convolution of
// the detector bins with the taps h[k] = (1/pi) int_0^pi H(w) cos(k w) dw of
// the band-limited filter response H.  Every view shares one symmetric
// Toeplitz matrix T[j][i] = h[i - j], so D over all views is the dense
// contraction OUT[v][i] = sum_j S[v][j] T[j][i]  (M = views, N = K = bins),
// which runs on the matrix cores (v_mfma_f32_16x16x4_f32).  T is never
// stored: its tiles are read straight out of the 2nb-1 taps kept in LDS.
//
// The float32 kernel fuses the dual-variable algebra around D
// (Eqs. 18, 20, 31): the prologue forms the filter input from up to four
// sinograms while staging it in LDS, the epilogue combines the result with up
// to two sinograms.  A float64 variant (v_mfma_f64_16x16x4_f64) serves the
// operator-norm computation.
#include <mutex>

#include "internal.h"

namespace ctpd {

// ---------------------------------------------------------------------------
// Taps.  Ramp (kappa == 0, Eq. 32): h[0] = pi/2, h[k] = -2/(pi k^2) for odd k,
// 0 for even k != 0, all over 2 m tau.  Smoothed ramp (Eq. 24): composite
// 16-point Gauss-Legendre quadrature of w cos(k w)/(2 m tau + kappa w) over
// [0, pi] with at least two panels per period of cos(k w).
struct GaussLegendre16 {
    double x[16];   // nodes on [-1, 1]
    double w[16];   // weights
};

// With d_tau, the taps of dH/dtau = -2m w / (2 m tau + kappa w)^2 (c1 = 2m):
// for the ramp that is -h / tau.
__global__ __launch_bounds__(256) void taps_kernel(double* __restrict__ taps64, float* __restrict__ taps32,
                                                   int nb, double c0, double kappa, int panels,
                                                   GaussLegendre16 gl, double c1, int d_tau) {
    const int k = blockIdx.x;   // offset 0..nb-1
    double h;
    if (kappa == 0.0) {
        const double pi = 3.14159265358979323846;
        h = (k == 0) ? pi / 2.0 : ((k & 1) ? -2.0 / (pi * (double)k * (double)k) : 0.0);
        h /= c0;
        if (d_tau) h *= -c1 / c0;
    } else {
        const double pi = 3.14159265358979323846;
        const double width = pi / panels;
        double acc = 0.0;
        for (int p = threadIdx.x; p < panels; p += 256) {
            const double mid = (p + 0.5) * width, half = 0.5 * width;
            double ps = 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const double w = fma(half, gl.x[q], mid);
                const double den = fma(kappa, w, c0);
                const double hw = d_tau ? -c1 * w / (den * den) : w / den;
                ps = fma(gl.w[q], hw * cos((double)k * w), ps);
            }
            acc += ps * half;
        }
        // fixed-order block reduction
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        __shared__ double red[4];
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        h = (red[0] + red[1] + red[2] + red[3]) / pi;
    }
    if (threadIdx.x == 0) {
        taps64[nb - 1 + k] = h;
        taps64[nb - 1 - k] = h;
        taps32[nb - 1 + k] = (float)h;
        taps32[nb - 1 - k] = (float)h;
    }
}

static GaussLegendre16 make_gl16() {
    // Roots of P_16 by Newton's method from Chebyshev guesses; w = 2/((1-x^2) P'(x)^2).
    GaussLegendre16 g;
    const int n = 16;
    for (int i = 0; i < n / 2; ++i) {
        double x = cos(3.14159265358979323846 * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            const double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
        }
        const double w = 2.0 / ((1.0 - x * x) * dp * dp);
        g.x[i] = -x;
        g.w[i] = w;
        g.x[n - 1 - i] = x;
        g.w[n - 1 - i] = w;
    }
    return g;
}

hipError_t launch_taps(double* taps64, float* taps32, int nb, int m, double tau, double kappa, hipStream_t s,
                       bool d_tau) {
    static const GaussLegendre16 gl = make_gl16();
    const int panels = nb < 32 ? 64 : 2 * nb;
    taps_kernel<<<nb, 256, 0, s>>>(taps64, taps32, nb, 2.0 * m * tau, kappa, panels, gl, 2.0 * m, d_tau ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// float32 matrix-core filter.
//
// Work split: a workgroup owns one output block of 16 views x FNT*16 bins
// (FNT 16 x 16 MFMA tiles sharing the A operand) and splits the contraction
// over the bins j into 32-bin steps dealt round-robin to its FKS waves, so
// that every wave of the chip has a short, equal share of the matrix-core work
// (the 720-view, 736-bin shape makes 720 such workgroups, all resident at
// once).  The partial sums of the FKS waves meet in LDS and are added in a
// fixed pairwise order, so every launch form gives the same bits.  In step s
// lane (i, g) (i = lane % 16, g = lane / 16) holds
//     A[i][u] = s[v0 + i][32 s + 8 g + u],  B[u][c] = h[n0 + c - (32 s + 8 g + u)],
// u = 0..7, so a lane reads its 8 input values with two 16-byte loads (where
// the row length and alignment allow) and its taps as four aligned words of
// LDS, where the taps of the block's range of offsets are staged once.  The
// next step's loads are issued before the current step's MFMAs.
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int FNT = 3;                    // 16 x 16 output tiles per workgroup (along the bins)
constexpr int FKS = 4;                    // waves per workgroup, each a share of the contraction
constexpr int FTHREADS = 64 * FKS;
constexpr int FBN = 16 * FNT;             // output bins per workgroup
constexpr int FBM = 16;                   // views per workgroup
static_assert((FKS & (FKS - 1)) == 0, "pairwise reduction over a power of two of waves");

// Number of sinogram arrays the prologue of each mode reads, and the input of
// D formed from their raw values.
template <int MODE>
struct FilterIn {
    static constexpr int N = MODE == FILT_DUAL_LD ? 4 : MODE == FILT_EXTRAP ? 3 : MODE == FILT_DUAL_FV ? 2 : 1;
    __device__ static __forceinline__ float combine(const float* r) {
#pragma clang fp contract(off)
        if (MODE == FILT_EXTRAP) return r[0] * (r[1] - r[2]);
        if (MODE == FILT_DUAL_LD) return fmaf(-r[2], r[3], r[0] - r[1]);
        if (MODE == FILT_DUAL_FV) return r[0] - r[1];
        return r[0];
    }
};

// The filter input s[v][kk + t], t = 0..3, of one lane (kk = k0 + 4q).  VW is
// the load width the row allows: 4 (nb % 4 == 0 and every input 16-byte
// aligned: one 16-byte load per input), 2 (nb even, 8-byte aligned: two
// 8-byte loads) or 1 (four scalar loads).  Loads past the row end are clamped
// into it and masked after the load; there are no branches, so the compiler
// keeps the loads in flight.
template <int MODE, int VW>
__device__ __forceinline__ void filter_load_chunk(const FilterArgs& a, size_t row, int nb, int kk, float (&dst)[4]) {
    constexpr int NIN = FilterIn<MODE>::N;
    const float* src[4] = {a.in0, a.in1, a.in2, a.in3};
    float r[NIN][4];
    if (VW == 4) {
        const size_t col = row + min(kk, nb - 4);
#pragma unroll
        for (int q = 0; q < NIN; ++q) {
            const float4 x = *reinterpret_cast<const float4*>(src[q] + col);
            r[q][0] = x.x;
            r[q][1] = x.y;
            r[q][2] = x.z;
            r[q][3] = x.w;
        }
    } else if (VW == 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const size_t col = row + min(kk + 2 * h, nb - 2);
#pragma unroll
            for (int q = 0; q < NIN; ++q) {
                const float2 x = *reinterpret_cast<const float2*>(src[q] + col);
                r[q][2 * h] = x.x;
                r[q][2 * h + 1] = x.y;
            }
        }
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const size_t col = row + min(kk + t, nb - 1);
#pragma unroll
            for (int q = 0; q < NIN; ++q) r[q][t] = src[q][col];
        }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        float rr[NIN];
#pragma unroll
        for (int q = 0; q < NIN; ++q) rr[q] = r[q][t];
        dst[t] = kk + t < nb ? FilterIn<MODE>::combine(rr) : 0.0f;
    }
}

// FP32 on the bf16 matrix cores.  Every operand x is split into three bf16
// terms, x = x1 + x2 + x3 + e (x1 = bf16(x), x2 = bf16(x - x1),
// x3 = bf16(x - x1 - x2), rounded to nearest; both differences are exact in
// FP32): each rounding loses at most 2^-8 of what it rounds, so |x2| <= 2^-8
// |x|, |x3| <= 2^-16 |x| and |e| <= 2^-24 |x|.  A product s h is formed from
// the six term products of order 2^-16 of it or more (s1 h1, s1 h2, s2 h1,
// s1 h3, s3 h1, s2 h2); the dropped ones are at most 2^-23 of it together,
// so a product errs by at most about 2^-22 relative, a few times the FP32
// rounding of one product.  A bf16 term product is exact in FP32 and the
// matrix core accumulates in FP32, so beyond that the contraction carries the
// rounding of an FP32 accumulation, as with FP32 matrix instructions (the
// accumulation's rounding dominates the error measured against float64), at
// 6 v_mfma_f32_16x16x32_bf16 (16 cycles each) per 32 x 16 x 16 block instead
// of 8 v_mfma_f32_16x16x4_f32 (32 cycles each).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split3(float x, __bf16& t1, __bf16& t2, __bf16& t3) {
    // x must be the rounded float: a product that forms x may not fuse with
    // the subtraction below (the same input, formed in a prologue or read
    // from memory, must split the same)
#pragma clang fp contract(off)
    t1 = (__bf16)x;
    const float r1 = x - (float)t1;
    t2 = (__bf16)r1;
    t3 = (__bf16)(r1 - (float)t2);
}

// The inputs s[v][kk + t], t = 0..3, as filter_load_chunk reads them, but for
// a single-input mode unmasked (past the row end they are values of the row,
// zeroed by the caller where it uses them), so that nothing consumes the
// loads until then and they stay in flight.
template <int MODE, int VW>
__device__ __forceinline__ void filter_load_raw(const FilterArgs& a, size_t row, int nb, int kk, float (&dst)[4]) {
    if constexpr (FilterIn<MODE>::N > 1) {
        filter_load_chunk<MODE, VW>(a, row, nb, kk, dst);
    } else if constexpr (VW == 4) {
        const float4 x = *reinterpret_cast<const float4*>(a.in0 + row + min(kk, nb - 4));
        dst[0] = x.x;
        dst[1] = x.y;
        dst[2] = x.z;
        dst[3] = x.w;
    } else if constexpr (VW == 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float2 x = *reinterpret_cast<const float2*>(a.in0 + row + min(kk + 2 * h, nb - 2));
            dst[2 * h] = x.x;
            dst[2 * h + 1] = x.y;
        }
    } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) dst[t] = a.in0[row + min(kk + t, nb - 1)];
    }
}

// Lay-out of the dynamic LDS: the block's taps, reversed (R[y] = h[n0 + FBN -
// 1 - y]) and split into three bf16 terms, each term stored twice as bf16
// pairs (copy e, word q = (R[2q + e], R[2q + e + 1])) so that every lane's
// eight taps are four aligned words of one copy.
__host__ __device__ constexpr int filter_tap_words(int nb) {
    // ntl = kpad + FBN - 1 taps (kpad: nb rounded up to 32), one spare word
    return ((((nb + 31) / 32) * 32 + FBN + 2) / 2 + 3) & ~3;
}
__host__ __device__ constexpr int filter_taps_floats(int nb) {
    return ((6 * filter_tap_words(nb) + 63) / 64) * 64;
}

// LDS: the taps in the dynamic allocation (smem, its size set by the row
// length), the waves' partial tiles in a static array of the kernel (red).
constexpr int FRED = FKS * FNT * 256;   // [FKS][FNT][4][64] partial tiles

// SPW > 0: every wave has at most SPW steps (nb <= 32 FKS SPW), which run
// unrolled, so that the compiler tracks each load on its own and the loads
// stay in flight across steps; SPW = 0: any row length, a loop over steps.
template <int MODE, int VW, int SPW>
__device__ __forceinline__ void filter_tile(const FilterArgs& a, const float* __restrict__ taps, int m, int nb,
                                            float* smem, float* red, int tile) {
    const int tiles_x = (nb + FBN - 1) / FBN;
    const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
    const int v0 = ty * FBM, n0 = tx * FBN;
    const int nst = (nb + 31) >> 5, kpad = nst * 32;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int TQ = filter_tap_words(nb);
    unsigned int* tb = reinterpret_cast<unsigned int*>(smem);   // [term][copy][TQ]
    const size_t row = (size_t)min(v0 + li, m - 1) * nb;   // rows past m only feed outputs never stored
    // step s (bins 32 s .. 32 s + 31) of lane (i, g): A[i][u] = s[v0 + i][32 s + 8 g + u]
    auto load_step = [&](int st, float (&dst)[8]) {
        float lo4[4], hi4[4];
        filter_load_raw<MODE, VW>(a, row, nb, 32 * st + 8 * lq, lo4);
        filter_load_raw<MODE, VW>(a, row, nb, 32 * st + 8 * lq + 4, hi4);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            dst[t] = lo4[t];
            dst[4 + t] = hi4[t];
        }
    };
    // two steps in flight: this wave's first two steps now, each later one as
    // soon as a buffer is split
    float cur[8], nxt[8];
    int c = w;
    if (SPW > 0 || c < nst) load_step(min(c, nst - 1), cur);
    if (SPW > 0 || c + FKS < nst) load_step(min(c + FKS, nst - 1), nxt);
    // the taps, split and laid out as above (R[y] = 0 outside the filter):
    // thread q forms word q of both copies from R[2q], R[2q + 1], R[2q + 2]
    // (loads from clamped indices, so that they carry no branch and are
    // issued together; the unrolled form knows how many words a thread has)
    const int ntl = kpad + FBN - 1;
    auto stage = [&](int q) {
        // a thread past the last word stores the last word again: it, like
        // every word from TQ - 1 on, holds only taps past the window (zeros),
        // so the store needs no branch
        q = min(q, TQ - 1);
        float v[3];
#pragma unroll
        for (int h = 0; h < 3; ++h) {
            const int y = 2 * q + h;
            const int d = n0 + FBN - 1 - y;
            // (a product, not a select: the compiler may not skip the load of
            // a value that could be a NaN, so the load carries no branch)
            const float t = taps[min(max(nb - 1 + d, 0), 2 * nb - 2)];
            v[h] = t * ((y < ntl && d > -nb && d < nb) ? 1.0f : 0.0f);
        }
        unsigned int t[3][3];
#pragma unroll
        for (int h = 0; h < 3; ++h) {
            __bf16 t1, t2, t3;
            split3(v[h], t1, t2, t3);
            t[0][h] = __builtin_bit_cast(unsigned short, t1);
            t[1][h] = __builtin_bit_cast(unsigned short, t2);
            t[2][h] = __builtin_bit_cast(unsigned short, t3);
        }
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            tb[(2 * p) * TQ + q] = t[p][0] | (t[p][1] << 16);
            tb[(2 * p + 1) * TQ + q] = t[p][1] | (t[p][2] << 16);
        }
    };
    if constexpr (SPW > 0) {
        constexpr int NQ = (filter_tap_words(32 * FKS * SPW) + FTHREADS - 1) / FTHREADS;
#pragma unroll
        for (int k = 0; k < NQ; ++k) stage(tid + k * FTHREADS);
    } else {
        for (int q = tid; q < TQ; q += FTHREADS) stage(q);
    }
    // the epilogue's operands (element e = tid + r FTHREADS of the block),
    // loaded by each wave with its last step, into the registers its input
    // buffers free, so that their round trip overlaps that step's MFMAs
    constexpr int NE = (FBM * FBN + FTHREADS - 1) / FTHREADS;
    float ee0[NE], ee1[NE], esw[NE];
    // (unconditional loads: an operand the launch lacks is read from the
    // input in its place, an element outside the block from the block's
    // first, and neither is used; branches here would make the compiler wait
    // for every load in flight)
    const float* pe0 = a.E0 ? a.E0 : a.in0;
    const float* pe1 = a.E1 ? a.E1 : a.in0;
    const float* psw = a.Sout ? a.Sw : a.in0;
    auto epi_load = [&]() {
#pragma unroll
        for (int r = 0; r < NE; ++r) {
            const int e = tid + r * FTHREADS;
            const int i = e / FBN, jj = e - i * FBN;
            const int v = v0 + i, col = n0 + jj;
            const bool on = e < FBM * FBN && v < m && col < nb;
            const size_t idx = on ? (size_t)v * nb + col : (size_t)v0 * nb + n0;
            ee0[r] = pe0[idx];
            ee1[r] = pe1[idx];
            esw[r] = psw[idx];
        }
    };
    v4f acc[FNT];
#pragma unroll
    for (int j = 0; j < FNT; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
    // the taps are in LDS once every wave's LDS writes are done; the global
    // loads issued so far stay in flight across this barrier (a
    // __syncthreads would wait for them too)
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    // B[u][ci] = h[n0 + 16 j + ci - 32 s - 8 g - u] = R[yb + u] with
    // yb = FBN - 1 - ci - 16 j + 32 s + 8 g, whose parity is that of FBN - 1 - ci
    const int ecp = (FBN - 1 - li) & 1;
    const int qb = (FBN - 1 - li - ecp) / 2 + 4 * lq;
    const unsigned int* tc = tb + ecp * TQ;
    auto bterm = [&](int p, int q0) {
        const unsigned int* src = tc + 2 * p * TQ + q0;
        const u32x4 wv = u32x4{src[0], src[1], src[2], src[3]};
        return __builtin_bit_cast(bf16x8, wv);
    };
    // step st: its inputs (buf) are split into their bf16 terms, then (ahead)
    // the step two further on is loaded into the freed registers, or (epi)
    // the epilogue's operands, then the MFMAs run.  A step past the row end
    // (st >= nst: the even step count of the unrolled form) has its inputs
    // zeroed and adds exact zeros.
    auto step = [&](float (&buf)[8], int st, bool ahead, bool epi) {
        bf16x8 a1, a2, a3;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            __bf16 t1, t2, t3;
            split3(32 * st + 8 * lq + u < nb ? buf[u] : 0.0f, t1, t2, t3);
            a1[u] = t1;
            a2[u] = t2;
            a3[u] = t3;
        }
        if (ahead)
            load_step(min(st + 2 * FKS, nst - 1), buf);
        else if (epi)
            epi_load();
        __builtin_amdgcn_sched_barrier(0);
        const int sb = min(st, nst - 1);   // keeps the tap reads in the staged range
#pragma unroll
        for (int j = 0; j < FNT; ++j) {
            const int q0 = qb - 8 * j + 16 * sb;
            const bf16x8 b1 = bterm(0, q0), b2 = bterm(1, q0), b3 = bterm(2, q0);
            // smallest terms first
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3, b1, acc[j], 0, 0, 0);
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b3, acc[j], 0, 0, 0);
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b2, acc[j], 0, 0, 0);
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b1, acc[j], 0, 0, 0);
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b2, acc[j], 0, 0, 0);
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[j], 0, 0, 0);
        }
    };
    if constexpr (SPW > 0) {
        // exactly SPW steps per wave, no branches: every load is tracked on
        // its own and stays in flight until its step
#pragma unroll
        for (int k = 0; k < SPW; ++k) {
            if (k & 1)
                step(nxt, c + k * FKS, k + 2 < SPW, k == SPW - 1);
            else
                step(cur, c + k * FKS, k + 2 < SPW, k == SPW - 1);
        }
    } else {
        // steps c, c + FKS, ... (the two buffers alternate)
        for (; c < nst; c += 2 * FKS) {
            const bool last0 = c + FKS >= nst, last1 = c + 2 * FKS >= nst;
            step(cur, c, c + 2 * FKS < nst, last0);
            if (c + FKS < nst) step(nxt, c + FKS, c + 3 * FKS < nst, last1);
        }
        if (w >= nst) epi_load();   // a wave without steps
    }
    // MFMA 16x16 result: D[i][c] in lane c + 16 (i / 4), element i % 4
#pragma unroll
    for (int j = 0; j < FNT; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[((w * FNT + j) * 4 + r) * 64 + lane] = acc[j][r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NE; ++r) {
        const int e = tid + r * FTHREADS;
        const int i = e / FBN, jj = e - i * FBN;
        const int v = v0 + i, col = n0 + jj;
        if (!(e < FBM * FBN && v < m && col < nb)) continue;
        const int off = ((jj >> 4) * 4 + (i & 3)) * 64 + (jj & 15) + 16 * (i >> 2);
        float p[FKS];
#pragma unroll
        for (int q = 0; q < FKS; ++q) p[q] = red[q * FNT * 256 + off];
#pragma unroll
        for (int st = 1; st < FKS; st <<= 1)
#pragma unroll
            for (int q = 0; q < FKS; q += 2 * st) p[q] += p[q + st];
        const size_t idx = (size_t)v * nb + col;
        {
            // no contraction here: where a launch form fixes e0 = 1 at
            // compile time the fmaf below folds to an add, which would fuse
            // with this product, and that form would round once where the
            // others round twice
#pragma clang fp contract(off)
            float val = a.c * p[0];
            float e0v = 0.0f;
            if (a.E0) {
                e0v = ee0[r];
                val = fmaf(a.e0, e0v, val);
            }
            if (a.E1) val = fmaf(a.e1, ee1[r], val);
            a.out[idx] = val;
            if (a.Sout) a.Sout[idx] = esw[r] * (val - e0v);
        }
    }
}

// Every load width gives the same values and the same MFMA sequence, so the
// choice (per workgroup, from nb and the input addresses) never changes a bit.
template <int MODE>
__device__ __forceinline__ void filter_body(const FilterArgs& a, const float* __restrict__ taps, int m, int nb,
                                            float* smem, float* red, int tile) {
    constexpr int NIN = FilterIn<MODE>::N;
    const uintptr_t bits = (uintptr_t)a.in0 | (NIN > 1 ? (uintptr_t)a.in1 : 0) | (NIN > 2 ? (uintptr_t)a.in2 : 0) |
                           (NIN > 3 ? (uintptr_t)a.in3 : 0);
    if ((nb & 3) == 0 && (bits & 15) == 0) {
        const int spw = ((nb + 31) / 32 + FKS - 1) / FKS;
        if (spw <= 2)
            filter_tile<MODE, 4, 2>(a, taps, m, nb, smem, red, tile);
        else if (spw <= 4)
            filter_tile<MODE, 4, 4>(a, taps, m, nb, smem, red, tile);
        else if (spw <= 6)
            filter_tile<MODE, 4, 6>(a, taps, m, nb, smem, red, tile);
        else if (spw <= 8)
            filter_tile<MODE, 4, 8>(a, taps, m, nb, smem, red, tile);
        else
            filter_tile<MODE, 4, 0>(a, taps, m, nb, smem, red, tile);
    } else if ((nb & 1) == 0 && (bits & 7) == 0) {
        filter_tile<MODE, 2, 0>(a, taps, m, nb, smem, red, tile);
    } else {
        filter_tile<MODE, 1, 0>(a, taps, m, nb, smem, red, tile);
    }
}

template <int MODE>
__global__ __launch_bounds__(FTHREADS) __attribute__((amdgpu_waves_per_eu(3))) void filter_mfma_kernel(
    FilterArgs a, const float* __restrict__ taps, int m, int nb) {
    extern __shared__ float smem[];
    __shared__ float red[FRED];
    // Workgroups are dealt to the 8 XCDs round-robin (workgroup b to XCD
    // b mod 8); XCD x takes the x-th contiguous run of tiles (view-block
    // major), so the rows of a view block are fetched into one or two XCDs'
    // L2 instead of all eight.  A permutation of the tiles: same bits.
    const int G = gridDim.x, per = G >> 3, rem = G & 7, x = blockIdx.x & 7;
    const int tile = x * per + min(x, rem) + (blockIdx.x >> 3);
    filter_body<MODE>(a, taps, m, nb, smem, red, tile);
}

// the dynamic part (the taps); the partial tiles are static
size_t filter_lds_bytes(int nb) { return sizeof(float) * (size_t)filter_taps_floats(nb); }

// past 64 KB of LDS in all (rows of more than ~3400 bins) the limit of the
// filter kernels is lifted, once, to what the longest row needs
static hipError_t filter_lds_lift();

hipError_t launch_filter_f32(const FilterArgs& a, const float* taps32, int m, int nb, hipStream_t s) {
    const int grid = filter_blocks_x(nb) * filter_blocks_y(m);
    const size_t lds = filter_lds_bytes(nb);
    if (lds + sizeof(float) * FRED > 65536) {
        const hipError_t e = filter_lds_lift();
        if (e != hipSuccess) return e;
    }
    switch (a.mode) {
        case FILT_EXTRAP: filter_mfma_kernel<FILT_EXTRAP><<<grid, FTHREADS, lds, s>>>(a, taps32, m, nb); break;
        case FILT_DUAL_LD: filter_mfma_kernel<FILT_DUAL_LD><<<grid, FTHREADS, lds, s>>>(a, taps32, m, nb); break;
        case FILT_DUAL_FV: filter_mfma_kernel<FILT_DUAL_FV><<<grid, FTHREADS, lds, s>>>(a, taps32, m, nb); break;
        default: filter_mfma_kernel<FILT_PLAIN><<<grid, FTHREADS, lds, s>>>(a, taps32, m, nb); break;
    }
    return hipGetLastError();
}

// Batched filter: the solver's two uses of D per iteration, with the
// epilogue operands taken from each problem's workspaces (mu^k = mu[rot],
// mu^{k-1} = mu[(rot+1)%3], mu^{k+1} -> mu[(rot+2)%3]).  The filter inputs are
// written by the kernels before: the dual update's residual by the projector
// (q), the extrapolation's W^-1 (mu^k - mu^{k-1}) by the previous dual update
// (sx), so every launch runs the plain prologue.
template <int MODE>
__global__ __launch_bounds__(FTHREADS) __attribute__((amdgpu_waves_per_eu(3))) void filter_batched(
    const BatchItem* __restrict__ items, const BlockRef* __restrict__ map, int rot) {
    extern __shared__ float smem[];
    __shared__ float red[FRED];
    const BlockRef e = map[blockIdx.x];
    if (e.prob < 0) return;
    const BatchItem& it = items[e.prob];
    float* mu = it.mu[rot];
    float* mup = it.mu[(rot + 1) % 3];
    FilterArgs a{};
    a.mode = FILT_PLAIN;
    if (MODE == FILT_PLAIN) {   // k = 0: D b (z = -sigma (x - tau A^T D b) follows)
        a.in0 = it.b;
        a.c = 1.f;
        a.out = it.mubar;
    } else if (MODE == FILT_EXTRAP) {   // mubar = 2 mu - mu_prev - sigma D W^-1 (mu - mu_prev)
        a.in0 = it.sx;
        a.E0 = mu;
        a.e0 = 2.f;
        a.E1 = mup;
        a.e1 = -1.f;
        a.c = -it.sigma;
        a.out = it.mubar;
    } else {   // mu^{k+1} = mu + sigma D (A x - b [- W^-1 mu]), and the next extrapolation's input
        a.in0 = it.q;
        a.E0 = mu;
        a.e0 = 1.f;
        a.c = it.sigma;
        a.out = it.mu[(rot + 2) % 3];
        a.Sw = it.winv;
        a.Sout = it.sx;
    }
    filter_body<FILT_PLAIN>(a, it.taps, it.m, it.nb, smem, red, e.local);
}

hipError_t launch_filter_batched(const BatchItem* items, const BlockRef* map, int nblocks, int mode, int rot,
                                 int max_nb, hipStream_t s) {
    const size_t lds = filter_lds_bytes(max_nb);
    if (lds + sizeof(float) * FRED > 65536) {
        const hipError_t e = filter_lds_lift();
        if (e != hipSuccess) return e;
    }
    switch (mode) {
        case FILT_EXTRAP: filter_batched<FILT_EXTRAP><<<nblocks, FTHREADS, lds, s>>>(items, map, rot); break;
        case FILT_DUAL_LD: filter_batched<FILT_DUAL_LD><<<nblocks, FTHREADS, lds, s>>>(items, map, rot); break;
        case FILT_DUAL_FV: filter_batched<FILT_DUAL_FV><<<nblocks, FTHREADS, lds, s>>>(items, map, rot); break;
        default: filter_batched<FILT_PLAIN><<<nblocks, FTHREADS, lds, s>>>(items, map, rot); break;
    }
    return hipGetLastError();
}

// One recorded filter step per problem (the unrolled passes).
template <int MODE>
__global__ __launch_bounds__(FTHREADS) __attribute__((amdgpu_waves_per_eu(3))) void step_filter_kernel(
    const UStep* __restrict__ steps, const BlockRef* __restrict__ map) {
    extern __shared__ float smem[];
    __shared__ float red[FRED];
    const BlockRef e = map[blockIdx.x];
    if (e.prob < 0) return;
    const UStep& st = steps[e.prob];
    if (!st.active) return;
    filter_body<MODE>(st.fa, st.taps, st.m, st.nb, smem, red, e.local);
}

hipError_t launch_step_filter(const UStep* steps, const BlockRef* map, int nblocks, int mode, int max_nb,
                              hipStream_t s) {
    const size_t lds = filter_lds_bytes(max_nb);
    if (lds + sizeof(float) * FRED > 65536) {
        const hipError_t e = filter_lds_lift();
        if (e != hipSuccess) return e;
    }
    switch (mode) {
        case FILT_EXTRAP: step_filter_kernel<FILT_EXTRAP><<<nblocks, FTHREADS, lds, s>>>(steps, map); break;
        case FILT_DUAL_LD: step_filter_kernel<FILT_DUAL_LD><<<nblocks, FTHREADS, lds, s>>>(steps, map); break;
        case FILT_DUAL_FV: step_filter_kernel<FILT_DUAL_FV><<<nblocks, FTHREADS, lds, s>>>(steps, map); break;
        default: step_filter_kernel<FILT_PLAIN><<<nblocks, FTHREADS, lds, s>>>(steps, map); break;
    }
    return hipGetLastError();
}

static hipError_t filter_lds_lift() {
    static std::once_flag once;
    static hipError_t attr = hipSuccess;
    std::call_once(once, [] {
        const void* k[] = {
            (const void*)filter_mfma_kernel<FILT_PLAIN>,  (const void*)filter_mfma_kernel<FILT_EXTRAP>,
            (const void*)filter_mfma_kernel<FILT_DUAL_LD>, (const void*)filter_mfma_kernel<FILT_DUAL_FV>,
            (const void*)filter_batched<FILT_PLAIN>,      (const void*)filter_batched<FILT_EXTRAP>,
            (const void*)filter_batched<FILT_DUAL_LD>,    (const void*)filter_batched<FILT_DUAL_FV>,
            (const void*)step_filter_kernel<FILT_PLAIN>,  (const void*)step_filter_kernel<FILT_EXTRAP>,
            (const void*)step_filter_kernel<FILT_DUAL_LD>, (const void*)step_filter_kernel<FILT_DUAL_FV>};
        for (const void* f : k)
            if (attr == hipSuccess)
                attr = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)filter_lds_bytes(CTPD_MAX_BINS));
    });
    return attr;
}

// Upper bound of the largest eigenvalue of the nb x nb Toeplitz section of
// the taps: its eigenvalues lie between the extremes of the generating
// function f(w) = h_0 + 2 sum_{k=1}^{nb-1} h_k cos(k w) (symmetric taps), and
// f is evaluated on kSymGrid equispaced points of [0, pi] (the cosines by
// their three-term recurrence) plus the Lipschitz margin (spacing / 2) *
// 2 sum_k k |h_k|, so the result is not below the true maximum.
constexpr int kSymGrid = kSymBlocks * 256;

__global__ __launch_bounds__(256) void symbol_grid_kernel(const double* __restrict__ taps64, int nb,
                                                          double* __restrict__ partial) {
    __shared__ double red[4];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const double w = M_PI * (double)i / (double)(kSymGrid - 1);
    const double* h = taps64 + (nb - 1);
    const double c1 = cos(w);
    double cprev = 1.0, c = c1, f = 0.0;
    for (int k = 1; k < nb; ++k) {
        f = fma(h[k], c, f);
        const double cn = fma(2.0 * c1, c, -cprev);
        cprev = c;
        c = cn;
    }
    double v = fma(2.0, f, h[0]);
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ __launch_bounds__(256) void symbol_final_kernel(const double* __restrict__ taps64, int nb,
                                                           double* __restrict__ out) {
    __shared__ double rl[4], rm[4];
    const double* h = taps64 + (nb - 1);
    double lip = 0.0;
    for (int k = 1 + threadIdx.x; k < nb; k += 256) lip = fma((double)k, fabs(h[k]), lip);
    double mx = threadIdx.x < kSymBlocks ? out[1 + threadIdx.x] : -1e300;
    for (int off = 32; off > 0; off >>= 1) {
        lip += __shfl_xor(lip, off);
        mx = fmax(mx, __shfl_xor(mx, off));
    }
    if ((threadIdx.x & 63) == 0) {
        rl[threadIdx.x >> 6] = lip;
        rm[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double L = 2.0 * ((rl[0] + rl[1]) + (rl[2] + rl[3]));
        const double m = fmax(fmax(rm[0], rm[1]), fmax(rm[2], rm[3]));
        out[0] = m + 0.5 * (M_PI / (double)(kSymGrid - 1)) * L;
    }
}

__global__ __launch_bounds__(256) void taps_scale_kernel(const double* __restrict__ taps1, int ntap, double kappa,
                                                         double* __restrict__ taps64, float* __restrict__ taps32,
                                                         const double* __restrict__ sym1,
                                                         double* __restrict__ sym_out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < ntap) {
        const double t = taps1[i] / kappa;
        taps64[i] = t;
        taps32[i] = (float)t;
    }
    if (i == 0 && sym_out) sym_out[0] = sym1[0] / kappa;
}

hipError_t launch_taps_scale(const double* taps1, int ntap, double kappa, double* taps64, float* taps32,
                             const double* sym1, double* sym_out, hipStream_t s) {
    taps_scale_kernel<<<(ntap + 255) / 256, 256, 0, s>>>(taps1, ntap, kappa, taps64, taps32, sym1, sym_out);
    return hipGetLastError();
}

hipError_t launch_symbol_max(const double* taps64, int nb, double* out, hipStream_t s) {
    symbol_grid_kernel<<<kSymBlocks, 256, 0, s>>>(taps64, nb, out + 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    symbol_final_kernel<<<1, 256, 0, s>>>(taps64, nb, out);
    return hipGetLastError();
}

// filter work decomposition (for batched block maps)
int filter_blocks_x(int nb) { return (nb + FBN - 1) / FBN; }
int filter_blocks_y(int m) { return (m + FBM - 1) / FBM; }


// ---------------------------------------------------------------------------
// float64 filter on the matrix cores (v_mfma_f64_16x16x4_f64), for the
// operator norms: out = post .* D (pre .* in)  (pre / post optional).
// DBM views x DBN bins per workgroup cut into 16 x 16 MFMA tiles, wave w owns
// DACC consecutive tiles of one tile row; per 64-bin stage of the input the
// workgroup keeps only the 127 taps that stage touches, and the next stage is
// loaded into registers while the current one runs.  The A and B operand
// layouts match the f32 instruction; the result differs: D[i][j] sits in lane
// j + 16*(i%4), element i/4.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int DBM = 16;    // views per workgroup (float64 filter)
constexpr int DBN = 64;    // output bins per workgroup (float64 filter)
constexpr int DTPR = DBN / 16;            // 16 x 16 output tiles per tile row
constexpr int DACC = DBM * DBN / 1024;    // accumulators per wave (4 waves)
static_assert(DACC >= 1 && DTPR % DACC == 0, "a wave's tiles lie in one tile row");
constexpr int DBK = 64;
constexpr int DSTRIDE = DBK + 1;     // odd pitch: 16 lanes x 8 bytes cover all 32 banks
constexpr int DTW = DBN + DBK - 1;   // taps per stage
constexpr int DPER = DBM * DBK / 256;

template <bool PRE, bool POST>
__device__ __forceinline__ void filter_f64_body(const double* __restrict__ in, double* __restrict__ out,
                                                const double* __restrict__ taps, const double* __restrict__ pre,
                                                const double* __restrict__ post, int m, int nb, int bxi,
                                                int byi) {
    __shared__ double stile[DBM * DSTRIDE];
    __shared__ double hw[DTW + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n0 = bxi * DBN, v0 = byi * DBM;
    const int wr = (wave * DACC / DTPR) * 16, wc = (wave * DACC % DTPR) * 16;
    const int li = lane & 15, lk = lane >> 4;
    double stg[DPER], stp[DPER];
    double tstg = 0.0;
    auto fetch = [&](int k0) {
#pragma unroll
        for (int r = 0; r < DPER; ++r) {
            const int e = tid + 256 * r;
            const int row = e / DBK, cc = e - row * DBK;
            const int v = v0 + row, j = k0 + cc;
            const bool ok = v < m && j < nb;
            const size_t idx = ok ? (size_t)v * nb + j : 0;   // clamped, unconditional load
            stg[r] = ok ? in[idx] : 0.0;
            if (PRE) stp[r] = pre[idx];   // multiplied in at the LDS store, so all loads stay in flight
        }
        // offsets d = col - krow in [n0 - k0 - (DBK-1), n0 - k0 + DBN - 1]
        const int d = n0 - k0 - (DBK - 1) + tid;
        const bool tok = tid < DTW && d > -nb && d < nb;
        const double tv = taps[tok ? nb - 1 + d : 0];
        tstg = tok ? tv : 0.0;
    };
    v4d acc[DACC];
#pragma unroll
    for (int q = 0; q < DACC; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
    fetch(0);
    for (int k0 = 0; k0 < nb; k0 += DBK) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < DPER; ++r) {
            const int e = tid + 256 * r;
            const int row = e / DBK;
            stile[row * DSTRIDE + (e - row * DBK)] = PRE ? stg[r] * stp[r] : stg[r];
        }
        if (tid < DTW) hw[tid] = tstg;
        __syncthreads();
        if (k0 + DBK < nb) fetch(k0 + DBK);
        // T[krow][col] = h[col - krow] at hw[(col - n0) - (krow - k0) + DBK - 1]
        const int hb = wc + li - lk + DBK - 1;
#pragma unroll 4
        for (int kk = 0; kk < DBK; kk += 4) {
            const double av = stile[(wr + li) * DSTRIDE + kk + lk];
#pragma unroll
            for (int q = 0; q < DACC; ++q)
                acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, hw[hb - kk + 16 * q], acc[q], 0, 0, 0);
        }
    }
#pragma unroll
    for (int blk = 0; blk < DACC; ++blk) {
        const int col = n0 + wc + 16 * blk + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int v = v0 + wr + lk + 4 * r;   // f64 16x16x4: D[i][j] in lane j + 16*(i%4), element i/4
            if (v < m && col < nb) {
                const size_t idx = (size_t)v * nb + col;
                double val = acc[blk][r];
                if (POST) val *= post[idx];
                out[idx] = val;
            }
        }
    }
}

template <bool PRE, bool POST>
__global__ __launch_bounds__(256) void filter_f64_kernel(const double* __restrict__ in, double* __restrict__ out,
                                                         const double* __restrict__ taps,
                                                         const double* __restrict__ pre,
                                                         const double* __restrict__ post, int m, int nb) {
    filter_f64_body<PRE, POST>(in, out, taps, pre, post, m, nb, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(256) void norm_filter_batched(const NormItem* __restrict__ items,
                                                           const BlockRef* __restrict__ map, int rot) {
    const BlockRef e = map[blockIdx.x];
    if (e.prob < 0) return;
    const NormItem& it = items[e.prob];
    const int gx = (it.nb + DBN - 1) / DBN;
    // views whose chain has stopped are neither stepped nor read again: a
    // workgroup whose views have all stopped has nothing to do
    const int v = (e.local / gx) * DBM + (int)threadIdx.x;
    const int live = threadIdx.x < DBM && v < it.m && !it.done[v];
    if (!__syncthreads_or(live)) return;
    filter_f64_body<true, true>(it.v[rot], it.v[(rot + 2) % 3], it.taps64, it.rs, it.rs, it.m, it.nb, e.local % gx,
                                e.local / gx);
}

hipError_t launch_norm_filter_batched(const NormItem* it, const BlockRef* map, int nblocks, int rot,
                                      hipStream_t s) {
    norm_filter_batched<<<nblocks, 256, 0, s>>>(it, map, rot);
    return hipGetLastError();
}

hipError_t launch_filter_f64(const double* in, double* out, const double* taps64, const double* pre,
                             const double* post, int m, int nb, hipStream_t s) {
    dim3 grid((nb + DBN - 1) / DBN, (m + DBM - 1) / DBM);
    if (pre && post)
        filter_f64_kernel<true, true><<<grid, 256, 0, s>>>(in, out, taps64, pre, post, m, nb);
    else if (pre)
        filter_f64_kernel<true, false><<<grid, 256, 0, s>>>(in, out, taps64, pre, post, m, nb);
    else if (post)
        filter_f64_kernel<false, true><<<grid, 256, 0, s>>>(in, out, taps64, pre, post, m, nb);
    else
        filter_f64_kernel<false, false><<<grid, 256, 0, s>>>(in, out, taps64, pre, post, m, nb);
    return hipGetLastError();
}

int norm_blocks_x(int nb) { return (nb + DBN - 1) / DBN; }
int norm_blocks_y(int m) { return (m + DBM - 1) / DBM; }

}  // namespace ctpd
