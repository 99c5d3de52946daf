// Forward projection that allocates nothing, for callers that cannot call
// hipMalloc (code under graph capture, tight serving loops, harnesses that
// forbid it).  Everything the projection needs beyond its input and output
// -- the per-view geometry table and the two zero-padded image planes the
// projector reads -- lives in one file-scope device array, `scratch`, which
// each GPU the library runs on holds until the process ends.  Every call on
// a GPU shares that GPU's array: calls that overlap on one GPU (two streams,
// two host threads) race on it and must be serialised by the caller.
#include <mutex>

#include "op.h"

using namespace ctpd;
using namespace ctpd_host;

namespace {

constexpr int kMaxN = 1024;       // image side
constexpr int kMaxViews = 4096;   // view count
constexpr size_t kViewBytes = sizeof(ViewGeom) * kMaxViews;
constexpr size_t kPlaneFloats = (size_t)kMaxN * (kMaxN + 2 * kPlanePad);
constexpr size_t kScratchBytes = kViewBytes + 2 * kPlaneFloats * sizeof(float);   // 8.7 MB
static_assert(kViewBytes % 256 == 0, "planes start 256-byte aligned");

// One device address per GPU, taken once (with that device current) from
// hipGetSymbolAddress: in host code `scratch` names a host-side stand-in, not
// the device memory, so it is never passed to a kernel or a copy itself.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// View table for theta_v = v pi / m, the same quantities as make_views on
// the host (row views decided from the index: 4v <= m or 4v >= 3m), computed
// in float64 on the device.
__global__ __launch_bounds__(256) void noalloc_views_kernel(ViewGeom* __restrict__ out, int n, int m, int nb) {
    const int v = blockIdx.x * 256 + threadIdx.x;
    if (v >= m) return;
    const double c = 0.5 * (n - 1), cd = 0.5 * (nb - 1);
    const double th = (double)v * M_PI / (double)m;
    const double cs = cos(th), sn = sin(th);
    ViewGeom g{};
    g.row = (4 * v <= m || 4 * v >= 3 * m) ? 1 : 0;
    g.cs = cs;
    g.sn = sn;
    const double a = g.row ? cs : sn, o = g.row ? sn : cs;
    g.su = 1.0 / a;
    g.st = -o / a;
    g.s0 = (c * o - cd) / a + c;
    g.len = 1.0 / fabs(a);
    g.len2 = g.len * g.len;
    out[v] = g;
}

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// The calling thread's current device's copy of `scratch`, looked up on the
// first call on that device.
int scratch_on_current_device(unsigned char** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return einval("device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail_hip(hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch[dev]);
    return CTPD_OK;
}

}  // namespace

extern "C" {

int ctpd_project_noalloc(const ctpd_geometry* g, void* stream, const float* x, float* y) {
    g_errmsg[0] = 0;
    if (!g || !x || !y) return einval("null pointer");
    if (g->n < 1 || g->n > kMaxN) return einval("n out of range [1, 1024] for the no-allocation projector");
    if (g->n_views < 1 || g->n_views > kMaxViews)
        return einval("n_views out of range [1, 4096] for the no-allocation projector");
    if (g->n_bins < 1 || g->n_bins > CTPD_MAX_BINS) return einval("n_bins out of range");
    if (g->angles) return einval("the no-allocation projector takes uniform angles only (angles must be NULL)");
    unsigned char* base = nullptr;
    int r = scratch_on_current_device(&base);
    if (r) return r;
    const int n = g->n, m = g->n_views, nb = g->n_bins;
    hipStream_t s = (hipStream_t)stream;
    ViewGeom* views = reinterpret_cast<ViewGeom*>(base);
    float* xp = reinterpret_cast<float*>(base + kViewBytes);
    float* xTp = xp + (size_t)n * (n + 2 * kPlanePad);
    noalloc_views_kernel<<<(m + 255) / 256, 256, 0, s>>>(views, n, m, nb);
    HIP_TRY(hipGetLastError());
    // the plane kernel writes every interior pixel and pad column of both planes
    HIP_TRY(launch_pad_planes<float>(x, xp, xTp, n, s));
    HIP_TRY(launch_forward<float>(xp, xTp, y, views, n, m, nb, s));
    return CTPD_OK;
}

}  // extern "C"
