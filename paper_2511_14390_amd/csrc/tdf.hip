// tdf.hip -- the transposed direct form II with an initial state (the
// paper's own realisation, Sec. 2: the state-space form of Eqs. 4-5 with the
// companion matrix transposed and B, C swapped; SciPy's lfilter with zi),
// time-invariant coefficients.
//
// With K = max(M, N), b_j = 0 past M and a_j = 0 past N, the state z after
// sample n satisfies y(n) = b_0 x(n) + z_0(n-1) and
// z_i(n) = b_{i+1} x(n) - a_{i+1} y(n) + z_{i+1}(n-1), z(-1) = zi.  Unrolled,
// y(n) = sum_k b_k x(n-k) - sum_k a_k y(n-k) + zi_n [n < K] with x and y zero
// before time 0: the direct form driven by u = b * x plus the initial state
// entering as an input over the first K samples.  So the forward forms u in
// one pass and runs the all-pole path on it, and the backward is the
// all-pole adjoint ybar of gy (the adjoint filter of Sec. 3.1 Eq. 7, with ga
// from its reductions) followed by one pass for the feed-forward part:
// gx(n) = sum_k b_k ybar(n+k), gzi_j = ybar(j), gb_k = sum_n ybar(n) x(n-k).
#include "common.h"

namespace filt_detail {
namespace {

constexpr int kTdfThreads = 256;
constexpr int kTdfBlock = 256;  // samples per partial sum of gb

// u of every (channel, sample), consecutive threads consecutive elements of
// the layout; FP64 sums.
__global__ void __launch_bounds__(kTdfThreads)
k_tdf_input(Dims d, const float *__restrict__ x, const float *__restrict__ b,
            const float *__restrict__ zi, int K, float *__restrict__ u)
{
    const int64_t total = d.B * d.T;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const bool tb = d.layout == FILT_LAYOUT_TB;
        const int64_t bb = tb ? g % d.B : g / d.T;
        const int64_t t = tb ? g / d.B : g % d.T;
        double acc = 0.0;
        const float *br = b + bb * (d.M + 1);
        for (int k = 0; k <= d.M; ++k)
            if (t - k >= 0)
                acc += (double)br[k] * (double)x[sig_at(d, bb, t - k)];
        if (zi != nullptr && t < K)
            acc += (double)zi[bb * K + t];
        u[g] = (float)acc;
    }
}

// gx(n) = sum_k b_k ybar(n+k) (n + k < T) and gzi_j = ybar(j) (zero past T).
__global__ void __launch_bounds__(kTdfThreads)
k_tdf_fir_adjoint(Dims d, const float *__restrict__ ybar, const float *__restrict__ b, int K,
                  float *__restrict__ gx, float *__restrict__ gzi)
{
    const int64_t total = d.B * d.T;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const bool tb = d.layout == FILT_LAYOUT_TB;
        const int64_t bb = tb ? g % d.B : g / d.T;
        const int64_t t = tb ? g / d.B : g % d.T;
        if (gx != nullptr) {
            double acc = 0.0;
            const float *br = b + bb * (d.M + 1);
            for (int k = 0; k <= d.M; ++k)
                if (t + k < d.T)
                    acc += (double)br[k] * (double)ybar[sig_at(d, bb, t + k)];
            gx[g] = (float)acc;
        }
        if (gzi != nullptr && t < K)
            gzi[bb * K + t] = ybar[g];
    }
    // initial-state entries past the signal's end get no gradient
    if (gzi != nullptr)
        for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < d.B * K;
             g += (int64_t)gridDim.x * blockDim.x)
            if (g % K >= d.T)
                gzi[g] = 0.f;
}

// gb partial sums: thread (channel, block of kTdfBlock samples) sums
// ybar(n) x(n-k) for k = 0..M over its block, with the x values its taps
// read in a shift register.  part[(b * nblk + blk) * (M + 1) + k].
__global__ void __launch_bounds__(kTdfThreads)
k_tdf_gb_partial(Dims d, const float *__restrict__ ybar, const float *__restrict__ x,
                 int64_t nblk, double *__restrict__ part)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= d.B * nblk)
        return;
    // channels fastest in [T, B] (coalesced), blocks fastest in [B, T]
    const bool tb = d.layout == FILT_LAYOUT_TB;
    const int64_t bb = tb ? g % d.B : g / nblk;
    const int64_t blk = tb ? g / d.B : g % nblk;
    const int64_t t0 = blk * kTdfBlock, t1 = min(t0 + kTdfBlock, d.T);
    constexpr int KM = kMaxOrder + 1;
    double acc[KM], w[KM];  // w[k] = x(t - k) for the step t about to run
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        acc[k] = 0.0;
        const int64_t s = t0 - k;
        w[k] = (k <= d.M && s >= 0) ? (double)x[sig_at(d, bb, s)] : 0.0;
    }
    for (int64_t t = t0; t < t1; ++t) {
        const double yb = (double)ybar[sig_at(d, bb, t)];
#pragma unroll
        for (int k = 0; k < KM; ++k)
            acc[k] = __builtin_fma(yb, w[k], acc[k]);
#pragma unroll
        for (int k = KM - 1; k > 0; --k)
            w[k] = w[k - 1];
        w[0] = t + 1 < d.T ? (double)x[sig_at(d, bb, t + 1)] : 0.0;
    }
    double *o = part + (bb * nblk + blk) * (d.M + 1);
#pragma unroll
    for (int k = 0; k < KM; ++k)
        if (k <= d.M)
            o[k] = acc[k];
}

__global__ void __launch_bounds__(kTdfThreads)
k_tdf_gb_final(Dims d, const double *__restrict__ part, int64_t nblk, float *__restrict__ gb)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int K = d.M + 1;
    if (g >= d.B * K)
        return;
    const int64_t bb = g / K;
    const int k = (int)(g % K);
    double acc = 0.0;
    for (int64_t blk = 0; blk < nblk; ++blk)
        acc += part[(bb * nblk + blk) * K + k];
    gb[g] = (float)acc;
}

__global__ void __launch_bounds__(kTdfThreads) k_tdf_zero(float *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

unsigned grid_of(int64_t n)
{
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kTdfThreads - 1) / kTdfThreads,
                                                             kCUs * 16));
}

// The all-pole problem the transposed form runs (b = [1], zero initial
// conditions).
filt_problem allpole_of(const filt_problem *p)
{
    filt_problem q = *p;
    q.M = 0;
    return q;
}

filt_status tdf_check(const filt_problem *p)
{
    if (p == nullptr)
        return fail(FILT_EINVAL, "problem is NULL");
    if (p->time_varying != 0)
        return fail(FILT_EUNSUPPORTED,
                    "the transposed direct form takes time-invariant coefficients only");
    if (p->flags & ~(FILT_F32_STATE | FILT_RECURRENCE | FILT_TOEPLITZ))
        return fail(FILT_EINVAL, "unknown flags 0x%x", p->flags);
    return FILT_OK;
}

struct TdfWs {
    size_t sig, inner, part, total;  // offsets from the 256-byte aligned start
    int64_t nblk;
};

filt_status tdf_ws(const filt_problem *p, TdfWs &w)
{
    filt_problem q = allpole_of(p);
    size_t inner = 0;
    filt_status s = filt_workspace_bytes(&q, &inner);
    if (s != FILT_OK)
        return s;
    w.nblk = (p->T + kTdfBlock - 1) / kTdfBlock;
    w.sig = 0;
    w.inner = align256((size_t)(p->B * p->T) * sizeof(float));
    w.part = w.inner + align256(inner);
    w.total = w.part + align256((size_t)(p->B * w.nblk * (p->M + 1)) * sizeof(double)) + 256;
    return FILT_OK;
}

}  // namespace
}  // namespace filt_detail

using namespace filt_detail;

extern "C" {

filt_status filt_tdf_workspace_bytes(const filt_problem *p, size_t *bytes)
{
    filt_status s = tdf_check(p);
    if (s != FILT_OK)
        return s;
    if (bytes == nullptr)
        return fail(FILT_EINVAL, "bytes is NULL");
    size_t plain = 0;
    s = filt_workspace_bytes(p, &plain);  // validates the problem
    if (s != FILT_OK)
        return s;
    if (p->B == 0 || p->T == 0) {
        *bytes = 0;
        return FILT_OK;
    }
    TdfWs w;
    s = tdf_ws(p, w);
    if (s == FILT_OK)
        *bytes = w.total;
    return s;
}

filt_status filt_tdf_forward(const filt_problem *p, const float *x, const float *b,
                             const float *a, const float *zi, float *y, void *ws, size_t ws_bytes,
                             void *stream)
{
    size_t need = 0;
    filt_status s = filt_tdf_workspace_bytes(p, &need);
    if (s != FILT_OK)
        return s;
    if (p->B == 0 || p->T == 0)
        return FILT_OK;
    if (x == nullptr || y == nullptr || b == nullptr)
        return fail(FILT_EINVAL, "x, b and y are required");
    if (a == nullptr && p->N > 0)
        return fail(FILT_EINVAL, "a is NULL but N=%d", p->N);
    if (ws == nullptr || ws_bytes < need)
        return fail(FILT_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need,
                    ws == nullptr ? (size_t)0 : ws_bytes);
    TdfWs w;
    tdf_ws(p, w);
    char *base = (char *)(((uintptr_t)ws + 255) & ~uintptr_t(255));
    const size_t used = (size_t)(base - (char *)ws);
    Dims d{};
    d.B = p->B;
    d.T = p->T;
    d.M = p->M;
    d.N = p->N;
    d.layout = p->layout;
    const int K = std::max(std::max(p->M, p->N), 1);
    hipStream_t st = (hipStream_t)stream;
    float *u = (float *)(base + w.sig);
    FILT_LAUNCH("tdf_input", k_tdf_input, dim3(grid_of(p->B * p->T)), dim3(kTdfThreads), 0, st,
                d, x, b, zi, K, u);
    s = check_launch("transposed-form input");
    if (s != FILT_OK)
        return s;
    const filt_problem q = allpole_of(p);
    return filt_forward(&q, u, nullptr, a, nullptr, nullptr, y, base + w.inner,
                        ws_bytes - used - w.inner, stream);
}

filt_status filt_tdf_backward(const filt_problem *p, const float *gy, const float *x,
                              const float *y, const float *b, const float *a, const float *zi,
                              float *gx, float *gb, float *ga, float *gzi, void *ws,
                              size_t ws_bytes, void *stream)
{
    (void)zi;  // the gradients do not depend on the initial state's value
    size_t need = 0;
    filt_status s = filt_tdf_workspace_bytes(p, &need);
    if (s != FILT_OK)
        return s;
    const int K = std::max(std::max(p->M, p->N), 1);
    hipStream_t st = (hipStream_t)stream;
    if (p->B == 0)
        return FILT_OK;
    if (p->T == 0) {
        // no output: the per-channel gradients are zero (a fill kernel, not a
        // memset node, so the call stays capturable)
        const int64_t n[3] = {gb != nullptr ? p->B * (p->M + 1) : 0,
                              ga != nullptr ? p->B * p->N : 0, gzi != nullptr ? p->B * K : 0};
        float *o[3] = {gb, ga, gzi};
        for (int i = 0; i < 3; ++i)
            if (n[i] > 0)
                FILT_LAUNCH("tdf_zero", k_tdf_zero, dim3(grid_of(n[i])), dim3(kTdfThreads), 0,
                            st, o[i], n[i]);
        return check_launch("transposed-form zero fill");
    }
    if (gy == nullptr || b == nullptr)
        return fail(FILT_EINVAL, "gy and b are required");
    if (ga != nullptr && (y == nullptr || a == nullptr || p->N == 0))
        return fail(FILT_EINVAL, "ga requested but y or a is NULL, or N == 0");
    if (gb != nullptr && x == nullptr)
        return fail(FILT_EINVAL, "gb requested but x is NULL");
    if (a == nullptr && p->N > 0)
        return fail(FILT_EINVAL, "a is NULL but N=%d", p->N);
    if (ws == nullptr || ws_bytes < need)
        return fail(FILT_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need,
                    ws == nullptr ? (size_t)0 : ws_bytes);
    TdfWs w;
    tdf_ws(p, w);
    char *base = (char *)(((uintptr_t)ws + 255) & ~uintptr_t(255));
    const size_t used = (size_t)(base - (char *)ws);
    float *ybar = (float *)(base + w.sig);
    // the all-pole adjoint: gx of the problem with b = [1] is ybar, ga its
    // reduction with y (zero before time 0)
    const filt_problem q = allpole_of(p);
    s = filt_backward(&q, gy, nullptr, y, nullptr, a, nullptr, nullptr, ybar, nullptr, ga,
                      nullptr, nullptr, base + w.inner, ws_bytes - used - w.inner, stream);
    if (s != FILT_OK)
        return s;
    Dims d{};
    d.B = p->B;
    d.T = p->T;
    d.M = p->M;
    d.N = p->N;
    d.layout = p->layout;
    if (gx != nullptr || gzi != nullptr) {
        FILT_LAUNCH("tdf_fir_adjoint", k_tdf_fir_adjoint, dim3(grid_of(p->B * p->T)),
                    dim3(kTdfThreads), 0, st, d, ybar, b, K, gx, gzi);
        s = check_launch("transposed-form adjoint");
        if (s != FILT_OK)
            return s;
    }
    if (gb != nullptr) {
        double *part = (double *)(base + w.part);
        const int64_t n = p->B * w.nblk;
        FILT_LAUNCH("tdf_gb_partial", k_tdf_gb_partial,
                    dim3((unsigned)((n + kTdfThreads - 1) / kTdfThreads)), dim3(kTdfThreads), 0,
                    st, d, ybar, x, w.nblk, part);
        const int64_t m = p->B * (p->M + 1);
        FILT_LAUNCH("tdf_gb_final", k_tdf_gb_final,
                    dim3((unsigned)((m + kTdfThreads - 1) / kTdfThreads)), dim3(kTdfThreads), 0,
                    st, d, part, w.nblk, gb);
        s = check_launch("transposed-form gb");
    }
    return s;
}

}  // extern "C"
