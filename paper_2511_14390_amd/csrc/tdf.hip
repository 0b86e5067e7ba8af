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

// Kernels templated on the feed-forward order M (0..16).
#define TDF_ORDERS(X)                                                                              \
    X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)
constexpr int kTdfBlock = 256;  // samples per partial sum of gb

// Tiles of kTdfThreads consecutive elements of a row of the layout (a time
// step in [T, B], a channel in [B, T]) over the grid, one element per
// thread: consecutive threads take consecutive elements (coalesced), and
// indices are divided once per tile, not per element.
template <typename F>
__device__ __forceinline__ void tdf_for_each(const Dims &d, F &&f)
{
    const bool tb = d.layout == FILT_LAYOUT_TB;
    const int64_t rows = tb ? d.T : d.B, cols = tb ? d.B : d.T;
    const int64_t tiles = (cols + kTdfThreads - 1) / kTdfThreads;
    for (int64_t i = blockIdx.x; i < rows * tiles; i += gridDim.x) {
        const int64_t r = i / tiles;
        const int64_t c = (i - r * tiles) * kTdfThreads + threadIdx.x;
        if (c < cols)
            f(tb ? r : c, tb ? c : r);  // (t, channel)
    }
}

// u of every (channel, sample); FP64 sums.  MM = M (taps b_0..b_MM, all
// loads of an element issued together).
template <int MM>
__global__ void __launch_bounds__(kTdfThreads)
k_tdf_input(Dims d, const float *__restrict__ x, const float *__restrict__ b,
            const float *__restrict__ zi, int K, float *__restrict__ u)
{
    const int64_t step = d.layout == FILT_LAYOUT_TB ? d.B : 1;
    tdf_for_each(d, [&](int64_t t, int64_t bb) {
        const float *br = b + bb * (MM + 1);
        const int64_t e = sig_at(d, bb, t);
        float xv[MM + 1];
#pragma unroll
        for (int k = 0; k <= MM; ++k)
            xv[k] = t - k >= 0 ? x[e - k * step] : 0.f;
        double acc = (zi != nullptr && t < K) ? (double)zi[bb * K + t] : 0.0;
#pragma unroll
        for (int k = 0; k <= MM; ++k)
            acc = __builtin_fma((double)br[k], (double)xv[k], acc);
        u[e] = (float)acc;
    });
}

// gx(n) = sum_k b_k ybar(n+k) (n + k < T) and gzi_j = ybar(j) (zero past T).
template <int MM>
__global__ void __launch_bounds__(kTdfThreads)
k_tdf_fir_adjoint(Dims d, const float *__restrict__ ybar, const float *__restrict__ b, int K,
                  float *__restrict__ gx, float *__restrict__ gzi)
{
    const int64_t step = d.layout == FILT_LAYOUT_TB ? d.B : 1;
    tdf_for_each(d, [&](int64_t t, int64_t bb) {
        const int64_t e = sig_at(d, bb, t);
        if (gx != nullptr) {
            const float *br = b + bb * (MM + 1);
            float yv[MM + 1];
#pragma unroll
            for (int k = 0; k <= MM; ++k)
                yv[k] = t + k < d.T ? ybar[e + k * step] : 0.f;
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k <= MM; ++k)
                acc = __builtin_fma((double)br[k], (double)yv[k], acc);
            gx[e] = (float)acc;
        }
        if (gzi != nullptr && t < K)
            gzi[bb * K + t] = ybar[e];
    });
    // initial-state entries past the signal's end get no gradient
    if (gzi != nullptr && d.T < K)
        for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < d.B * K;
             g += (int64_t)gridDim.x * blockDim.x)
            if (g % K >= d.T)
                gzi[g] = 0.f;
}

// [T, B]: one thread per channel walks kTdfRows consecutive time steps
// with the MM + 1 values its taps read in a shift register (one load per
// sample instead of MM + 1, and the coefficients loaded once); neighbouring
// threads are neighbouring channels.
constexpr int kTdfRows = kTdfBlock;  // adjoint runs: also the gb partial-sum block
constexpr int kTdfInRows = 64;       // forward input runs (more workgroups)
static_assert(kTdfRows % 16 == 0 && kTdfInRows % 16 == 0, "whole load blocks per run");

template <int MM>
__global__ void __launch_bounds__(kTdfThreads)
k_tdf_input_tb(Dims d, const float *__restrict__ x, const float *__restrict__ b,
               const float *__restrict__ zi, int K, float *__restrict__ u)
{
    const int64_t ntile = (d.B + kTdfThreads - 1) / kTdfThreads;
    const int64_t bb = (blockIdx.x % ntile) * kTdfThreads + threadIdx.x;
    const int64_t t0 = (int64_t)(blockIdx.x / ntile) * kTdfInRows;
    if (bb >= d.B || t0 >= d.T)
        return;
    const int64_t t1 = min(t0 + (int64_t)kTdfInRows, d.T);
    float bv[MM + 1];
    double w[MM + 1];  // w[k] = x(t - 1 - k) before step t shifts x(t) in
#pragma unroll
    for (int k = 0; k <= MM; ++k) {
        bv[k] = b[bb * (MM + 1) + k];
        w[k] = t0 - 1 - k >= 0 ? (double)x[(t0 - 1 - k) * d.B + bb] : 0.0;
    }
    // blocks of P steps: the block's loads issued before its arithmetic
    constexpr int P = 16;
    for (int64_t tq = t0; tq < t1; tq += P) {
        float xv[P];
#pragma unroll
        for (int q = 0; q < P; ++q)
            xv[q] = tq + q < t1 ? x[(tq + q) * d.B + bb] : 0.f;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int64_t t = tq + q;
            if (t >= t1)
                break;
#pragma unroll
            for (int k = MM; k > 0; --k)
                w[k] = w[k - 1];
            w[0] = (double)xv[q];
            double acc = (zi != nullptr && t < K) ? (double)zi[bb * K + t] : 0.0;
#pragma unroll
            for (int k = 0; k <= MM; ++k)
                acc = __builtin_fma((double)bv[k], w[k], acc);
            u[t * d.B + bb] = (float)acc;
        }
    }
}

// With x (gb wanted) the thread also keeps the MM + 1 values x(t - k) and
// writes its run's partial sums of gb_k = sum_t ybar(t) x(t - k) to
// part[(channel * nblk + run) * (MM + 1) + k].
template <int MM>
__global__ void __launch_bounds__(kTdfThreads)
k_tdf_fir_adjoint_tb(Dims d, const float *__restrict__ ybar, const float *__restrict__ b, int K,
                     float *__restrict__ gx, float *__restrict__ gzi,
                     const float *__restrict__ x, int64_t nblk, double *__restrict__ part)
{
    const int64_t ntile = (d.B + kTdfThreads - 1) / kTdfThreads;
    const int64_t bb = (blockIdx.x % ntile) * kTdfThreads + threadIdx.x;
    const int64_t t0 = (int64_t)(blockIdx.x / ntile) * kTdfRows;
    if (bb >= d.B || t0 >= d.T)
        return;
    const int64_t t1 = min(t0 + (int64_t)kTdfRows, d.T);
    float bv[MM + 1];
    // w[k] = ybar(t + 1 + k) before step t (time descending) shifts ybar(t) in
    double w[MM + 1];
#pragma unroll
    for (int k = 0; k <= MM; ++k) {
        bv[k] = b[bb * (MM + 1) + k];
        const int64_t s = t1 + k;
        w[k] = s < d.T ? (double)ybar[s * d.B + bb] : 0.0;
    }
    double xw[MM + 1], gacc[MM + 1];  // xw[k] = x(t - k) at step t
#pragma unroll
    for (int k = 0; k <= MM; ++k) {
        gacc[k] = 0.0;
        const int64_t s = t1 - 1 - k;
        xw[k] = (x != nullptr && s >= 0) ? (double)x[s * d.B + bb] : 0.0;
    }
    constexpr int P = 16;
    for (int64_t tq = t1 - 1; tq >= t0; tq -= P) {
      // the block's loads (steps tq, tq - 1, ..) issued before its arithmetic
      float yv[P], xv[P];
#pragma unroll
      for (int q = 0; q < P; ++q) {
          const int64_t t = tq - q, s = t - 1 - MM;
          yv[q] = t >= t0 ? ybar[t * d.B + bb] : 0.f;
          xv[q] = (x != nullptr && t >= t0 && s >= 0) ? x[s * d.B + bb] : 0.f;
      }
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const int64_t t = tq - q;
        if (t < t0)
            break;
#pragma unroll
        for (int k = MM; k > 0; --k)
            w[k] = w[k - 1];
        w[0] = (double)yv[q];
        if (gx != nullptr) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k <= MM; ++k)
                acc = __builtin_fma((double)bv[k], w[k], acc);
            gx[t * d.B + bb] = (float)acc;
        }
        if (gzi != nullptr && t < K)
            gzi[bb * K + t] = (float)w[0];
        if (x != nullptr) {
#pragma unroll
            for (int k = 0; k <= MM; ++k)
                gacc[k] = __builtin_fma(w[0], xw[k], gacc[k]);
            // the window moves one step back in time
#pragma unroll
            for (int k = 0; k < MM; ++k)
                xw[k] = xw[k + 1];
            xw[MM] = (double)xv[q];
        }
      }
    }
    if (x != nullptr) {
        double *o = part + (bb * nblk + t0 / kTdfRows) * (MM + 1);
#pragma unroll
        for (int k = 0; k <= MM; ++k)
            o[k] = gacc[k];
    }
    // initial-state entries past the signal's end get no gradient
    if (gzi != nullptr && t0 == 0)
        for (int j = (int)d.T; j < K; ++j)
            gzi[bb * K + j] = 0.f;
}

// gb partial sums: thread (channel, block of kTdfBlock samples) sums
// ybar(n) x(n-k) for k = 0..M over its block, with the x values its taps
// read in a shift register.  part[(b * nblk + blk) * (M + 1) + k].
template <int MM>
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
    constexpr int KM = MM + 1;
    double acc[KM], w[KM];  // w[k] = x(t - k) for the step t about to run
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        acc[k] = 0.0;
        const int64_t s = t0 - k;
        w[k] = s >= 0 ? (double)x[sig_at(d, bb, s)] : 0.0;
    }
    // blocks of P samples: every load of a block issued before its
    // arithmetic
    constexpr int P = 16;
    for (int64_t tb0 = t0; tb0 < t1; tb0 += P) {
        float yv[P], xv[P];
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int64_t t = tb0 + q;
            yv[q] = t < t1 ? ybar[sig_at(d, bb, t)] : 0.f;  // zero past the block
            xv[q] = t + 1 < d.T ? x[sig_at(d, bb, t + 1)] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const double yb = (double)yv[q];
#pragma unroll
            for (int k = 0; k < KM; ++k)
                acc[k] = __builtin_fma(yb, w[k], acc[k]);
#pragma unroll
            for (int k = KM - 1; k > 0; --k)
                w[k] = w[k - 1];
            w[0] = (double)xv[q];
        }
    }
    double *o = part + (bb * nblk + blk) * KM;
#pragma unroll
    for (int k = 0; k < KM; ++k)
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
    // eight independent sums so eight loads are in flight, added in a fixed
    // order at the end
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const double *pp = part + bb * nblk * K + k;
    int64_t blk = 0;
    for (; blk + 8 <= nblk; blk += 8)
#pragma unroll
        for (int i = 0; i < 8; ++i)
            acc[i] += pp[(blk + i) * K];
    for (; blk < nblk; ++blk)
        acc[0] += pp[blk * K];
    gb[g] = (float)(((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7])));
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

// One workgroup per tile of a row, at most 128 per CU (the rest in turn):
// these passes are one memory latency per tile, so they need many
// workgroups in flight.
unsigned rows_grid(const filt_problem *p)
{
    const bool tb = p->layout == FILT_LAYOUT_TB;
    const int64_t rows = tb ? p->T : p->B, cols = tb ? p->B : p->T;
    const int64_t tiles = rows * ((cols + kTdfThreads - 1) / kTdfThreads);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(tiles, kCUs * 128));
}

// [T, B] kernels: (channel tile, run of kTdfRows time steps) workgroups.
unsigned tb_grid(const filt_problem *p, int rows)
{
    const int64_t ntile = (p->B + kTdfThreads - 1) / kTdfThreads;
    return (unsigned)(ntile * ((p->T + rows - 1) / rows));
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
#define TDF_IN(MM)                                                                                 \
    case MM:                                                                                       \
        if (p->layout == FILT_LAYOUT_TB)                                                           \
            FILT_LAUNCH("tdf_input", k_tdf_input_tb<MM>, dim3(tb_grid(p, kTdfInRows)),             \
                        dim3(kTdfThreads), 0, st, d, x, b, zi, K, u);                              \
        else                                                                                       \
            FILT_LAUNCH("tdf_input", k_tdf_input<MM>, dim3(rows_grid(p)), dim3(kTdfThreads), 0,    \
                        st, d, x, b, zi, K, u);                                                    \
        break;
    switch (p->M) { TDF_ORDERS(TDF_IN) }
#undef TDF_IN
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
    // [T, B]: one pass forms gx, gzi and the gb partial sums; [B, T]: the
    // element pass for gx and gzi, the gb partial sums in a pass of their own
    double *part = (double *)(base + w.part);
    const bool tb = p->layout == FILT_LAYOUT_TB;
    if (gx != nullptr || gzi != nullptr || (tb && gb != nullptr)) {
#define TDF_ADJ(MM)                                                                                \
    case MM:                                                                                       \
        if (tb)                                                                                    \
            FILT_LAUNCH("tdf_fir_adjoint", k_tdf_fir_adjoint_tb<MM>, dim3(tb_grid(p, kTdfRows)),   \
                        dim3(kTdfThreads), 0, st, d, ybar, b, K, gx, gzi,                          \
                        gb != nullptr ? x : nullptr, w.nblk, part);                                \
        else                                                                                       \
            FILT_LAUNCH("tdf_fir_adjoint", k_tdf_fir_adjoint<MM>, dim3(rows_grid(p)),              \
                        dim3(kTdfThreads), 0, st, d, ybar, b, K, gx, gzi);                         \
        break;
        switch (p->M) { TDF_ORDERS(TDF_ADJ) }
#undef TDF_ADJ
        s = check_launch("transposed-form adjoint");
        if (s != FILT_OK)
            return s;
    }
    if (gb != nullptr) {
        if (!tb) {
            const int64_t n = p->B * w.nblk;
#define TDF_GB(MM)                                                                                 \
    case MM:                                                                                       \
        FILT_LAUNCH("tdf_gb_partial", k_tdf_gb_partial<MM>,                                        \
                    dim3((unsigned)((n + kTdfThreads - 1) / kTdfThreads)), dim3(kTdfThreads), 0,   \
                    st, d, ybar, x, w.nblk, part);                                                 \
        break;
            switch (p->M) { TDF_ORDERS(TDF_GB) }
#undef TDF_GB
        }
        const int64_t m = p->B * (p->M + 1);
        FILT_LAUNCH("tdf_gb_final", k_tdf_gb_final,
                    dim3((unsigned)((m + kTdfThreads - 1) / kTdfThreads)), dim3(kTdfThreads), 0,
                    st, d, part, w.nblk, gb);
        s = check_launch("transposed-form gb");
    }
    return s;
}

}  // extern "C"
