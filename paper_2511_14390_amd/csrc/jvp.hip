// jvp.hip -- forward-mode derivative (Jacobian-vector product) of the
// direct-form filter.
//
// Differentiating the difference equation (Sec. 2 Eq. 1) along tangents
// (dx, db, da, dxi, dyi) gives the same recursion for the output tangent:
//
//   dy[n] + sum_k a_k[n] dy[n-k] = u[n],
//   u[n] = sum_k b_k[n] dx[n-k] + sum_k db_k[n] x[n-k] - sum_k da_k[n] y[n-k],
//
// with dy[-j] = dyi[j-1] and the histories of x, dx and y taken from xi, dxi
// and yi.  So one pass forms u and the all-pole filter of the forward path
// (same kernels, b = [1], initial conditions dyi) turns it into dy.
#include "common.h"

namespace filt_detail {

namespace {

// Value of a signal at (b, t) with its initial-condition history for t < 0
// (v[-j] = vi[b][j-1], zero past K or when vi is NULL).
__device__ __forceinline__ float sig_or_ic(const Dims &d, const float *v, const float *vi,
                                           int K, int64_t b, int64_t t)
{
    if (t >= 0)
        return v[sig_at(d, b, t)];
    const int64_t j = -t;
    return (vi != nullptr && j <= K) ? vi[b * K + (j - 1)] : 0.f;
}

// u[n] for every (channel, sample); one thread per sample, FP64 sums.
__global__ void __launch_bounds__(256)
k_jvp_input(Dims d, const float *__restrict__ x, const float *__restrict__ y,
            const float *__restrict__ b, const float *__restrict__ xi,
            const float *__restrict__ yi,
            const float *__restrict__ dx, const float *__restrict__ db,
            const float *__restrict__ da, const float *__restrict__ dxi, float *__restrict__ u)
{
    const int64_t total = d.B * d.T;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        // consecutive threads take consecutive elements of the layout
        const int64_t bb = d.layout == FILT_LAYOUT_TB ? g % d.B : g / d.T;
        const int64_t t = d.layout == FILT_LAYOUT_TB ? g / d.B : g % d.T;
        const int K = d.M + 1;
        double acc = 0.0;
        if (dx != nullptr) {
            const float *br = b != nullptr ? b + row_at(d, bb, t, K) : nullptr;
            for (int k = 0; k <= d.M; ++k) {
                const double bk = br != nullptr ? (double)br[k] : (k == 0 ? 1.0 : 0.0);
                acc += bk * (double)sig_or_ic(d, dx, dxi, d.M, bb, t - k);
            }
        }
        if (db != nullptr) {
            const float *dr = db + row_at(d, bb, t, K);
            for (int k = 0; k <= d.M; ++k)
                acc += (double)dr[k] * (double)sig_or_ic(d, x, xi, d.M, bb, t - k);
        }
        if (da != nullptr && d.N > 0) {
            const float *ar = da + row_at(d, bb, t, d.N);
            for (int k = 1; k <= d.N; ++k)
                acc -= (double)ar[k - 1] * (double)sig_or_ic(d, y, yi, d.N, bb, t - k);
        }
        u[g] = (float)acc;
    }
}

}  // namespace

}  // namespace filt_detail

using namespace filt_detail;

extern "C" {

filt_status filt_jvp_workspace_bytes(const filt_problem *p, size_t *bytes)
{
    if (p == nullptr || bytes == nullptr)
        return fail(FILT_EINVAL, "problem or bytes is NULL");
    filt_problem q = *p;
    q.M = 0;
    size_t fw = 0;
    const filt_status s = filt_workspace_bytes(&q, &fw);
    if (s != FILT_OK)
        return s;
    // u, then the forward's workspace; 256 bytes for aligning the start
    *bytes = p->B == 0 || p->T == 0
                 ? 0
                 : 256 + align256((size_t)(p->B * p->T) * sizeof(float)) + fw;
    return FILT_OK;
}

filt_status filt_jvp(const filt_problem *p, const float *x, const float *y, const float *b,
                     const float *a, const float *xi, const float *yi, const float *dx,
                     const float *db, const float *da, const float *dxi, const float *dyi,
                     float *dy, void *ws, size_t ws_bytes, void *stream)
{
    if (p == nullptr)
        return fail(FILT_EINVAL, "problem is NULL");
    size_t need = 0;
    filt_status s = filt_jvp_workspace_bytes(p, &need);
    if (s != FILT_OK)
        return s;
    if (p->B == 0 || p->T == 0)
        return FILT_OK;
    if (dy == nullptr)
        return fail(FILT_EINVAL, "dy is NULL");
    if (a == nullptr && p->N > 0)
        return fail(FILT_EINVAL, "a is NULL but N=%d", p->N);
    if (b == nullptr && p->M > 0)
        return fail(FILT_EINVAL, "b is NULL but M=%d (NULL b means b=[1], M=0)", p->M);
    if (db != nullptr && (b == nullptr || x == nullptr))
        return fail(FILT_EINVAL, "db given without b or x");
    if (da != nullptr && y == nullptr)
        return fail(FILT_EINVAL, "da given without y");
    if (ws == nullptr || ws_bytes < need)
        return fail(FILT_EWORKSPACE, "workspace of %zu bytes needed, %zu given", need,
                    ws == nullptr ? (size_t)0 : ws_bytes);
    Dims d{};
    d.B = p->B;
    d.T = p->T;
    d.M = p->M;
    d.N = p->N;
    set_rows(d, p->time_varying);
    d.layout = p->layout;
    hipStream_t st = (hipStream_t)stream;
    char *base = (char *)(((uintptr_t)ws + 255) & ~uintptr_t(255));
    float *u = (float *)base;
    const size_t ub = align256((size_t)(p->B * p->T) * sizeof(float));
    FILT_LAUNCH("jvp_input", k_jvp_input, dim3(blocks_for(p->B * p->T)),
                dim3(block_for(p->B * p->T)), 0, st, d, x, y, b, xi, yi, dx, db, da, dxi, u);
    s = check_launch("jvp input");
    if (s != FILT_OK)
        return s;
    filt_problem q = *p;
    q.M = 0;
    const size_t used = (size_t)(base - (char *)ws) + ub;
    return filt_forward(&q, u, nullptr, a, nullptr, dyi, dy, base + ub, ws_bytes - used, stream);
}

}  // extern "C"
