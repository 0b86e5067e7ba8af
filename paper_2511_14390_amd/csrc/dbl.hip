// dbl.hip -- derivative of the backward pass (second-order use: Hessian-
// vector products by reverse over reverse; the paper's closing remarks name
// second-order optimisation as the use of forward-mode differentiation, which
// this builds on).
//
// filt_backward maps gy (and x, y, a, b, xi, yi, with y an input of its own)
// to g = (gx, gb, ga, gxi, gyi), the transposed Jacobian of the forward
// applied to gy.  For cotangents v = (vx, vb, va, vxi, vyi) of those outputs,
// Q = <v, g> = <gy, dy> with dy the forward-mode tangent along v (filt_jvp),
// and with ybar the adjoint of gy (ybar[n] = gy[n] - sum_k a_k[n+k] ybar[n+k])
//   dQ/dgy      = dy
//   dQ/dx[m]    = sum_{k=0..M} vb_k[m+k] ybar[m+k],   dQ/dxi likewise
//   dQ/db_k[n]  = ybar[n] vx[n-k]          (vx's history vxi)
//   dQ/dy[m]    = -sum_{k=1..N} va_k[m+k] ybar[m+k],  dQ/dyi likewise
//   dQ/da_k[n]  = -ybar[n] dy[n-k]         (dy's history vyi)
// (time-invariant coefficients: the last lines summed over n, frame-held
// ones over each frame).
//
// Every line is a pass the library already has:
//   dy   : filt_jvp;
//   ybar : filt_backward with b = [1] (its gx is the adjoint);
//   x, xi, b lines : filt_backward of the feed-forward filter vb (N = 0) on
//          ybar with input vx (history vxi): gx, gxi, gb;
//   y, yi, a lines : filt_backward of the feed-forward filter
//          c = [0, va_1 .. va_N] (N = 0, N + 1 taps) on -ybar with input dy
//          (history vyi): gx, gxi, and gb taps 1..N.
// The small kernels below negate ybar, build c and drop c's tap 0 from its
// gradient.
#include "common.h"

namespace filt_detail {
namespace {

__global__ void __launch_bounds__(256) k_fill(float *__restrict__ p, int64_t n, float v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void __launch_bounds__(256) k_negate(float *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = -p[i];
}

// c[r][0] = 0, c[r][k] = va[r][k-1] (zero when va is NULL), r < R rows.
__global__ void __launch_bounds__(256)
k_prepend_zero_tap(const float *__restrict__ va, float *__restrict__ c, int64_t R, int N)
{
    const int64_t n = R * (N + 1);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / (N + 1);
        const int k = (int)(i - r * (N + 1));
        c[i] = (k == 0 || va == nullptr) ? 0.f : va[r * N + (k - 1)];
    }
}

// wa[r][k-1] = g[r][k] for k = 1..N.
__global__ void __launch_bounds__(256)
k_drop_tap0(const float *__restrict__ g, float *__restrict__ wa, int64_t R, int N)
{
    const int64_t n = R * N;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / N;
        const int k = (int)(i - r * N);
        wa[i] = g[r * (N + 1) + k + 1];
    }
}

// grid-stride launches: at most 8192 groups of 256
unsigned stride_grid(int64_t n)
{
    const int64_t g = (n + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

filt_status fill(float *p, int64_t n, float v, hipStream_t st)
{
    if (p == nullptr || n <= 0)
        return FILT_OK;
    FILT_LAUNCH("dbl_fill", k_fill, dim3(stride_grid(n)), dim3(256), 0, st, p, n, v);
    return check_launch("fill");
}

// Coefficient rows of the problem: one per channel (time-invariant), per
// sample, or per frame of time_varying samples.
int64_t coef_rows(const filt_problem *p)
{
    if (p->time_varying == 0)
        return p->B;
    if (p->time_varying == 1)
        return p->B * p->T;
    return p->B * ((p->T + p->time_varying - 1) / p->time_varying);
}

struct DblPlan {
    filt_problem p0, p3, p4;  // adjoint (b = [1]); feed-forward vb; feed-forward c
    size_t ybar, z, zsig, zcoef, c, gc, inner, total;
};

filt_status dbl_plan(const filt_problem *p, DblPlan &w)
{
    w.p0 = *p;
    w.p0.M = 0;
    w.p3 = *p;
    w.p3.N = 0;
    w.p4 = *p;
    w.p4.M = p->N;
    w.p4.N = 0;
    size_t b0 = 0, b3 = 0, b4 = 0, bj = 0;
    filt_status s = filt_workspace_bytes(&w.p0, &b0);
    if (s == FILT_OK)
        s = filt_workspace_bytes(&w.p3, &b3);
    if (s == FILT_OK)
        s = filt_workspace_bytes(&w.p4, &b4);
    if (s == FILT_OK)
        s = filt_jvp_workspace_bytes(p, &bj);
    if (s != FILT_OK)
        return s;
    const size_t sig = align256((size_t)(p->B * p->T) * sizeof(float));
    const int64_t R = coef_rows(p);
    size_t off = 0;
    w.ybar = off;
    off += sig;
    w.z = off;
    off += sig;
    w.zsig = off;
    off += sig;
    w.zcoef = off;
    off += align256((size_t)R * (p->M + 1) * sizeof(float));
    w.c = off;
    off += align256((size_t)R * (p->N + 1) * sizeof(float));
    w.gc = off;
    off += align256((size_t)R * (p->N + 1) * sizeof(float));
    w.inner = off;
    off += align256(std::max(std::max(b0, b3), std::max(b4, bj)));
    w.total = 256 + off;
    return FILT_OK;
}

}  // namespace
}  // namespace filt_detail

using namespace filt_detail;

extern "C" {

filt_status filt_backward2_workspace_bytes(const filt_problem *p, size_t *bytes)
{
    if (p == nullptr || bytes == nullptr)
        return fail(FILT_EINVAL, "problem or bytes is NULL");
    if (p->B < 0 || p->T < 0)
        return fail(FILT_EINVAL, "B and T must be >= 0");
    if (p->B == 0 || p->T == 0) {
        *bytes = 0;
        return FILT_OK;
    }
    DblPlan w;
    const filt_status s = dbl_plan(p, w);
    if (s != FILT_OK)
        return s;
    *bytes = w.total;
    return FILT_OK;
}

filt_status filt_backward2(const filt_problem *p, const float *gy, const float *x,
                           const float *y, const float *b, const float *a, const float *xi,
                           const float *yi, const float *vx, const float *vb, const float *va,
                           const float *vxi, const float *vyi, float *wgy, float *wx, float *wy,
                           float *wb, float *wa, float *wxi, float *wyi, void *ws,
                           size_t ws_bytes, void *stream)
{
    if (p == nullptr)
        return fail(FILT_EINVAL, "problem is NULL");
    if (p->B < 0 || p->T < 0 || p->M < 0 || p->N < 0)
        return fail(FILT_EINVAL, "B, T, M and N must be >= 0");
    if (b == nullptr && (p->M != 0 || vb != nullptr || wb != nullptr))
        return fail(FILT_EINVAL, "b is NULL (b = [1]): M must be 0 and vb, wb NULL");
    if (a == nullptr && p->N > 0)
        return fail(FILT_EINVAL, "a is NULL but N=%d", p->N);
    if (p->N == 0 && (va != nullptr || wa != nullptr))
        return fail(FILT_EINVAL, "va / wa given but N == 0");
    hipStream_t st = (hipStream_t)stream;
    if (p->B == 0 || p->T == 0) {
        // per-channel outputs are zero, per-sample ones empty (as filt_backward)
        if (p->B == 0)
            return FILT_OK;
        const bool ti = p->time_varying == 0;
        filt_status s = fill(wxi, p->B * (int64_t)p->M, 0.f, st);
        if (s == FILT_OK)
            s = fill(wyi, p->B * (int64_t)p->N, 0.f, st);
        if (s == FILT_OK && ti)
            s = fill(wb, p->B * (int64_t)(p->M + 1), 0.f, st);
        if (s == FILT_OK && ti)
            s = fill(wa, p->B * (int64_t)p->N, 0.f, st);
        return s;
    }
    if (gy == nullptr)
        return fail(FILT_EINVAL, "gy is NULL");
    if (vb != nullptr && x == nullptr)
        return fail(FILT_EINVAL, "vb given without x");
    if (va != nullptr && y == nullptr)
        return fail(FILT_EINVAL, "va given without y");
    DblPlan w;
    filt_status s = dbl_plan(p, w);
    if (s != FILT_OK)
        return s;
    if (ws == nullptr || ws_bytes < w.total)
        return fail(FILT_EWORKSPACE, "workspace of %zu bytes needed, %zu given", w.total,
                    ws == nullptr ? (size_t)0 : ws_bytes);
    char *base = (char *)(((uintptr_t)ws + 255) & ~uintptr_t(255));
    const size_t inner_bytes = ws_bytes - (size_t)(base - (char *)ws) - w.inner;
    void *inner = base + w.inner;
    float *ybar = (float *)(base + w.ybar);
    float *zs = (float *)(base + w.z);
    float *zsig = (float *)(base + w.zsig);
    float *zcoef = (float *)(base + w.zcoef);
    float *cc = (float *)(base + w.c);
    float *gcc = (float *)(base + w.gc);
    const int64_t n = p->B * p->T;
    const int64_t R = coef_rows(p);
    const int N = p->N, M = p->M;

    // dy, the forward-mode tangent along the cotangents
    const bool need_dy = wgy != nullptr || wa != nullptr;
    float *dy = wgy != nullptr ? wgy : zs;
    if (need_dy) {
        s = filt_jvp(p, x, y, b, a, xi, yi, vx, vb, va, vxi, vyi, dy, inner, inner_bytes,
                     stream);
        if (s != FILT_OK)
            return s;
    }
    const bool ff_part = wx != nullptr || wxi != nullptr || wb != nullptr;
    const bool ar_part = N > 0 && (wy != nullptr || wyi != nullptr || wa != nullptr);
    if (!ff_part && !ar_part) {
        return fill(wy, n, 0.f, st);
    }
    // ybar: the backward with b = [1] writes the adjoint as its gx
    s = filt_backward(&w.p0, gy, x, y, nullptr, a, nullptr, yi, ybar, nullptr, nullptr, nullptr,
                      nullptr, inner, inner_bytes, stream);
    if (s != FILT_OK)
        return s;
    // x, xi, b lines: the feed-forward filter vb adjoint on ybar, input vx
    if (b == nullptr) {
        s = fill(wx, n, 0.f, st);  // b = [1] has no cotangent: dQ/dx = 0
    } else if (ff_part) {
        const float *vbc = vb;
        if (vbc == nullptr) {
            s = fill(zcoef, R * (M + 1), 0.f, st);
            vbc = zcoef;
        }
        const float *vxs = vx;
        if (s == FILT_OK && wb != nullptr && vxs == nullptr) {
            s = fill(zsig, n, 0.f, st);
            vxs = zsig;
        }
        if (s == FILT_OK)
            s = filt_backward(&w.p3, ybar, vxs != nullptr ? vxs : ybar, nullptr, vbc, nullptr,
                              wb != nullptr ? vxi : nullptr, nullptr, wx, wb, nullptr, wxi,
                              nullptr, inner, inner_bytes, stream);
    }
    if (s != FILT_OK)
        return s;
    if (!ar_part)
        return fill(wy, n, 0.f, st);
    // y, yi, a lines: the feed-forward filter [0, va] adjoint on -ybar,
    // input dy with history vyi
    FILT_LAUNCH("dbl_negate", k_negate, dim3(stride_grid(n)), dim3(256), 0, st, ybar, n);
    FILT_LAUNCH("dbl_taps", k_prepend_zero_tap, dim3(stride_grid(R * (N + 1))), dim3(256), 0, st,
                va, cc, R, N);
    s = check_launch("cotangent taps");
    if (s != FILT_OK)
        return s;
    s = filt_backward(&w.p4, ybar, wa != nullptr ? dy : ybar, nullptr, cc, nullptr,
                      wa != nullptr ? vyi : nullptr, nullptr, wy, wa != nullptr ? gcc : nullptr,
                      nullptr, wyi, nullptr, inner, inner_bytes, stream);
    if (s != FILT_OK || wa == nullptr)
        return s;
    FILT_LAUNCH("dbl_drop_tap0", k_drop_tap0, dim3(stride_grid(R * N)), dim3(256), 0, st, gcc, wa,
                R, N);
    return check_launch("coefficient gradient taps");
}

}  // extern "C"
