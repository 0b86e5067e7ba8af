// grads.hip -- per-sample coefficient gradients from a stored adjoint.
//
// With per-sample coefficients the gradients are one product per tap and
// sample (Sec. 3.1 Eqs. 8-9 without the sum over time):
//   ga_k[n] = -ybar[n] y[n-k]  (k = 1..N),   gb_k[n] = ybar[n] x[n-k]  (k = 0..M),
// with y[-j] = yi[j-1] and x[-j] = xi[j-1].
#include "common.h"

namespace filt_detail {
namespace {

constexpr int kGradThreads = 256;
constexpr int kGradRunTB = 16;  // consecutive samples per thread group in [T, B]

// Four neighbouring threads share a (channel, run of TT consecutive samples)
// and each owns four consecutive taps, so every row store of a wavefront is
// one contiguous 16-byte piece per thread.  A thread loads the TT + 3 signal
// values its taps need once.  Taps k = k0 + j, j < K <= 17, of
// out[e*K + j] = sign * ybar[e] * s[n - k] (s[-i] = hist[i-1] for i <= nh,
// else 0).  [T, B] takes TT = 4 (neighbouring thread groups are neighbouring
// channels, whose rows of one time are contiguous); [B, T] takes TT = 1
// (neighbouring samples of one channel).
// G = (K + 3) / 4 threads per row; the launch keeps B * runs * G below 2^31
// so the index arithmetic is 32-bit.
template <int TT, int G>
__global__ void __launch_bounds__(kGradThreads)
k_tv_coef_grads(Dims d, const float *__restrict__ ybar, const float *__restrict__ s,
                const float *__restrict__ hist, int nh, int k0, int K, float sign,
                float *__restrict__ out, int vec)
{
    const uint32_t runs = (uint32_t)((d.T + TT - 1) / TT);
    const uint32_t g = blockIdx.x * kGradThreads + threadIdx.x;
    const uint32_t r = g / G;
    if (r >= (uint32_t)d.B * runs)
        return;
    const int q = (int)(g - r * G);
    const bool tb = d.layout == FILT_LAYOUT_TB;
    const uint32_t B32 = (uint32_t)d.B;
    const int64_t b = tb ? r % B32 : r / runs;
    const int64_t t0 = (int64_t)(tb ? r / B32 : r % runs) * TT;
    const int64_t step = tb ? d.B : 1;
    const int64_t e0 = tb ? t0 * d.B + b : b * d.T + t0;
    const int kq = k0 + 4 * q;  // first tap of this thread
    // w[v] = s[t0 - kq - 3 + v]
    float w[TT + 3];
#pragma unroll
    for (int v = 0; v < TT + 3; ++v) {
        const int64_t t = t0 - kq - 3 + v;
        float x = 0.f;
        if (t >= 0) {
            if (t < d.T)
                x = s[e0 + (t - t0) * step];
        } else if (hist != nullptr && -t <= nh) {
            x = hist[b * nh + (-t - 1)];
        }
        w[v] = x;
    }
#pragma unroll
    for (int u = 0; u < TT; ++u) {
        if (t0 + u >= d.T)
            break;
        const int64_t e = e0 + u * step;
        const float v = sign * ybar[e];
        float rr[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
            rr[jj] = (4 * q + jj < K) ? v * w[u - jj + 3] : 0.f;
        float *o = out + e * K + 4 * q;
        // the gradient rows are written once and not read again here:
        // non-temporal stores stream them past the caches
        if (vec) {
            using f4 = float __attribute__((ext_vector_type(4)));
            const f4 v4 = {rr[0], rr[1], rr[2], rr[3]};
            __builtin_nontemporal_store(v4, reinterpret_cast<f4 *>(o));
        } else {
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
                if (4 * q + jj < K)
                    __builtin_nontemporal_store(rr[jj], o + jj);
        }
    }
}

// Frame-held coefficients: the gradient of a frame's row is the sum of the
// per-sample products over the frame's samples (Sec. 3.1 Eqs. 8-9 through
// the frame hold, by the chain rule):
//   out[row(b, f)][j] = sign * sum_{t in frame f} ybar[t] s[t - k0 - j],
// s[-i] = hist[b][i-1] for i <= nh, else 0.  FP64 sums.

// Value of signal s at (b, t), from the history before time 0.
template <typename io_t>
__device__ __forceinline__ double sig_hist(const Dims &d, const io_t *s, const io_t *hist,
                                           int nh, int64_t b, int64_t t)
{
    if (t >= 0)
        return (double)s[sig_at(d, b, t)];
    return (hist != nullptr && -t <= nh) ? (double)hist[b * nh + (-t - 1)] : 0.0;
}

// [B, T]: one wavefront (workgroup) per (channel, 64 consecutive frames).
template <typename io_t>
__global__ void __launch_bounds__(64)
k_frame_grads_bt(Dims d, const io_t *__restrict__ ybar, const io_t *__restrict__ s,
                 const io_t *__restrict__ hist, int nh, int k0, int K, double sign,
                 io_t *__restrict__ out)
{
    __shared__ io_t lds[kFrameLds];
    const int64_t nfb = (d.F + 63) / 64;
    const int64_t b = blockIdx.x / nfb, f0 = (blockIdx.x % nfb) * 64;
    frame_sums_wave(ybar + b * d.T, s + b * d.T, hist != nullptr ? hist + b * nh : nullptr, nh,
                    k0, K, sign, d.T, d.hop, f0, (int)min<int64_t>(64, d.F - f0),
                    out + b * d.F * K, lds, (int)threadIdx.x);
}

// [T, B]: one lane per (channel, frame, group of four taps), neighbouring
// lanes neighbouring channels (every load of a wavefront is one contiguous
// run).  The lane walks its frame with the four signal values its taps read
// in a shift register: two loads and four FMAs per sample, the loads of 16
// samples issued together.
template <typename io_t>
__global__ void __launch_bounds__(kGradThreads)
k_frame_grads_tb(Dims d, const io_t *__restrict__ ybar, const io_t *__restrict__ s,
                 const io_t *__restrict__ hist, int nh, int k0, int K, double sign,
                 io_t *__restrict__ out)
{
    const int G = (K + 3) / 4;
    const int64_t g = (int64_t)blockIdx.x * kGradThreads + threadIdx.x;
    if (g >= d.B * d.F * G)
        return;
    const int64_t b = g % d.B, rest = g / d.B;
    const int q = (int)(rest % G);
    const int64_t f = rest / G;
    const int64_t t0 = f * d.hop, t1 = min(t0 + d.hop, d.T);
    const int kq = k0 + 4 * q;  // first tap of this lane
    double acc[4], w[4];        // w[i] = s(t - kq - i) for the step t about to run
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        acc[i] = 0.0;
        w[i] = sig_hist(d, s, hist, nh, b, t0 - kq - i);
    }
    constexpr int P = 16;
    for (int64_t tb = t0; tb < t1; tb += P) {
        io_t yv[P], nv[P];
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const int64_t t = tb + r;
            const int64_t u = t + 1 - kq;  // enters the register after step t
            yv[r] = t < t1 ? ybar[t * d.B + b] : io_t(0);
            nv[r] = (t + 1 < t1) ? (io_t)sig_hist(d, s, hist, nh, b, u) : io_t(0);
        }
#pragma unroll
        for (int r = 0; r < P; ++r) {
            const double yb = (double)yv[r];  // zero past the frame
#pragma unroll
            for (int i = 0; i < 4; ++i)
                acc[i] = __builtin_fma(yb, w[i], acc[i]);
            w[3] = w[2];
            w[2] = w[1];
            w[1] = w[0];
            w[0] = (double)nv[r];
        }
    }
    io_t *o = out + row_at(d, b, t0, K) + 4 * q;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (4 * q + i < K)
            o[i] = (io_t)(sign * acc[i]);
}

}  // namespace

template <typename io_t>
filt_status frame_coef_grads_run(const Dims &d, const io_t *ybar, const io_t *x,
                                 const io_t *xi, const io_t *y, const io_t *yi, io_t *ga,
                                 io_t *gb, hipStream_t st)
{
    if (d.B * d.F == 0)
        return FILT_OK;
    auto launch = [&](const io_t *sig, const io_t *hist, int nh, int k0, int K, double sign,
                      io_t *o) {
        if (d.layout == FILT_LAYOUT_BT) {
            FILT_LAUNCH("frame_coef_grads", k_frame_grads_bt<io_t>,
                        dim3((unsigned)(d.B * ((d.F + 63) / 64))), dim3(64), 0, st, d, ybar, sig,
                        hist, nh, k0, K, sign, o);
        } else {
            const int64_t threads = d.B * d.F * ((K + 3) / 4);
            FILT_LAUNCH("frame_coef_grads", k_frame_grads_tb<io_t>,
                        dim3((unsigned)((threads + kGradThreads - 1) / kGradThreads)),
                        dim3(kGradThreads), 0, st, d, ybar, sig, hist, nh, k0, K, sign, o);
        }
    };
    if (ga != nullptr && d.N > 0)
        launch(y, yi, d.N, 1, d.N, -1.0, ga);
    if (gb != nullptr)
        launch(x, xi, d.M, 0, d.M + 1, 1.0, gb);
    return check_launch("frame coefficient gradients");
}

template filt_status frame_coef_grads_run<float>(const Dims &, const float *,
                                                 const float *, const float *, const float *,
                                                 const float *, float *, float *, hipStream_t);
template filt_status frame_coef_grads_run<double>(const Dims &, const double *,
                                                  const double *, const double *, const double *,
                                                  const double *, double *, double *,
                                                  hipStream_t);

bool tv_coef_grads_fits(const Dims &d)
{
    return d.B * d.T * 5 < ((int64_t)1 << 31);
}

filt_status tv_coef_grads_run(const Dims &d, const float *ybar, const float *x, const float *xi,
                              const float *y, const float *yi, float *ga, float *gb,
                              hipStream_t st)
{
    const int64_t n = d.B * d.T;
    if (n == 0)
        return FILT_OK;
    auto launch = [&](const float *sig, const float *hist, int nh, int k0, int K, float sign,
                      float *out) {
        // whole float4 pieces: rows a multiple of 4 wide and 16-byte aligned
        const int vec = (K % 4 == 0) && ((uintptr_t)out % 16 == 0);
        const int G = (K + 3) / 4;
        const bool tb = d.layout == FILT_LAYOUT_TB;
        const int64_t threads = d.B * (tb ? (d.T + kGradRunTB - 1) / kGradRunTB : d.T) * G;
        const dim3 grid((unsigned)((threads + kGradThreads - 1) / kGradThreads));
#define GRAD_LAUNCH(TT, GG)                                                                        \
    FILT_LAUNCH("coef_grads", (k_tv_coef_grads<TT, GG>), grid, dim3(kGradThreads), 0, st, d, ybar, \
                sig, hist, nh, k0, K, sign, out, vec)
#define GRAD_G(TT)                                                                                 \
    switch (G) {                                                                                   \
    case 1: GRAD_LAUNCH(TT, 1); break;                                                             \
    case 2: GRAD_LAUNCH(TT, 2); break;                                                             \
    case 3: GRAD_LAUNCH(TT, 3); break;                                                             \
    case 4: GRAD_LAUNCH(TT, 4); break;                                                             \
    default: GRAD_LAUNCH(TT, 5); break;                                                            \
    }
        if (tb) {
            GRAD_G(kGradRunTB)
        } else {
            GRAD_G(1)
        }
#undef GRAD_G
#undef GRAD_LAUNCH
    };
    if (ga != nullptr && d.N > 0)
        launch(y, yi, d.N, 1, d.N, -1.f, ga);
    if (gb != nullptr)
        launch(x, xi, d.M, 0, d.M + 1, 1.f, gb);
    return check_launch("coefficient gradients");
}

// Time-invariant all-pole [B, T] problems whose adjoint ran as a staged
// apply: ga_k = -sum_t ybar[t] y[t-k] (Sec. 3.1 Eq. 9 summed over time; y
// before time 0 from yi).  One workgroup per (channel, block of samples):
// FP64 sums over its samples, a fixed tree in LDS per tap, partials
// part[(b*nblk + blk)*(N+1) + k] (slot N, the b_0 tap, zero) for the
// time-invariant reduction.
namespace {

template <int KW>
__global__ void __launch_bounds__(256)
k_lti_ga_partial(Dims d, int64_t nblk, int64_t blk, const float *__restrict__ ybar,
                 const float *__restrict__ y, const float *__restrict__ yi,
                 double *__restrict__ part)
{
    __shared__ double red[256];
    const int64_t b = blockIdx.x / nblk, k0 = blockIdx.x % nblk;
    const int64_t t0 = k0 * blk;
    const int64_t t1 = t0 + blk < d.T ? t0 + blk : d.T;
    const int N = d.N;
    const float *yb = ybar + b * d.T;
    const float *yy = y + b * d.T;
    double acc[KW];
#pragma unroll
    for (int k = 0; k < KW; ++k)
        acc[k] = 0.0;
    // consecutive threads take consecutive samples (coalesced loads); four
    // samples per thread in flight at a time
    constexpr int U = 4;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += (int64_t)U * blockDim.x) {
        float v[U], w[U][KW];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t tu = t + (int64_t)u * blockDim.x;
            const bool in = tu < t1;
            v[u] = in ? yb[tu] : 0.f;
#pragma unroll
            for (int k = 1; k <= KW; ++k) {
                float x = 0.f;
                if (in && k <= N) {
                    if (tu - k >= 0)
                        x = yy[tu - k];
                    else if (yi != nullptr)
                        x = yi[b * N + (k - tu - 1)];
                }
                w[u][k - 1] = x;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < KW; ++k)
                acc[k] += (double)v[u] * (double)w[u][k];
    }
    double *o = part + (b * nblk + k0) * (N + 1);
    for (int k = 0; k < N; ++k) {
        double a = 0.0;
#pragma unroll
        for (int kk = 0; kk < KW; ++kk)
            if (kk == k)
                a = acc[kk];
        red[threadIdx.x] = a;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w)
                red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0)
            o[k] = -red[0];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        o[N] = 0.0;
}

}  // namespace

filt_status lti_allpole_ga_run(const Dims &d, const float *ybar, const float *y,
                               const float *yi, float *ga, double *part, hipStream_t st)
{
    // blocks of 8192 samples, at most one per chunk (the partial buffer holds
    // one record per chunk)
    int64_t nblk = (d.T + 8191) / 8192;
    if (nblk > d.C)
        nblk = d.C;
    const int64_t blk = (d.T + nblk - 1) / nblk;
    // taps padded to a power of two (N <= 8 here): the missing taps read zero
#define GA_LAUNCH(KW)                                                                              \
    FILT_LAUNCH("lti_ga_partial", k_lti_ga_partial<KW>, dim3((unsigned)(d.B * nblk)), dim3(256),  \
                0, st, d, nblk, blk, ybar, y, yi, part)
    if (d.N <= 1)
        GA_LAUNCH(1);
    else if (d.N <= 2)
        GA_LAUNCH(2);
    else if (d.N <= 4)
        GA_LAUNCH(4);
    else if (d.N <= 8)
        GA_LAUNCH(8);
    else
        return fail(FILT_EUNSUPPORTED, "time-invariant ga pass: order %d above 8", d.N);
#undef GA_LAUNCH
    filt_status s = check_launch("time-invariant ga partials");
    if (s != FILT_OK)
        return s;
    Dims r = d;
    r.C = nblk;
    r.M = 0;
    return reduce_lti_run(r, part, ga, nullptr, false, st);
}

}  // namespace filt_detail
