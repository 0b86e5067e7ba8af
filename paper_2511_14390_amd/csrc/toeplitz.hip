// toeplitz.hip -- time-invariant filters on [B, T] signals: the chunked
// time-parallel scan with every chunk's zero-state solve done as a matrix
// product on the FP32 matrix cores.
//
// With coefficients fixed per channel, the output of a chunk of kTzL samples
// starting at t0 is linear in the chunk's input and in what precedes it
// (the chunked form of Sec. 3.2):
//
//   y[t0 + i] = sum_j h[i - j] x[t0 + j]              (T_L, lower-triangular Toeplitz)
//             + sum_m Px[i][m] x[t0 - m]               (input history, m = 1..M)
//             + sum_m Py[i][m] y[t0 - m]               (output history, m = 1..N)
//
// h is the impulse response of B(z)/A(z); Px, Py are the responses to unit
// histories.  All chunks of a channel share the matrix [Px | T_L | Py], so a
// channel's chunks are the columns of one GEMM.  The state entering chunk
// c + 1 (the last N outputs of chunk c) is S_{c+1} = Phi S_c + s_c with Phi
// the Py rows of those outputs (the companion power A^L) and s_c the same rows
// of the zero-state part; the carry of carry.h resolves it in FP64.
//
// The backward runs the adjoint (Sec. 3.1 Eq. 7): inside a chunk
// ybar = T_L(h_A)^T gy + Pyb W and gx = T_L(h)^T gy + Pgx W, where h_A is the
// impulse response of 1/A(z) and W = (ybar[t1], ..., ybar[t1 + K - 1]) the
// first K = max(N, M) adjoint values of the next chunk.  W is carried
// backwards through the chunks the same way.  The coefficient gradients are
// correlations of ybar with y and x (Eqs. 8-9), summed in FP32 over 16
// samples per thread and in FP64 beyond.
//
// Tiles: one workgroup = one channel x 64 consecutive chunks (a 64 x 64
// output tile, 4096 samples), four wavefronts of 16 chunks each.  The signal
// windows of the 64 chunks are staged in LDS, one padded row per chunk, so
// that the 16 lanes of an MFMA operand read 16 different bank groups.
#include "carry.h"

namespace filt_detail {

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kTzCols = 64;  // chunks per workgroup
constexpr int kTzThreads = 256;

// Row stride of a staged window of K floats: K / 4 odd puts the rows of 16
// consecutive chunks on 16 disjoint groups of four banks.
__host__ __device__ inline int tz_lp(int K)
{
    return ((K >> 2) & 1) ? K : K + 4;
}

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Per-channel matrices (FP64 arithmetic, stored FP32 for the GEMMs and FP64
// for the carry).  One workgroup per channel.
//   Af  [KPF][64]  forward [Px | T_L | Py], k-major (column k of the matrix
//                  is 64 consecutive floats, one per output row)
//   Ayb [KPB][64]  backward [T_L(h_A)^T | Pyb]
//   Agx [KPB][64]  backward [T_L(h)^T | Pgx]
//   phif [N][N]    S_{c+1} = phif S_c + s_c, S_c[q] = y[t0 - 1 - q]
//   phib [KW][KW]  W_c = phib W_{c+1} + sbar_c
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kTzThreads)
k_tz_prep(Dims d, const float *__restrict__ bc, const float *__restrict__ ac, int fwd,
          float *__restrict__ Af, float *__restrict__ Ayb, float *__restrict__ Agx,
          double *__restrict__ phif, double *__restrict__ phib)
{
    __shared__ double ca[kMaxD + 1], cb[kMaxD + 1];
    __shared__ double hA[kTzL], h[kTzL];
    __shared__ double pyb[kTzL][kMaxD + 1];
    const int N = d.N, M = d.M;
    const TzGeom g = tz_geom(N, M);
    const int64_t b = blockIdx.x;
    const int tid = threadIdx.x;
    if (tid <= kMaxD) {
        ca[tid] = tid == 0 ? 1.0 : (tid <= N ? (double)ac[b * N + tid - 1] : 0.0);
        cb[tid] = tid > M ? 0.0
                          : (d.has_b ? (double)bc[b * (M + 1) + tid] : (tid == 0 ? 1.0 : 0.0));
    }
    __syncthreads();
    if (tid == 0) {
        // impulse response of 1/A(z), history hist[k-1] = hA[n-k] in registers
        double ar[kMaxD], hist[kMaxD];
#pragma unroll
        for (int k = 0; k < kMaxD; ++k) {
            ar[k] = ca[k + 1];
            hist[k] = 0.0;
        }
        for (int n = 0; n < kTzL; ++n) {
            double v0 = n == 0 ? 1.0 : 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
#pragma unroll
            for (int k = 0; k < kMaxD; k += 4) {
                v0 -= ar[k] * hist[k];
                v1 -= ar[k + 1] * hist[k + 1];
                v2 -= ar[k + 2] * hist[k + 2];
                v3 -= ar[k + 3] * hist[k + 3];
            }
            const double v = (v0 + v1) + (v2 + v3);
#pragma unroll
            for (int k = kMaxD - 1; k > 0; --k)
                hist[k] = hist[k - 1];
            hist[0] = v;
            hA[n] = v;
        }
    }
    __syncthreads();
    if (tid < kTzL) {
        // impulse response of B(z)/A(z)
        double v = 0.0;
        for (int k = 0; k <= M && k <= tid; ++k)
            v += cb[k] * hA[tid - k];
        h[tid] = v;
    }
    if (!fwd) {
        // Pyb[i][w]: ybar[t0 + i] for a unit ybar[t1 + w] beyond the chunk.
        // That value drives the adjoint at position i' = 64 + w - k through
        // the term -a_k, which then spreads backwards by h_A.
        for (int e = tid; e < kTzL * g.KW; e += kTzThreads) {
            const int i = e / g.KW, w = e % g.KW;
            double v = 0.0;
            for (int k = w + 1; k <= N; ++k) {
                const int ip = kTzL + w - k;
                if (ip >= i)
                    v -= ca[k] * hA[ip - i];
            }
            pyb[i][w] = v;
        }
    }
    __syncthreads();
    // each thread keeps one output row i (the element loops step by a
    // multiple of 64) and the response values it needs in registers
    const int ri = tid & (kTzL - 1);
    double hr[kMaxD + 1];
#pragma unroll
    for (int n = 0; n <= kMaxD; ++n)
        hr[n] = ri - n >= 0 ? hA[ri - n >= 0 ? ri - n : 0] : 0.0;
    if (fwd) {
        float *A = Af + b * (int64_t)g.KPF * kTzL;
        for (int e = tid; e < g.KPF * kTzL; e += kTzThreads) {
            const int k = e / kTzL;  // uniform across a wavefront
            double v = 0.0;
            if (k < g.KH) {
                // unit x[t0 - m] enters through b_{n+m} at n = 0..M-m
                const int m = g.KH - k;
                if (m <= M)
#pragma unroll
                    for (int n = 0; n <= kMaxD; ++n)
                        if (n <= M - m)
                            v += cb[n + m <= kMaxD ? n + m : kMaxD] * hr[n];
            } else if (k < g.KH + kTzL) {
                const int j = k - g.KH;
                v = ri >= j ? h[ri - j] : 0.0;
            } else {
                // unit y[t0 - m] enters through -a_{n+m} at n = 0..N-m
                const int m = k - g.KH - kTzL + 1;
                if (m <= N)
#pragma unroll
                    for (int n = 0; n <= kMaxD; ++n)
                        if (n <= N - m)
                            v -= ca[n + m <= kMaxD ? n + m : kMaxD] * hr[n];
            }
            A[e] = (float)v;
        }
        // phif[q][m-1] = Py[63 - q][m]
        for (int e = tid; e < N * N; e += kTzThreads) {
            const int q = e / N, m = e % N + 1;
            const int i = kTzL - 1 - q;
            double v = 0.0;
            for (int n = 0; n <= N - m && n <= i; ++n)
                v -= ca[n + m] * hA[i - n];
            phif[b * N * N + e] = v;
        }
    } else {
        float *Y = Ayb + b * (int64_t)g.KPB * kTzL;
        float *X = Agx + b * (int64_t)g.KPB * kTzL;
        for (int e = tid; e < g.KPB * kTzL; e += kTzThreads) {
            const int k = e / kTzL, i = e % kTzL;
            double vy = 0.0, vx = 0.0;
            if (k < kTzL) {
                if (k >= i) {
                    vy = hA[k - i];
                    vx = h[k - i];
                }
            } else {
                const int w = k - kTzL;
                if (w < g.KW) {
                    vy = pyb[i][w];
                    // gx[t0 + i] = sum_q b_q ybar[t0 + i + q]
                    for (int q = 0; q <= M; ++q) {
                        const int ip = i + q;
                        if (ip < kTzL)
                            vx += cb[q] * pyb[ip][w];
                        else if (ip - kTzL == w)
                            vx += cb[q];
                    }
                }
            }
            Y[e] = (float)vy;
            X[e] = (float)vx;
        }
        for (int e = tid; e < g.KW * g.KW; e += kTzThreads)
            phib[b * g.KW * g.KW + e] = pyb[e / g.KW][e % g.KW];
    }
}

// Stage the windows of the tile's chunks: window col holds, at k in
// [0, KH + 64), the signal at t = t0(col) - KH + k; zero at t >= T; for t < 0
// hist[-t - 1] when -t <= nh (hist may be null).  Runs of four samples move
// as one float4 when the signal is 16-byte aligned there (vec).
__device__ __forceinline__ float tz_sample(const float *__restrict__ s, int64_t T,
                                           const float *__restrict__ hist, int nh, int64_t t)
{
    if (t >= 0)
        return t < T ? s[t] : 0.f;
    return (hist != nullptr && -t <= nh) ? hist[-t - 1] : 0.f;
}

__device__ __forceinline__ void tz_stage_signal(const float *__restrict__ s, int64_t T,
                                                const float *__restrict__ hist, int nh,
                                                int64_t c0, int KH, int lp, float *win, int vec)
{
    const int n4 = (KH + kTzL * kTzCols) / 4;  // KH is a multiple of 4
    const int64_t base = c0 * kTzL - KH;
    for (int p4 = threadIdx.x; p4 < n4; p4 += blockDim.x) {
        const int p = 4 * p4;
        const int64_t t = base + p;
        float4 v;
        if (vec && t >= 0 && t + 3 < T) {
            v = *reinterpret_cast<const float4 *>(s + t);
        } else {
            v.x = tz_sample(s, T, hist, nh, t);
            v.y = tz_sample(s, T, hist, nh, t + 1);
            v.z = tz_sample(s, T, hist, nh, t + 2);
            v.w = tz_sample(s, T, hist, nh, t + 3);
        }
        const int ca = p >> 6, ka = p & 63;
        if (ca < kTzCols)
            *reinterpret_cast<float4 *>(win + ca * lp + ka) = v;
        if (ka < KH && ca >= 1)
            *reinterpret_cast<float4 *>(win + (ca - 1) * lp + ka + kTzL) = v;
    }
}

// Stage the signal s[t], t in [c0*64 - 16, (c0 + 64)*64), as a flat array
// (lin[16 + n] = s[c0*64 + n]), history from hist.
__device__ __forceinline__ void tz_stage_linear(const float *__restrict__ s, int64_t T,
                                                const float *__restrict__ hist, int nh,
                                                int64_t c0, float *lin, int vec)
{
    const int n4 = (16 + kTzL * kTzCols) / 4;
    const int64_t base = c0 * kTzL - 16;
    for (int p4 = threadIdx.x; p4 < n4; p4 += blockDim.x) {
        const int64_t t = base + 4 * p4;
        float4 v;
        if (vec && t >= 0 && t + 3 < T) {
            v = *reinterpret_cast<const float4 *>(s + t);
        } else {
            v.x = tz_sample(s, T, hist, nh, t);
            v.y = tz_sample(s, T, hist, nh, t + 1);
            v.z = tz_sample(s, T, hist, nh, t + 2);
            v.w = tz_sample(s, T, hist, nh, t + 3);
        }
        *reinterpret_cast<float4 *>(lin + 4 * p4) = v;
    }
}

// Copy a channel's k-major matrix rows [k0, k1) into LDS (same layout).
__device__ __forceinline__ void tz_stage_matrix(const float *__restrict__ A, int k0, int k1,
                                                float *As)
{
    const float4 *src = (const float4 *)(A + k0 * kTzL);
    float4 *dst = (float4 *)(As + k0 * kTzL);
    const int n = (k1 - k0) * kTzL / 4;
    for (int e = threadIdx.x; e < n; e += blockDim.x)
        dst[e] = src[e];
}

// Store a [64 chunks][64] tile from LDS (row stride 68) to a [B, T] signal.
__device__ __forceinline__ void tz_store_tile(const float *out, float *__restrict__ dst,
                                              int64_t T, int64_t C, int64_t c0, int vec)
{
    for (int q = threadIdx.x; q < kTzCols * kTzL / 4; q += blockDim.x) {
        const int col = q >> 4, i4 = (q & 15) * 4;
        const int64_t c = c0 + col;
        if (c >= C)
            continue;
        const int64_t t = c * kTzL + i4;
        const float4 v = *(const float4 *)(out + col * 68 + i4);
        if (vec && t + 3 < T) {
            *(float4 *)(dst + t) = v;
        } else {
            if (t < T)
                dst[t] = v.x;
            if (t + 1 < T)
                dst[t + 1] = v.y;
            if (t + 2 < T)
                dst[t + 2] = v.z;
            if (t + 3 < T)
                dst[t + 3] = v.w;
        }
    }
}

// ---------------------------------------------------------------------------
// Forward.  mode 0: chunk summaries s_c (rows 48..63 of the zero-state part)
// for chunks 0..C-2 into summ[B][C][N]; mode 1: the outputs, with the states
// S_c from states[B][C][N] (c >= 1) and yi (c = 0).
// LDS: win [64][lp] then A [KPF][64] floats.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kTzThreads)
k_tz_fwd(Dims d, int mode, const float *__restrict__ x, const float *__restrict__ xi,
         const float *__restrict__ yi, const float *__restrict__ Af,
         const double *__restrict__ states, double *__restrict__ summ, float *__restrict__ y,
         int vec, int vin)
{
    extern __shared__ float tz_lds[];
    const int N = d.N, M = d.M;
    const TzGeom g = tz_geom(N, M);
    const int lp = tz_lp(g.KPF);
    float *win = tz_lds;
    float *As = tz_lds + kTzCols * lp;
    const int64_t nwg = (d.C + kTzCols - 1) / kTzCols;
    const int64_t b = blockIdx.x / nwg;
    const int64_t c0 = (blockIdx.x % nwg) * kTzCols;
    const int tid = threadIdx.x;
    const float *A = Af + b * (int64_t)g.KPF * kTzL;
    tz_stage_matrix(A, 0, mode ? g.KPF : g.KH + kTzL, As);
    tz_stage_signal(x + b * d.T, d.T, xi != nullptr ? xi + b * M : nullptr, M, c0, g.KH, lp, win,
                    vin);
    if (mode) {
        for (int e = tid; e < kTzCols * g.KS; e += kTzThreads) {
            const int col = e / g.KS, q = e % g.KS;
            const int64_t c = c0 + col;
            float v = 0.f;
            if (q < N && c < d.C) {
                if (c == 0)
                    v = yi != nullptr ? yi[b * N + q] : 0.f;
                else
                    v = (float)states[(b * d.C + c) * N + q];
            }
            win[col * lp + g.KH + kTzL + q] = v;
        }
    }
    __syncthreads();
    const int w = tid >> 6, l = tid & 63, gq = l >> 4, cl = l & 15;
    const int col = 16 * w + cl;
    const float *bw = win + col * lp + gq;
    const float *aw = As + gq * kTzL + cl;
    if (mode == 0) {
        // rows 48..63 only: the last N outputs of each chunk
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        const int ks = (g.KH + kTzL) / 4;
        for (int s = 0; s < ks; ++s)
            acc = mfma4(aw[4 * s * kTzL + 48], bw[4 * s], acc);
        const int64_t c = c0 + col;
        if (c <= d.C - 2) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = 15 - 4 * gq - r;  // row 63 - m
                if (m < N)
                    summ[(b * d.C + c) * N + m] = (double)acc[r];
            }
        }
        return;
    }
    floatx4 acc[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
        acc[rb] = floatx4{0.f, 0.f, 0.f, 0.f};
    // x part: row block rb needs columns j <= 16 rb + 15 of T_L
    const int kx = g.KH / 4 + 16;
    for (int s = 0; s < kx; ++s) {
        const float bv = bw[4 * s];
        const float *ar = aw + 4 * s * kTzL;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
            if (4 * s < g.KH + 16 * rb + 16)
                acc[rb] = mfma4(ar[16 * rb], bv, acc[rb]);
    }
    for (int s = (g.KH + kTzL) / 4; s < g.KPF / 4; ++s) {
        const float bv = bw[4 * s];
        const float *ar = aw + 4 * s * kTzL;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
            acc[rb] = mfma4(ar[16 * rb], bv, acc[rb]);
    }
    __syncthreads();
    float *out = win;  // [64][68]
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
        *(floatx4 *)(out + col * 68 + 16 * rb + 4 * gq) = acc[rb];
    __syncthreads();
    tz_store_tile(out, y + b * d.T, d.T, d.C, c0, vec);
}

// ---------------------------------------------------------------------------
// Backward.  mode 0: summaries sbar_c (rows 0..KW-1 of the zero-future
// adjoint) for chunks 1..C-1 into summ[B][C][KW]; mode 1: gx, the per-tile
// partial sums of the coefficient gradients (part[B][nwg][N + M + 1], ga
// taps first) and, from the tile holding t = 0, gxi and gyi.  W_{c+1} comes
// from states[B][C][KW] (zero for the last chunk).
// LDS: win [64][lp], Ayb [KPB][64], Agx [KPB][64] floats.
// ---------------------------------------------------------------------------
struct TzBwdOut {
    float *gx, *gxi, *gyi;
    double *part;
    int want_ab;  // ga or gb requested
    int want_ga, want_gb;
};

__global__ void __launch_bounds__(kTzThreads)
k_tz_bwd(Dims d, int mode, const float *__restrict__ gy, const float *__restrict__ x,
         const float *__restrict__ xi, const float *__restrict__ y, const float *__restrict__ yi,
         const float *__restrict__ bc, const float *__restrict__ ac, const float *__restrict__ Ayb,
         const float *__restrict__ Agx, const double *__restrict__ states,
         double *__restrict__ summ, TzBwdOut o, int vec, int vin)
{
    extern __shared__ float tz_lds[];
    __shared__ double red[4][2 * kMaxD + 2];
    const int N = d.N, M = d.M;
    const TzGeom g = tz_geom(N, M);
    const int lp = tz_lp(g.KPB);
    float *win = tz_lds;
    float *Ys = tz_lds + kTzCols * lp;
    float *Xs = Ys + g.KPB * kTzL;
    const int64_t nwg = (d.C + kTzCols - 1) / kTzCols;
    const int64_t b = blockIdx.x / nwg;
    const int64_t cw = blockIdx.x % nwg;
    const int64_t c0 = cw * kTzCols;
    const int tid = threadIdx.x;
    const bool want_y = mode == 0 || o.want_ab || o.gxi != nullptr || o.gyi != nullptr;
    const bool want_x = mode == 1 && o.gx != nullptr;
    if (want_y)
        tz_stage_matrix(Ayb + b * (int64_t)g.KPB * kTzL, 0, mode ? g.KPB : kTzL, Ys);
    if (want_x)
        tz_stage_matrix(Agx + b * (int64_t)g.KPB * kTzL, 0, g.KPB, Xs);
    tz_stage_signal(gy + b * d.T, d.T, nullptr, 0, c0, 0, lp, win, vin);
    if (mode) {
        for (int e = tid; e < kTzCols * g.KWp; e += kTzThreads) {
            const int col = e / g.KWp, q = e % g.KWp;
            const int64_t c = c0 + col;
            float v = 0.f;
            if (q < g.KW && c < d.C - 1)
                v = (float)states[(b * d.C + c) * g.KW + q];
            win[col * lp + kTzL + q] = v;
        }
    }
    __syncthreads();
    const int w = tid >> 6, l = tid & 63, gq = l >> 4, cl = l & 15;
    const int col = 16 * w + cl;
    const float *bw = win + col * lp + gq;
    if (mode == 0) {
        // rows 0..15: the first KW adjoint values of each chunk
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        const float *aw = Ys + gq * kTzL + cl;
        for (int s = 0; s < kTzL / 4; ++s)
            acc = mfma4(aw[4 * s * kTzL], bw[4 * s], acc);
        const int64_t c = c0 + col;
        if (c >= 1 && c < d.C) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = 4 * gq + r;
                if (i < g.KW)
                    summ[(b * d.C + c) * g.KW + i] = (double)acc[r];
            }
        }
        return;
    }
    // ybar and gx tiles; row block rb needs columns j >= 16 rb of the
    // upper-triangular part
    floatx4 ay[4], ax[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        ay[rb] = floatx4{0.f, 0.f, 0.f, 0.f};
        ax[rb] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    const float *awy = Ys + gq * kTzL + cl;
    const float *awx = Xs + gq * kTzL + cl;
    for (int s = 0; s < g.KPB / 4; ++s) {
        const float bv = bw[4 * s];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
            if (s >= kTzL / 4 || 4 * s + 3 >= 16 * rb) {
                if (want_y)
                    ay[rb] = mfma4(awy[4 * s * kTzL + 16 * rb], bv, ay[rb]);
                if (want_x)
                    ax[rb] = mfma4(awx[4 * s * kTzL + 16 * rb], bv, ax[rb]);
            }
        }
    }
    __syncthreads();
    // gx tile through win, ybar tile through the Ayb region
    float *outx = win;
    float *outy = Ys;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
        if (want_x)
            *(floatx4 *)(outx + col * 68 + 16 * rb + 4 * gq) = ax[rb];
        if (want_y)
            *(floatx4 *)(outy + col * 68 + 16 * rb + 4 * gq) = ay[rb];
    }
    __syncthreads();
    if (want_x)
        tz_store_tile(outx, o.gx + b * d.T, d.T, d.C, c0, vec);
    if (o.want_ab) {
        // the signals are staged flat in LDS (the Agx region is free now):
        // lin[16 + n] = y[c0*64 + n]; thread tid takes samples n = tid + 256 u
        // of the tile, so neighbouring lanes read neighbouring words
        float *lin = Xs;
        float ga_acc[kMaxD], gb_acc[kMaxD + 1];
#pragma unroll
        for (int k = 0; k < kMaxD; ++k)
            ga_acc[k] = 0.f;
#pragma unroll
        for (int k = 0; k <= kMaxD; ++k)
            gb_acc[k] = 0.f;
        if (o.want_ga) {
            tz_stage_linear(y + b * d.T, d.T, yi != nullptr ? yi + b * N : nullptr, N, c0, lin,
                            vin);
            __syncthreads();
            for (int u = 0; u < kTzL * kTzCols / kTzThreads; ++u) {
                const int n = tid + kTzThreads * u;
                const float v = outy[(n >> 6) * 68 + (n & 63)];
#pragma unroll
                for (int k = 1; k <= kMaxD; ++k)
                    if (k <= N)
                        ga_acc[k - 1] -= v * lin[16 + n - k];
            }
            __syncthreads();
        }
        if (o.want_gb) {
            tz_stage_linear(x + b * d.T, d.T, xi != nullptr ? xi + b * M : nullptr, M, c0, lin,
                            vin);
            __syncthreads();
            for (int u = 0; u < kTzL * kTzCols / kTzThreads; ++u) {
                const int n = tid + kTzThreads * u;
                const float v = outy[(n >> 6) * 68 + (n & 63)];
#pragma unroll
                for (int k = 0; k <= kMaxD; ++k)
                    if (k <= M)
                        gb_acc[k] += v * lin[16 + n - k];
            }
        }
        // workgroup sums in FP64: wavefront butterfly, then across waves
        const int K = N + M + 1;
#pragma unroll
        for (int k = 0; k < kMaxD; ++k) {
            if (k < N && o.want_ga) {
                double v = (double)ga_acc[k];
                for (int off = 32; off > 0; off >>= 1)
                    v += __shfl_xor(v, off);
                if (l == 0)
                    red[w][k] = v;
            }
        }
#pragma unroll
        for (int k = 0; k <= kMaxD; ++k) {
            if (k <= M && o.want_gb) {
                double v = (double)gb_acc[k];
                for (int off = 32; off > 0; off >>= 1)
                    v += __shfl_xor(v, off);
                if (l == 0)
                    red[w][N + k] = v;
            }
        }
        __syncthreads();
        if (tid < K)
            o.part[(b * nwg + cw) * K + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    }
    if (c0 == 0 && tid < kMaxD) {
        // gyi[j-1] = -sum_{k=j..N} a_k ybar[k-j]; gxi[j-1] = sum_{k=j..M} b_k ybar[k-j]
        const int j = tid + 1;
        if (o.gyi != nullptr && j <= N) {
            double v = 0.0;
            for (int k = j; k <= N; ++k)
                v -= (double)ac[b * N + k - 1] * (double)outy[k - j];
            o.gyi[b * N + j - 1] = (float)v;
        }
        if (o.gxi != nullptr && j <= M) {
            double v = 0.0;
            for (int k = j; k <= M; ++k)
                v += (double)bc[b * (M + 1) + k] * (double)outy[k - j];
            o.gxi[b * M + j - 1] = (float)v;
        }
    }
}

// Dynamic LDS bytes of the two tile kernels.
size_t tz_fwd_lds(const Dims &d)
{
    const TzGeom g = tz_geom(d.N, d.M);
    return ((size_t)kTzCols * tz_lp(g.KPF) + (size_t)g.KPF * kTzL) * sizeof(float);
}

size_t tz_bwd_lds(const Dims &d)
{
    const TzGeom g = tz_geom(d.N, d.M);
    return ((size_t)kTzCols * tz_lp(g.KPB) + 2 * (size_t)g.KPB * kTzL) * sizeof(float);
}

}  // namespace

TzPlan tz_plan(const Dims &d)
{
    const TzGeom g = tz_geom(d.N, d.M);
    TzPlan p{};
    p.KW = g.KW;
    p.KPF = g.KPF;
    p.KPB = g.KPB;
    p.nwg = (d.C + kTzCols - 1) / kTzCols;
    return p;
}

filt_status tz_forward(const Dims &d, const float *x, const float *bc, const float *ac,
                       const float *xi, const float *yi, float *y, const WsPlan &w, char *ws,
                       hipStream_t st)
{
    const TzPlan tp = tz_plan(d);
    float *Af = (float *)(ws + w.tz_af);
    double *phif = (double *)(ws + w.phi);
    double *summ = (double *)(ws + w.summ);
    double *states = (double *)(ws + w.states);
    const unsigned grid = (unsigned)(d.B * tp.nwg);
    const int vec = (d.T % 4 == 0) && ((uintptr_t)y % 16 == 0);
    const int vin = (d.T % 4 == 0) && ((uintptr_t)x % 16 == 0);
    FILT_LAUNCH("tz_prep", k_tz_prep, dim3((unsigned)d.B), dim3(kTzThreads), 0, st, d, bc, ac, 1,
                Af, (float *)nullptr, (float *)nullptr, phif, (double *)nullptr);
    if (d.C > 1) {
        FILT_LAUNCH("tz_fwd_summary", k_tz_fwd, dim3(grid), dim3(kTzThreads), tz_fwd_lds(d), st,
                    d, 0, x, xi, yi, (const float *)Af, (const double *)states, summ,
                    (float *)nullptr, vec, vin);
        CarryArgs a{};
        a.summ = summ;
        a.phi = phif;
        a.SS = d.N;
        a.soff = 0;
        a.D = d.N;
        a.R = 0;
        a.bwd = 0;
        a.agg = (double *)(ws + w.agg);
        a.bstart = (double *)(ws + w.bstart);
        a.states = states;
        const filt_status s = carry_run(d, a, yi, false, st);
        if (s != FILT_OK)
            return s;
    }
    FILT_LAUNCH("tz_fwd_apply", k_tz_fwd, dim3(grid), dim3(kTzThreads), tz_fwd_lds(d), st, d, 1,
                x, xi, yi, (const float *)Af, (const double *)states, (double *)nullptr, y, vec,
                vin);
    return check_launch("time-invariant forward");
}

filt_status tz_backward(const Dims &d, const float *gy, const float *x, const float *y,
                        const float *bc, const float *ac, const float *xi, const float *yi,
                        float *gx, float *gb, float *ga, float *gxi, float *gyi, const WsPlan &w,
                        char *ws, hipStream_t st)
{
    const TzPlan tp = tz_plan(d);
    float *Ayb = (float *)(ws + w.tz_ayb);
    float *Agx = (float *)(ws + w.tz_agx);
    double *phib = (double *)(ws + w.tz_phib);
    double *summ = (double *)(ws + w.summ);
    double *states = (double *)(ws + w.states);
    double *part = (double *)(ws + w.part);
    const unsigned grid = (unsigned)(d.B * tp.nwg);
    const int vec = (d.T % 4 == 0) && (gx == nullptr || (uintptr_t)gx % 16 == 0);
    auto al = [](const float *p) { return p == nullptr || (uintptr_t)p % 16 == 0; };
    const int vin = (d.T % 4 == 0) && al(gy) && al(y) && al(x);
    FILT_LAUNCH("tz_prep", k_tz_prep, dim3((unsigned)d.B), dim3(kTzThreads), 0, st, d, bc, ac, 0,
                (float *)nullptr, Ayb, Agx, (double *)nullptr, phib);
    TzBwdOut o{};
    o.gx = gx;
    o.gxi = gxi;
    o.gyi = gyi;
    o.part = part;
    o.want_ga = ga != nullptr;
    o.want_gb = gb != nullptr;
    o.want_ab = o.want_ga || o.want_gb;
    if (d.C > 1) {
        FILT_LAUNCH("tz_bwd_summary", k_tz_bwd, dim3(grid), dim3(kTzThreads), tz_bwd_lds(d), st,
                    d, 0, gy, x, xi, y, yi, bc, ac, (const float *)Ayb, (const float *)Agx,
                    (const double *)states, summ, o, vec, vin);
        CarryArgs a{};
        a.summ = summ;
        a.phi = phib;
        a.SS = tp.KW;
        a.soff = 0;
        a.D = tp.KW;
        a.R = 0;
        a.bwd = 1;
        a.agg = (double *)(ws + w.agg);
        a.bstart = (double *)(ws + w.bstart);
        a.states = states;
        const filt_status s = carry_run(d, a, nullptr, false, st);
        if (s != FILT_OK)
            return s;
    }
    FILT_LAUNCH("tz_bwd_apply", k_tz_bwd, dim3(grid), dim3(kTzThreads), tz_bwd_lds(d), st, d, 1,
                gy, x, xi, y, yi, bc, ac, (const float *)Ayb, (const float *)Agx,
                (const double *)states, (double *)nullptr, o, vec, vin);
    filt_status s = check_launch("time-invariant backward");
    if (s != FILT_OK || !o.want_ab)
        return s;
    Dims dr = d;
    dr.C = tp.nwg;
    return reduce_lti_run(dr, part, ga, gb, false, st);
}

}  // namespace filt_detail
