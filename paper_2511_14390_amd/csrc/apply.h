// apply.h -- phase 3 of the chunked scan and the per-direction driver.
//
// Every (channel, chunk) reruns its chunk from the exact entering state that
// the carry produced and writes the outputs: the forward writes y; the
// backward runs the adjoint in transposed form (the backward of a direct
// form is a transposed direct form run in reverse time, Sec. 3.1 after
// Eq. 9) and fuses the gradient products of Eqs. 6, 8 and 9: gx, the
// per-sample (or, for time-invariant filters, per-chunk partial sums of the)
// coefficient gradients, and the initial-condition gradients from the state
// left after time 0.
#pragma once

#include "common.h"
#include "stream.h"

namespace filt_detail {

// ---------------------------------------------------------------- forward

// KT bounds the taps the loops visit (a_1..a_KT, b_0..b_KT): the bucket width
// by default, max(N, M) for narrower time-invariant filters (lti_tap_bound).
template <int W, bool TV, bool FIR, bool AV, typename io_t, typename acc_t, int KT = W>
__device__ __forceinline__ void fwd_apply_item(const Dims &d, const io_t *__restrict__ x,
                                               const io_t *__restrict__ xi,
                                               const io_t *__restrict__ bc,
                                               const io_t *__restrict__ ac,
                                               const io_t *__restrict__ yi,
                                               const double *__restrict__ hin,
                                               io_t *__restrict__ y, int64_t b, int64_t c)
{
    constexpr int m = W - 1;
    const int64_t t0 = c * d.L;
    acc_t la[W + 1], lb[W];
    if constexpr (!TV)
        ld_row_lti<W, FIR>(d, bc, ac, b, la, lb);
    const Cursor<io_t> xc = cursor(d, x, b, t0, 1);
    const Cursor<io_t> acur = row_cursor(d, ac, b, t0, d.N);
    const Cursor<io_t> bcur = row_cursor(d, bc, b, t0, d.has_b ? d.M + 1 : 0);
    io_t *yrow = y + sig_at(d, b, t0);
    const int64_t ystride = d.layout == FILT_LAYOUT_TB ? d.B : 1;
    // y history: hy[t mod W] = y[t]; x history likewise
    acc_t hy[W], hx[W];
#pragma unroll
    for (int q = 0; q < W; ++q) {
        hy[q] = acc_t(0);
        hx[q] = acc_t(0);
    }
#pragma unroll
    for (int i = 0; i < W; ++i) {
        if (i < d.N) {
            acc_t v;
            if (c == 0)
                v = (yi != nullptr) ? (acc_t)yi[b * d.N + i] : acc_t(0);
            else
                v = (acc_t)hin[(b * d.C + c) * d.N + i];
            hy[(-(i + 1)) & m] = v;
        }
    }
    if constexpr (FIR) {
#pragma unroll
        for (int k = 1; k < W; ++k)
            hx[(-k) & m] = ld_x<io_t, acc_t>(d, x, xi, b, t0 - k);
    }
    const int64_t tend = t0 + d.L;
    using PF = Prefetch<W, TV, FIR, io_t>;
    auto fetch = [&](int64_t t, PF &p) {
        if constexpr (TV)
            ld_raw<W, FIR, AV>(d, acur.at(t0, t), bcur.at(t0, t), p.ra, p.rb);
        p.s0 = *xc.at(t0, t);  // outputs past T are not written
    };
    // circular prefetch: step t's data is fetched P steps ahead into buf[t % P];
    // the loop is unrolled by U = max(W, P) so every index is static
    constexpr int P = kApplyPrefetch;
    constexpr int U = W > P ? W : P;
    PF buf[P];
#pragma unroll
    for (int q = 0; q < P; ++q)
        fetch(t0 + q, buf[q]);
    for (int64_t tb = t0; tb < tend; tb += U) {
#pragma unroll
        for (int s = 0; s < U; ++s) {
            const int64_t t = tb + s;
            const PF cur = buf[s % P];
            fetch(t + P, buf[s % P]);
            acc_t ca[W + 1], cb[W];
            if constexpr (TV) {
                cvt_row<W, FIR>(cur.ra, cur.rb, ca, cb);
            } else {
#pragma unroll
                for (int k = 0; k <= W; ++k)
                    ca[k] = la[k];
#pragma unroll
                for (int k = 0; k < W; ++k)
                    cb[k] = lb[k];
            }
            hx[s & m] = (acc_t)cur.s0;
            acc_t p0 = acc_t(0), p1 = acc_t(0);
            if constexpr (FIR) {
#pragma unroll
                for (int k = W - 1; k >= 0; --k) {
                    if (k > KT)
                        continue;
                    if (k & 1)
                        p1 += cb[k] * hx[(s - k) & m];
                    else
                        p0 += cb[k] * hx[(s - k) & m];
                }
            } else {
                p0 = cb[0] * hx[s & m];
            }
            // oldest taps first; the newest output is the last dependency
#pragma unroll
            for (int k = W; k >= 2; --k) {
                if (k > KT)
                    continue;
                if (k & 1)
                    p1 -= ca[k] * hy[(s - k) & m];
                else
                    p0 -= ca[k] * hy[(s - k) & m];
            }
            const acc_t v = (p0 + p1) - ca[1] * hy[(s - 1) & m];
            hy[s & m] = v;
            if (t < d.T)
                yrow[(t - t0) * ystride] = (io_t)v;
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <int W, bool TV, bool FIR, bool AV, typename io_t, typename acc_t, int KT = W>
__global__ void __launch_bounds__(kThreads)
k_fwd_apply(Dims d, const io_t *__restrict__ x, const io_t *__restrict__ xi,
            const io_t *__restrict__ bc, const io_t *__restrict__ ac,
            const io_t *__restrict__ yi, const double *__restrict__ hin, io_t *__restrict__ y)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= d.B * d.C)
        return;
    int64_t b, c, jj;
    decode(d, idx, d.C, b, c, jj);
    fwd_apply_item<W, TV, FIR, AV, io_t, acc_t, KT>(d, x, xi, bc, ac, yi, hin, y, b, c);
}

// ---------------------------------------------------------------- backward

// gin[(b*C + c)*(N+M)] holds the (s, r) state entering chunk c from the
// future (zero for the last chunk).  Adjoint state slots as in the summary:
// before processing t, s_k is in ss[(k - t) mod W] and r_k in rs[(k - t) mod W].
// Per step: ybar = gy[t] + s_1, gx[t] = b_0 ybar + r_1, then the scatter
// updates; GB / GA also form gb_k[t] = ybar x[t-k] and ga_k[t] = -ybar y[t-k]
// from windows wx[t mod W] = x[t], wy[t mod W] = y[t] that slide down in time.
// Time-invariant filters write per-(b, c) FP64 partial sums to
// part[(b*C + c)*(N+M+1)] = (ga_1..ga_N, gb_0..gb_M).  Chunk 0 writes gyi / gxi.
template <int W, bool TV, bool FIR, bool GA, bool GB, bool AV, typename io_t, typename acc_t,
          int KT = W>
__device__ __forceinline__ void bwd_apply_item(
    const Dims &d, const io_t *__restrict__ gy, const io_t *__restrict__ x,
    const io_t *__restrict__ xi, const io_t *__restrict__ y, const io_t *__restrict__ yi,
    const io_t *__restrict__ bc, const io_t *__restrict__ ac, const double *__restrict__ gin,
    io_t *__restrict__ gx, io_t *__restrict__ gb, io_t *__restrict__ ga, io_t *__restrict__ gxi,
    io_t *__restrict__ gyi, double *__restrict__ part, io_t *__restrict__ ybo, int64_t b,
    int64_t c)
{
    constexpr int m = W - 1;
    const int64_t t0 = c * d.L;
    const int N = d.N, M = d.M;
    acc_t la[W + 1], lb[W];
    if constexpr (!TV)
        ld_row_lti<W, FIR>(d, bc, ac, b, la, lb);
    const Cursor<io_t> gc = cursor(d, gy, b, t0, 1);
    const Cursor<io_t> acur = row_cursor(d, ac, b, t0, d.N);
    const Cursor<io_t> bcur = row_cursor(d, bc, b, t0, d.has_b ? d.M + 1 : 0);
    const int64_t sstride = d.layout == FILT_LAYOUT_TB ? d.B : 1;
    io_t *gxrow = gx != nullptr ? gx + sig_at(d, b, t0) : nullptr;
    // the adjoint itself, for a separate coefficient-gradient pass
    io_t *ybrow = ybo != nullptr ? ybo + sig_at(d, b, t0) : nullptr;
    // per-sample gradient rows: row of time t at grow + (t - t0) * gstride
    const int64_t gstride = d.layout == FILT_LAYOUT_TB ? d.B : 1;
    io_t *garow = (TV && GA) ? ga + row_at(d, b, t0, N) : nullptr;
    io_t *gbrow = (TV && GB) ? gb + row_at(d, b, t0, M + 1) : nullptr;
    // coefficient-gradient windows read x[t-(W-1)] and y[t-W]; times before 0
    // (chunk 0, first block only) come from the initial conditions instead
    const Cursor<io_t> xw = cursor(d, x, b, t0, 1, W + 4);
    const Cursor<io_t> yw = cursor(d, y, b, t0, 1, W + 4);
    io_t xic[W], yic[W];
#pragma unroll
    for (int q = 0; q < W; ++q) {
        xic[q] = (GB && xi != nullptr && q < M) ? xi[b * M + q] : io_t(0);
        yic[q] = (GA && yi != nullptr && q < N) ? yi[b * N + q] : io_t(0);
    }
    acc_t ss[W], rs[W];
#pragma unroll
    for (int q = 0; q < W; ++q) {
        ss[q] = acc_t(0);
        rs[q] = acc_t(0);
    }
    if (c + 1 < d.C) {
        const double *g = gin + (b * d.C + c) * (int64_t)(N + M);
#pragma unroll
        for (int i = 0; i < W; ++i) {
            if (i < N)
                ss[(i + 2) & m] = (acc_t)g[i];
            if (FIR && i < M)
                rs[(i + 2) & m] = (acc_t)g[N + i];
        }
    }
    double sga[W + 1], sgb[W];
#pragma unroll
    for (int k = 0; k <= W; ++k)
        sga[k] = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k)
        sgb[k] = 0.0;
    // signal windows for the coefficient gradients: per-sample gradients are
    // single products rounded to io_t, so the windows stay in io_t (half the
    // registers of FP64 windows); the time-invariant sums accumulate in FP64
    using win_t = std::conditional_t<TV, io_t, acc_t>;
    win_t wx[W], wy[W];
    const int64_t thi = t0 + d.L - 1;
    constexpr bool want_gb = GB;
    constexpr bool want_ga = GA;
    constexpr bool COEF = GA || GB;
#pragma unroll
    for (int q = 0; q < W; ++q) {
        wx[q] = win_t(0);
        wy[q] = win_t(0);
    }
    // chunks start on multiples of 32 >= W, so thi = t0 + L - 1 sits in
    // window slot W - 1 and every slot index below is a compile-time constant
    if constexpr (want_gb) {
#pragma unroll
        for (int k = 0; k < W - 1; ++k)
            wx[(m - k) & m] = ld_x<io_t, win_t>(d, x, xi, b, thi - k);
    }
    if constexpr (want_ga) {
#pragma unroll
        for (int k = 1; k < W; ++k)
            wy[(m - k) & m] = ld_y<io_t, win_t>(d, y, yi, b, thi - k);
    }
    using PF = Prefetch<W, TV, FIR, io_t>;
    auto fetch = [&](int64_t t, PF &p) {
        if constexpr (TV)
            ld_raw<W, FIR, AV>(d, acur.at(t0, t), bcur.at(t0, t), p.ra, p.rb);
        const io_t g = *gc.at(t0, t);
        p.s0 = t < d.T ? g : io_t(0);
        if constexpr (want_gb)
            p.s1 = *xw.at(t0, t - (W - 1));
        if constexpr (want_ga)
            p.s2 = *yw.at(t0, t - W);
    };
    // circular prefetch in decreasing time: the i-th step processed (time
    // thi - i) reads buf[i % P], fetched P steps earlier
    constexpr int P = kApplyPrefetch;
    constexpr int U = W > P ? W : P;
    PF buf[P];
#pragma unroll
    for (int q = 0; q < P; ++q)
        fetch(thi - q, buf[q]);
    for (int64_t tb = t0 + d.L - U; tb >= t0; tb -= U) {
#pragma unroll
        for (int s = U - 1; s >= 0; --s) {
            const int64_t t = tb + s;
            const bool in = t < d.T;
            const PF cur = buf[(U - 1 - s) % P];
            fetch(t - P, buf[(U - 1 - s) % P]);
            acc_t ca[W + 1], cb[W];
            if constexpr (TV) {
                cvt_row<W, FIR>(cur.ra, cur.rb, ca, cb);
            } else {
#pragma unroll
                for (int k = 0; k <= W; ++k)
                    ca[k] = la[k];
#pragma unroll
                for (int k = 0; k < W; ++k)
                    cb[k] = lb[k];
            }
            const acc_t yb = (acc_t)cur.s0 + ss[(1 - s) & m];
            if (ybrow != nullptr && in)
                ybrow[(t - t0) * sstride] = (io_t)yb;
            if (gxrow != nullptr && in) {
                acc_t gxv = cb[0] * yb;
                if constexpr (FIR)
                    gxv += rs[(1 - s) & m];
                gxrow[(t - t0) * sstride] = (io_t)gxv;
            }
            ss[(1 - s) & m] = KT < W ? acc_t(0) : -ca[W] * yb;
#pragma unroll
            for (int k = 1; k < W; ++k)
                if (k <= KT)
                    ss[(k + 1 - s) & m] -= ca[k] * yb;
            if constexpr (FIR) {
                rs[(1 - s) & m] = acc_t(0);
#pragma unroll
                for (int k = 1; k < W; ++k)
                    if (k <= KT)
                        rs[(k + 1 - s) & m] += cb[k] * yb;
            }
            if constexpr (COEF) {
                // only chunk 0's first block reaches times before 0
                const bool pre0 = (c == 0) && (tb == 0);
                if constexpr (want_gb) {
                    // x[t-(W-1)] = x[s-(W-1)] = xi[W-2-s] when it is before time 0
                    const io_t xv = (s < W - 1) ? xic[(W - 2 - s) < 0 ? 0 : (W - 2 - s)] : io_t(0);
                    wx[(s + 1) & m] = (win_t)((pre0 && s < W - 1) ? xv : cur.s1);
                    if constexpr (TV) {
                        if (in) {
                            io_t *o = gbrow + (t - t0) * gstride * (M + 1);
                            const io_t ybo = (io_t)yb;
#pragma unroll
                            for (int k = 0; k < W; ++k)
                                if (k <= M)
                                    o[k] = ybo * wx[(s - k) & m];
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < W; ++k)
                            if (k <= KT)
                                sgb[k] += (double)(yb * wx[(s - k) & m]);
                    }
                }
                if constexpr (want_ga) {
                    // y[t-W] = y[s-W] = yi[W-1-s] when it is before time 0
                    const io_t yv = yic[(s < W) ? (W - 1 - s) : 0];
                    wy[s & m] = (win_t)((pre0 && s < W) ? yv : cur.s2);
                    if constexpr (TV) {
                        if (in) {
                            io_t *o = garow + (t - t0) * gstride * N;
                            const io_t nyb = -(io_t)yb;
                            bool done = false;
                            if constexpr (AV && sizeof(io_t) == 4 && W % 4 == 0) {
                                {
#pragma unroll
                                    for (int q = 0; q < W / 4; ++q) {
                                        if (4 * q < N) {
                                            float4 v;
                                            v.x = nyb * wy[(s - 4 * q - 1) & m];
                                            v.y = nyb * wy[(s - 4 * q - 2) & m];
                                            v.z = nyb * wy[(s - 4 * q - 3) & m];
                                            v.w = nyb * wy[(s - 4 * q - 4) & m];
                                            *reinterpret_cast<float4 *>(o + 4 * q) = v;
                                        }
                                    }
                                    done = true;
                                }
                            }
                            if (!done) {
#pragma unroll
                                for (int k = 1; k <= W; ++k)
                                    if (k <= N)
                                        o[k - 1] = nyb * wy[(s - k) & m];
                            }
                        }
                    } else {
#pragma unroll
                        for (int k = 1; k <= W; ++k)
                            if (k <= KT)
                                sga[k] -= (double)(yb * wy[(s - k) & m]);
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if constexpr (!TV && COEF) {
        double *o = part + (b * d.C + c) * (int64_t)(N + M + 1);
#pragma unroll
        for (int k = 1; k <= W; ++k)
            if (k <= N)
                o[k - 1] = sga[k];
#pragma unroll
        for (int k = 0; k < W; ++k)
            if (k <= M)
                o[N + k] = sgb[k];
    }
    if (c == 0) {
#pragma unroll
        for (int i = 0; i < W; ++i) {
            if (gyi != nullptr && i < N)
                gyi[b * N + i] = (io_t)ss[(i + 2) & m];
            if (FIR && gxi != nullptr && i < M)
                gxi[b * M + i] = (io_t)rs[(i + 2) & m];
        }
    }
}

template <int W, bool TV, bool FIR, bool GA, bool GB, bool AV, typename io_t, typename acc_t,
          int KT = W>
__global__ void __launch_bounds__(kThreads)
k_bwd_apply(Dims d, const io_t *__restrict__ gy, const io_t *__restrict__ x,
            const io_t *__restrict__ xi, const io_t *__restrict__ y,
            const io_t *__restrict__ yi, const io_t *__restrict__ bc,
            const io_t *__restrict__ ac, const double *__restrict__ gin, io_t *__restrict__ gx,
            io_t *__restrict__ gb, io_t *__restrict__ ga, io_t *__restrict__ gxi,
            io_t *__restrict__ gyi, double *__restrict__ part, io_t *__restrict__ ybo)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= d.B * d.C)
        return;
    int64_t b, c, jj;
    decode(d, idx, d.C, b, c, jj);
    bwd_apply_item<W, TV, FIR, GA, GB, AV, io_t, acc_t, KT>(d, gy, x, xi, y, yi, bc, ac, gin, gx,
                                                            gb, ga, gxi, gyi, part, ybo, b, c);
}

// ---------------------------------------------------------------- drivers

// ---------------------------------------------------------------- quad applies
//
// Per-sample coefficients of order 9..16 without an FIR part: each
// (channel, chunk) chain runs on a lane quad, lane q owning taps
// 4q+1 .. 4q+4 (the layout of the summaries' particular solves), with the
// history window and the butterfly sum of the forward, and the shifted
// adjoint state of the transposed backward.  Per lane a step costs four FMAs
// and conversions instead of sixteen, and four times as many lanes carry the
// chains: a wave on its own issues an FP64 instruction only every ~13
// cycles, so the one-lane-per-chain applies were bound by that issue rate.
// FP64 state; CLAMP: the chunk runs past T (rows clamped, nothing stored
// past T).

constexpr int kQuadApplyPrefetch = 16;

template <bool AV, bool HASB, bool CLAMP, typename io_t>
__device__ __forceinline__ void fwd_apply_quad(const Dims &d, const io_t *__restrict__ x,
                                               const io_t *__restrict__ bc,
                                               const io_t *__restrict__ ac,
                                               const io_t *__restrict__ yi,
                                               const double *__restrict__ hin,
                                               io_t *__restrict__ y, int64_t b, int64_t c, int q)
{
    constexpr int P = kQuadApplyPrefetch;
    const int N = d.N;
    const int64_t t0 = c * d.L;
    const int64_t e0 = sig_at(d, b, t0);
    const int64_t es = d.layout == FILT_LAYOUT_TB ? d.B : 1;
    const int last = CLAMP ? (int)min<int64_t>(d.T - 1 - t0, d.L - 1) : (int)d.L - 1;
    const io_t *xp = x + e0;
    const RowWalk<io_t> aw = row_walk(d, ac, b, c * d.L, N);
    // order-0 FIR part: one tap per row (b_0)
    const RowWalk<io_t> bw = row_walk(d, HASB ? bc : x, b, c * d.L, HASB ? 1 : 0);
    io_t *yp = y + e0;
    double w[4];  // w[i] = y[t - 4q - 1 - i], from the entering state
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = 4 * q + i;
        double v = 0.0;
        if (k < N) {
            if (c == 0)
                v = yi != nullptr ? (double)yi[b * N + k] : 0.0;
            else
                v = hin[(b * d.C + c) * N + k];
        }
        w[i] = v;
    }
    auto fetch = [&](int rel, QuadRaw<io_t> &r) {
        const int rc = CLAMP ? min(rel, last) : rel;
        quad_taps<AV>(aw.at(rc), q, N, r.a);
        r.s = xp[rc * es];
        if constexpr (HASB)
            r.g = *bw.at(rc);
    };
    QuadRaw<io_t> buf[P];
    static_for<P>([&](auto I) { fetch(decltype(I)::value, buf[decltype(I)::value]); });
    for (int rel = 0; rel < d.L; rel += P) {
        static_for<P>([&](auto I) {
            constexpr int s = decltype(I)::value;
            const QuadRaw<io_t> r = buf[s];
            fetch(min(rel + P + s, (int)d.L - 1), buf[s]);
            double p = 0.0;
#pragma unroll
            for (int i = 3; i >= 0; --i)
                p = __builtin_fma(quad_coef<AV>(r.a, i, q, N), w[i], p);
            double tot = p + quad_dpp<kQuadXor1>(p);
            tot = tot + quad_dpp<kQuadXor2>(tot);
            const double v = HASB ? __builtin_fma((double)r.g, (double)r.s, tot)
                                  : (double)r.s + tot;
            if (q == 0 && (!CLAMP || rel + s <= last))
                yp[(rel + s) * es] = (io_t)v;
            const double prev = quad_dpp<kQuadFromPrev>(w[3]);
            w[3] = w[2];
            w[2] = w[1];
            w[1] = w[0];
            w[0] = q == 0 ? v : prev;
        });
    }
}

template <bool AV, bool HASB, typename io_t>
__global__ void __launch_bounds__(kThreads)
k_fwd_apply_quad(Dims d, const io_t *__restrict__ x, const io_t *__restrict__ bc,
                 const io_t *__restrict__ ac, const io_t *__restrict__ yi,
                 const double *__restrict__ hin, io_t *__restrict__ y)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((idx >> 2) >= d.B * d.C)  // whole quads
        return;
    int64_t b, c, jj;
    decode(d, idx >> 2, d.C, b, c, jj);
    if ((c + 1) * d.L > d.T)
        fwd_apply_quad<AV, HASB, true>(d, x, bc, ac, yi, hin, y, b, c, (int)(idx & 3));
    else
        fwd_apply_quad<AV, HASB, false>(d, x, bc, ac, yi, hin, y, b, c, (int)(idx & 3));
}

// Adjoint of chunk c from the entering state gin (transposed form, as in
// bwd_apply_item without an FIR part): writes ybar to ybo and gx = b_0 ybar
// to gx (either may be null; they may be the same buffer without b), and
// gyi from chunk 0.  GA: also the per-sample gradient rows
// ga_k[t] = -ybar[t] y[t-k] (Sec. 3.1 Eq. 8 per sample), lane q its taps
// 4q+1 .. 4q+4 from a window wy[i] = y[t - 4q - 1 - i] that slides down one
// sample per step (one new y value per lane and step; y before time 0 from
// the initial conditions yi).
template <bool AV, bool HASB, bool CLAMP, bool GA, typename io_t>
__device__ __forceinline__ void bwd_apply_quad(const Dims &d, const io_t *__restrict__ gy,
                                               const io_t *__restrict__ bc,
                                               const io_t *__restrict__ ac,
                                               const double *__restrict__ gin, io_t *gx,
                                               io_t *__restrict__ gyi, io_t *ybo,
                                               const io_t *__restrict__ y,
                                               const io_t *__restrict__ yi,
                                               io_t *__restrict__ ga, int64_t b, int64_t c,
                                               int q)
{
    constexpr int P = kQuadApplyPrefetch;
    const int N = d.N;
    const int64_t t0 = c * d.L;
    const int64_t e0 = sig_at(d, b, t0);
    const int64_t es = d.layout == FILT_LAYOUT_TB ? d.B : 1;
    const int last = CLAMP ? (int)min<int64_t>(d.T - 1 - t0, d.L - 1) : (int)d.L - 1;
    const io_t *g0 = gy + e0;
    const RowWalk<io_t> aw = row_walk(d, ac, b, c * d.L, N);
    const RowWalk<io_t> bw = row_walk(d, HASB ? bc : gy, b, c * d.L, HASB ? 1 : 0);
    double st[4];  // st[i] = s_{4q+1+i}
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k = 4 * q + i;
        st[i] = (c + 1 < d.C && k < N) ? gin[(b * d.C + c) * N + k] : 0.0;
    }
    // y at chunk-relative time tt: clamped below T (such steps store nothing),
    // initial conditions before time 0 (zero past N, where no tap reads them)
    auto yat = [&](int tt) -> io_t {
        if (t0 + tt >= 0)
            return y[e0 + min((int64_t)tt, d.T - 1 - t0) * es];
        const int64_t m = -(t0 + tt);  // y[-m] = yi[m - 1]
        return (yi != nullptr && m <= N) ? yi[b * N + (m - 1)] : io_t(0);
    };
    io_t wy[4];  // wy[i] = y[t - 4q - 1 - i] for the step t about to run
    if constexpr (GA) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            wy[i] = yat((int)d.L - 1 - 4 * q - 1 - i);
    }
    auto fetch = [&](int rel, QuadRaw<io_t> &r) {
        const int rc = CLAMP ? min(rel, last) : rel;
        quad_taps<AV>(aw.at(rc), q, N, r.a);
        const io_t g = g0[rc * es];
        r.s = (!CLAMP || rel <= last) ? g : io_t(0);
        if constexpr (HASB)
            r.g = *bw.at(rc);
        if constexpr (GA)
            r.y = yat(rel - 4 * q - 5);  // enters the window after this step
    };
    QuadRaw<io_t> buf[P];
    static_for<P>([&](auto I) {
        fetch((int)d.L - P + decltype(I)::value, buf[decltype(I)::value]);
    });
    for (int rel = (int)d.L - P; rel >= 0; rel -= P) {
        static_for<P>([&](auto I) {
            constexpr int s = P - 1 - decltype(I)::value;
            const QuadRaw<io_t> r = buf[s];
            fetch(max(rel - P + s, 0), buf[s]);
            const double yb = (double)r.s + quad_dpp<kQuadLane0>(st[0]);
            if constexpr (GA) {
                if (!CLAMP || rel + s <= last) {
                    io_t gv[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        gv[i] = (io_t)(-yb * (double)wy[i]);
                    io_t *o = ga + (e0 + (int64_t)(rel + s) * es) * N + 4 * q;
                    if constexpr (sizeof(io_t) == 4) {
                        if (d.ga_vec) {
                            using f4 = float __attribute__((ext_vector_type(4)));
                            const f4 v4 = {gv[0], gv[1], gv[2], gv[3]};
                            __builtin_nontemporal_store(v4, reinterpret_cast<f4 *>(o));
                        } else {
#pragma unroll
                            for (int i = 0; i < 4; ++i)
                                if (4 * q + i < N)
                                    __builtin_nontemporal_store(gv[i], o + i);
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            if (4 * q + i < N)
                                o[i] = gv[i];
                    }
                }
                wy[0] = wy[1];
                wy[1] = wy[2];
                wy[2] = wy[3];
                wy[3] = r.y;
            }
            if (q == 0 && (!CLAMP || rel + s <= last)) {
                const int64_t o = (int64_t)(rel + s) * es;
                if (ybo != nullptr)
                    ybo[e0 + o] = (io_t)yb;
                if (gx != nullptr && (HASB || gx != ybo))
                    gx[e0 + o] = (io_t)(HASB ? (double)r.g * yb : yb);
            }
            const double nx = quad_dpp<kQuadFromNext>(st[0]);
            st[0] = __builtin_fma(quad_coef<AV>(r.a, 0, q, N), yb, st[1]);
            st[1] = __builtin_fma(quad_coef<AV>(r.a, 1, q, N), yb, st[2]);
            st[2] = __builtin_fma(quad_coef<AV>(r.a, 2, q, N), yb, st[3]);
            st[3] = __builtin_fma(quad_coef<AV>(r.a, 3, q, N), yb, q == 3 ? 0.0 : nx);
        });
    }
    if (c == 0 && gyi != nullptr) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (4 * q + i < N)
                gyi[b * N + 4 * q + i] = (io_t)st[i];
    }
}

template <bool AV, bool HASB, bool GA, typename io_t>
__global__ void __launch_bounds__(kThreads)
k_bwd_apply_quad(Dims d, const io_t *__restrict__ gy, const io_t *__restrict__ bc,
                 const io_t *__restrict__ ac, const double *__restrict__ gin, io_t *gx,
                 io_t *__restrict__ gyi, io_t *ybo, const io_t *__restrict__ y,
                 const io_t *__restrict__ yi, io_t *__restrict__ ga)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((idx >> 2) >= d.B * d.C)
        return;
    int64_t b, c, jj;
    decode(d, idx >> 2, d.C, b, c, jj);
    if ((c + 1) * d.L > d.T)
        bwd_apply_quad<AV, HASB, true, GA>(d, gy, bc, ac, gin, gx, gyi, ybo, y, yi, ga, b, c,
                                           (int)(idx & 3));
    else
        bwd_apply_quad<AV, HASB, false, GA>(d, gy, bc, ac, gin, gx, gyi, ybo, y, yi, ga, b, c,
                                            (int)(idx & 3));
}

// Quad applies take per-sample problems of the order-16 bucket without an
// FIR part and with FP64 state.
template <int W, typename io_t, typename acc_t>
constexpr bool kQuadApply = W == 16 && sizeof(acc_t) == 8;

inline bool quad_apply_eligible(const Dims &d) { return d.tv && d.M == 0 && d.N > 0; }

template <typename io_t>
filt_status fwd_apply_quad_run(const Dims &d, const io_t *x, const io_t *bc, const io_t *ac,
                               const io_t *yi, const double *states, io_t *y, hipStream_t st)
{
    const int64_t lanes = d.B * d.C * 4;
    const dim3 grid((unsigned)((lanes + kThreads - 1) / kThreads));
#define FILT_QF(AVV, HB)                                                                           \
    FILT_LAUNCH("fwd_apply", (k_fwd_apply_quad<AVV, HB, io_t>), grid, dim3(kThreads), 0, st, d,   \
                x, bc, ac, yi, states, y)
    if (d.a_vec) {
        if (d.has_b)
            FILT_QF(true, true);
        else
            FILT_QF(true, false);
    } else {
        if (d.has_b)
            FILT_QF(false, true);
        else
            FILT_QF(false, false);
    }
#undef FILT_QF
    return check_launch("forward apply");
}

// ga non-null: the gradient rows are formed in the same pass (needs y, yi).
template <typename io_t>
filt_status bwd_apply_quad_run(const Dims &d, const io_t *gy, const io_t *bc, const io_t *ac,
                               const double *states, io_t *gx, io_t *gyi, io_t *ybo,
                               const io_t *y, const io_t *yi, io_t *ga, hipStream_t st)
{
    const int64_t lanes = d.B * d.C * 4;
    const dim3 grid((unsigned)((lanes + kThreads - 1) / kThreads));
#define FILT_QB(AVV, HB, GAV)                                                                      \
    FILT_LAUNCH("bwd_apply", (k_bwd_apply_quad<AVV, HB, GAV, io_t>), grid, dim3(kThreads), 0, st, \
                d, gy, bc, ac, states, gx, gyi, ybo, y, yi, ga)
#define FILT_QB_G(AVV, HB)                                                                         \
    do {                                                                                           \
        if (ga != nullptr)                                                                         \
            FILT_QB(AVV, HB, true);                                                                \
        else                                                                                       \
            FILT_QB(AVV, HB, false);                                                               \
    } while (0)
    if (d.a_vec) {
        if (d.has_b)
            FILT_QB_G(true, true);
        else
            FILT_QB_G(true, false);
    } else {
        if (d.has_b)
            FILT_QB_G(false, true);
        else
            FILT_QB_G(false, false);
    }
#undef FILT_QB_G
#undef FILT_QB
    return check_launch("backward apply");
}

template <int W, bool FIR, typename io_t, typename acc_t>
filt_status fwd_apply(const Dims &d, const io_t *x, const io_t *bc, const io_t *ac,
                      const io_t *xi, const io_t *yi, const double *states, io_t *y,
                      hipStream_t st)
{
    if (d.tv && d.a_vec)
        FILT_LAUNCH("fwd_apply", (k_fwd_apply<W, true, FIR, true, io_t, acc_t>),
                    dim3(blocks_for(d.B * d.C)), dim3(block_for(d.B * d.C)), 0, st, d, x, xi, bc, ac, yi,
                    states, y);
    else if (d.tv)
        FILT_LAUNCH("fwd_apply", (k_fwd_apply<W, true, FIR, false, io_t, acc_t>),
                    dim3(blocks_for(d.B * d.C)), dim3(block_for(d.B * d.C)), 0, st, d, x, xi, bc, ac, yi,
                    states, y);
    else
        lti_tap_bound<W, FIR, io_t, acc_t>(d, [&](auto kt) {
            constexpr int KT = decltype(kt)::value;
            FILT_LAUNCH("fwd_apply", (k_fwd_apply<W, false, FIR, false, io_t, acc_t, KT>),
                        dim3(blocks_for(d.B * d.C)), dim3(block_for(d.B * d.C)), 0, st, d, x, xi,
                        bc, ac, yi, states, y);
        });
    return check_launch("forward apply");
}

template <int W, typename io_t, typename acc_t>
filt_status forward_w(const Dims &d, const io_t *x, const io_t *bc, const io_t *ac,
                      const io_t *xi, const io_t *yi, io_t *y, char *ws, hipStream_t st)
{
    const WsPlan w = ws_plan(d);
    double *summ = (double *)(ws + w.summ);
    double *phi = (double *)(ws + w.phi);
    double *states = (double *)(ws + w.states);
    const int N = d.N;
    if (d.C > 1 && N > 0) {
        filt_status s = fwd_summary_w<W, io_t>(d, x, xi, bc, ac, summ, phi, st);
        if (s != FILT_OK)
            return s;
        CarryArgs a{};
        a.summ = summ;
        a.phi = phi;
        a.SS = (int64_t)N * N + N;
        a.soff = (int64_t)N * N;
        a.D = N;
        a.R = 0;
        a.bwd = 0;
        a.agg = (double *)(ws + w.agg);
        a.bstart = (double *)(ws + w.bstart);
        a.states = states;
        s = carry_run(d, a, yi, sizeof(io_t) == 8, st);
        if (s != FILT_OK)
            return s;
    }
    if constexpr (sizeof(io_t) == 4 && sizeof(acc_t) == 8 && W <= 16) {
        if (stream_eligible(d))
            return stream_forward_run<W>(d, x, ac, yi, states, y, st);
        // time-invariant all-pole [B, T]: the same staged apply, the channel's
        // row read as the row of one frame of T samples
        if (lti_stream_eligible(d)) {
            Dims e = d;
            set_rows(e, d.T);
            return stream_forward_run<W>(e, x, ac, yi, states, y, st);
        }
    }
    if constexpr (kQuadApply<W, io_t, acc_t>) {
        if (quad_apply_eligible(d))
            return fwd_apply_quad_run<io_t>(d, x, bc, ac, yi, states, y, st);
    }
    if (d.M > 0)
        return fwd_apply<W, true, io_t, acc_t>(d, x, bc, ac, xi, yi, states, y, st);
    return fwd_apply<W, false, io_t, acc_t>(d, x, bc, ac, xi, yi, states, y, st);
}

template <int W, bool FIR, typename io_t, typename acc_t>
filt_status bwd_apply(const Dims &d, const io_t *gy, const io_t *x, const io_t *y,
                      const io_t *bc, const io_t *ac, const io_t *xi, const io_t *yi,
                      const double *states, io_t *gx, io_t *gb, io_t *ga, io_t *gxi, io_t *gyi,
                      double *part, io_t *ybo, hipStream_t st)
{
#define FILT_BWD_APPLY(TVV, GAV, GBV, AVV)                                                         \
    lti_tap_bound<W, FIR && !TVV, io_t, acc_t>(d, [&](auto kt) {                                   \
        constexpr int KT = decltype(kt)::value;                                                    \
        FILT_LAUNCH("bwd_apply", (k_bwd_apply<W, TVV, FIR, GAV, GBV, AVV, io_t, acc_t, KT>),       \
                    dim3(blocks_for(d.B * d.C)), dim3(block_for(d.B * d.C)), 0, st, d, gy, x, xi,  \
                    y, yi, bc, ac, states, gx, gb, ga, gxi, gyi, part, ybo);                       \
    })
#define FILT_BWD_APPLY_G(TVV, AVV)                                                                 \
    do {                                                                                           \
        if (ga != nullptr && gb != nullptr)                                                        \
            FILT_BWD_APPLY(TVV, true, true, AVV);                                                  \
        else if (ga != nullptr)                                                                    \
            FILT_BWD_APPLY(TVV, true, false, AVV);                                                 \
        else if (gb != nullptr)                                                                    \
            FILT_BWD_APPLY(TVV, false, true, AVV);                                                 \
        else                                                                                       \
            FILT_BWD_APPLY(TVV, false, false, AVV);                                                \
    } while (0)
    if (d.tv && d.a_vec)
        FILT_BWD_APPLY_G(true, true);
    else if (d.tv)
        FILT_BWD_APPLY_G(true, false);
    else
        FILT_BWD_APPLY_G(false, false);
#undef FILT_BWD_APPLY_G
#undef FILT_BWD_APPLY
    return check_launch("backward apply");
}

template <int W, typename io_t, typename acc_t>
filt_status backward_w(const Dims &d, const io_t *gy, const io_t *x, const io_t *y,
                       const io_t *bc, const io_t *ac, const io_t *xi, const io_t *yi, io_t *gx,
                       io_t *gb, io_t *ga, io_t *gxi, io_t *gyi, char *ws, hipStream_t st)
{
    const WsPlan w = ws_plan(d);
    double *summ = (double *)(ws + w.summ);
    double *phi = (double *)(ws + w.phi);
    double *states = (double *)(ws + w.states);
    double *part = (double *)(ws + w.part);
    const int N = d.N, M = d.M;
    if (d.C > 1 && N + M > 0) {
        filt_status s = bwd_summary_w<W, io_t>(d, gy, bc, ac, summ, phi, st);
        if (s != FILT_OK)
            return s;
        if (N > 0) {
            CarryArgs a{};
            a.summ = summ;
            a.phi = phi;
            a.SS = (int64_t)(N + 1) * (N + M);
            a.soff = (int64_t)N * N;
            a.D = N;
            a.R = M;
            a.bwd = 1;
            a.agg = (double *)(ws + w.agg);
            a.bstart = (double *)(ws + w.bstart);
            a.states = states;
            s = carry_run(d, a, nullptr, false, st);
        } else {
            s = fir_states_run(d, summ, states, st);
        }
        if (s != FILT_OK)
            return s;
    }
    if constexpr (sizeof(io_t) == 4 && sizeof(acc_t) == 8 && W <= 16) {
        // [B, T] all-pole: staged apply writes ybar (gx itself when wanted,
        // since gx = ybar for b = [1]); ga comes from the coalesced pass
        if (stream_eligible(d) && (ga == nullptr || d.fd.m != 0 || tv_coef_grads_fits(d))) {
            io_t *yb = gx != nullptr ? gx : (io_t *)(ws + w.yb);
            filt_status s = stream_backward_run<W>(d, gy, ac, states, yb, gyi, st);
            if (s != FILT_OK || ga == nullptr)
                return s;
            if (d.fd.m != 0)
                return frame_coef_grads_run<io_t>(d, yb, x, xi, y, yi, ga, nullptr, st);
            return tv_coef_grads_run(d, yb, x, xi, y, yi, ga, nullptr, st);
        }
        // time-invariant all-pole [B, T] with gx (= ybar): the staged adjoint
        // as one frame, then ga summed over time from ybar
        if (lti_stream_eligible(d) && gx != nullptr) {
            Dims e = d;
            set_rows(e, d.T);
            filt_status s = stream_backward_run<W>(e, gy, ac, states, gx, gyi, st);
            if (s != FILT_OK || ga == nullptr)
                return s;
            return lti_allpole_ga_run(d, gx, y, yi, ga, part, st);
        }
    }
    // Order-16 per-sample problems without an FIR part: quad adjoint writing
    // ybar (into gx itself without b, where gx = ybar), then the coefficient
    // gradients from it in a fully parallel pass.
    if constexpr (kQuadApply<W, io_t, acc_t>) {
        // per-sample ga alone is formed inside the adjoint pass; with gb (an
        // order-0 FIR part), or for frame-held rows, the gradients come from
        // ybar in a separate pass
        const bool fr = d.fd.m != 0;
        if (quad_apply_eligible(d) && gb == nullptr && !fr)
            return bwd_apply_quad_run<io_t>(d, gy, bc, ac, states, gx, gyi, nullptr, y, yi, ga,
                                            st);
        if (quad_apply_eligible(d) && (fr || (sizeof(io_t) == 4 && tv_coef_grads_fits(d)))) {
            io_t *yb = (gx != nullptr && !d.has_b) ? gx : (io_t *)(ws + w.yb);
            filt_status s = bwd_apply_quad_run<io_t>(d, gy, bc, ac, states, gx, gyi, yb, y, yi,
                                                     nullptr, st);
            if (s != FILT_OK || (ga == nullptr && gb == nullptr))
                return s;
            if (fr)
                return frame_coef_grads_run<io_t>(d, yb, x, xi, y, yi, ga, gb, st);
            if constexpr (sizeof(io_t) == 4)
                return tv_coef_grads_run(d, yb, x, xi, y, yi, ga, gb, st);
        }
    }
    // Other order-16 per-sample problems: the fused adjoint with the
    // coefficient products needs more registers than a wavefront has and
    // spills to AGPRs on every step, so the apply writes the adjoint (FP32)
    // and a fully parallel pass forms ga and gb from it.  Frame-held rows
    // always take that route: their gradients are sums over each frame.
    const bool frames = d.tv && d.fd.m != 0;
    const bool split = (ga != nullptr || gb != nullptr) &&
                       (frames || (d.tv && W >= 16 && sizeof(io_t) == 4 && tv_coef_grads_fits(d)));
    io_t *ybo = split ? (io_t *)(ws + w.yb) : nullptr;
    io_t *ga_f = split ? nullptr : ga;
    io_t *gb_f = split ? nullptr : gb;
    filt_status s = (M > 0) ? bwd_apply<W, true, io_t, acc_t>(d, gy, x, y, bc, ac, xi, yi, states,
                                                              gx, gb_f, ga_f, gxi, gyi, part, ybo,
                                                              st)
                            : bwd_apply<W, false, io_t, acc_t>(d, gy, x, y, bc, ac, xi, yi,
                                                               states, gx, gb_f, ga_f, gxi, gyi,
                                                               part, ybo, st);
    if (s != FILT_OK)
        return s;
    if (split && frames)
        return frame_coef_grads_run<io_t>(d, ybo, x, xi, y, yi, ga, gb, st);
    if constexpr (sizeof(io_t) == 4) {
        if (split)
            return tv_coef_grads_run(d, ybo, x, xi, y, yi, ga, gb, st);
    }
    if (!d.tv && (ga != nullptr || gb != nullptr))
        s = reduce_lti_run(d, part, ga, gb, sizeof(io_t) == 8, st);
    return s;
}

}  // namespace filt_detail
