// summary.h -- phase 1 of the chunked scan: per-chunk affine summaries.
//
// A chunk's summary is the map from the filter state entering the chunk to
// the state leaving it: the transition Phi_c (the product of the chunk's
// companion matrices, Sec. 2 Eq. 4) and the zero-state end state s_c.  Phi_c
// is found by solving the chunk from each unit state (column j), s_c by
// solving it from zero state with the real input.  All of it runs in FP64:
// companion-form transitions have entries far above 1 when poles cluster near
// the unit circle, and an FP32 Phi would lose the digits the carry needs.
//
// Per-sample coefficients: every chunk needs N + 1 solves.  Each lane runs S
// of them side by side, so one coefficient row fetched (and converted) per
// step feeds S recursions; nl = ceil((N + 1) / S) adjacent lanes cover one
// chunk.  Rows are fetched two steps ahead of their use.  Time-invariant
// coefficients: one particular solve per chunk, and the N homogeneous solves
// once per channel (Phi is the same for every chunk).
//
// Register histories live in W registers addressed modulo W; the time loop
// is unrolled by W so every index is a compile-time constant.
#pragma once

#include "common.h"

namespace filt_detail {

// ---------------------------------------------------------------- forward

// S forward recursions over [t0, t0 + L).  h[q][t mod W] = y_q[t]; hx[t mod
// W] = x[t].  Slot q is driven by wgt[q] * (b * x)[t] (XIN) and its history.
template <int W, int S, bool TV, bool FIR, bool XIN, bool AV, typename io_t>
__device__ __forceinline__ void fwd_solves(const Dims &d, int64_t t0, const Cursor<io_t> &xc,
                                           const Cursor<io_t> &acur, const Cursor<io_t> &bcur,
                                           double (&h)[S][W], double (&hx)[W],
                                           const double (&wgt)[S], const double (&la)[W + 1],
                                           const double (&lb)[W])
{
    constexpr int m = W - 1;
    const int64_t tend = t0 + d.L;
    using PF = Prefetch<W, TV, FIR, io_t>;
    auto fetch = [&](int64_t t, PF &p) {
        if constexpr (TV)
            ld_raw<W, FIR, AV>(d, acur.at(t0, t), bcur.at(t0, t), p.ra, p.rb);
        if constexpr (XIN)
            p.s0 = *xc.at(t0, t);  // steps past T are never summarised
    };
    // circular prefetch: step t's data is fetched P steps ahead into buf[t % P];
    // the loop is unrolled by U = max(W, P) so every index is static
    constexpr int P = kSummaryPrefetch;
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
            double ca[W + 1], cb[W];
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
            double u = 0.0;
            if constexpr (XIN) {
                hx[s & m] = (double)cur.s0;
                if constexpr (FIR) {
#pragma unroll
                    for (int k = W - 1; k >= 0; --k)
                        u += cb[k] * hx[(s - k) & m];
                } else {
                    u = cb[0] * hx[s & m];
                }
            }
#pragma unroll
            for (int q = 0; q < S; ++q) {
                double p0 = XIN ? wgt[q] * u : 0.0, p1 = 0.0;
#pragma unroll
                for (int k = W; k >= 2; --k) {
                    if (k & 1)
                        p1 -= ca[k] * h[q][(s - k) & m];
                    else
                        p0 -= ca[k] * h[q][(s - k) & m];
                }
                h[q][s & m] = (p0 + p1) - ca[1] * h[q][(s - 1) & m];
            }
            // keep each step's live range to itself (bounded registers); the
            // prefetch above already covers the load latency
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Items (r, b, c): lane r of chunk c = c_first + cc runs solves
// j = j_first + r*S + q (q < S, j < j_first + nj).  j < N: unit state
// y(t0-1-j) = 1, no input -> column j of Phi_c.  j == N: zero state, real
// input -> s_c.  State index i = 0..N-1 is y(t-1-i).
//   summ[(b*C + c)*(N*N + N) + i*N + j] = Phi_c[i][j] (per-sample coefficients)
//   phi[b*N*N + i*N + j]                = Phi[i][j]   (time-invariant)
//   summ[(b*C + c)*(N*N + N) + N*N + i] = s_c[i]
template <int W, int S, bool TV, bool FIR, bool XIN, bool AV, typename io_t>
__device__ __forceinline__ void fwd_summary_item(const Dims &d, const io_t *__restrict__ x,
                                                 const io_t *__restrict__ xi,
                                                 const io_t *__restrict__ bc,
                                                 const io_t *__restrict__ ac, int j_first, int nj,
                                                 double *__restrict__ summ,
                                                 double *__restrict__ phi, int64_t b, int64_t c,
                                                 int r)
{
    constexpr int m = W - 1;
    const int64_t t0 = c * d.L;
    const int N = d.N;

    double la[W + 1], lb[W];
    if constexpr (!TV)
        ld_row_lti<W, FIR>(d, bc, ac, b, la, lb);
    const Cursor<io_t> xc = cursor(d, x, b, t0, 1);
    const Cursor<io_t> acur = cursor(d, ac, b, t0, d.N);
    const Cursor<io_t> bcur = cursor(d, bc, b, t0, d.has_b ? d.M + 1 : 0);
    double h[S][W], hx[W], wgt[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const int j = j_first + r * S + q;
        wgt[q] = (j == N) ? 1.0 : 0.0;
#pragma unroll
        for (int e = 0; e < W; ++e)
            h[q][e] = (j < N && e == ((-(j + 1)) & m)) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int e = 0; e < W; ++e)
        hx[e] = 0.0;
    if constexpr (XIN && FIR) {
#pragma unroll
        for (int k = 1; k < W; ++k)
            hx[(-k) & m] = ld_x<io_t, double>(d, x, xi, b, t0 - k);
    }
    fwd_solves<W, S, TV, FIR, XIN, AV>(d, t0, xc, acur, bcur, h, hx, wgt, la, lb);
    const int64_t SS = (int64_t)N * N + N;
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const int j = j_first + r * S + q;
        if (j >= j_first + nj || j > N)
            continue;
        if (j == N) {
            double *o = summ + (b * d.C + c) * SS + (int64_t)N * N;
#pragma unroll
            for (int i = 0; i < W; ++i)
                if (i < N)
                    o[i] = h[q][(-(i + 1)) & m];
        } else {
            double *o = TV ? summ + (b * d.C + c) * SS : phi + b * (int64_t)N * N;
#pragma unroll
            for (int i = 0; i < W; ++i)
                if (i < N)
                    o[(int64_t)i * N + j] = h[q][(-(i + 1)) & m];
        }
    }
}

template <int W, int S, bool TV, bool FIR, bool XIN, bool AV, typename io_t>
__global__ void __launch_bounds__(kThreads)
k_fwd_summary(Dims d, const io_t *__restrict__ x, const io_t *__restrict__ xi,
              const io_t *__restrict__ bc, const io_t *__restrict__ ac, int64_t c_first,
              int64_t ncs, int j_first, int nj, double *__restrict__ summ,
              double *__restrict__ phi)
{
    const int nl = (nj + S - 1) / S;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= d.B * ncs * nl)
        return;
    int64_t b, cc;
    int r;
    decode_lanes(d, idx, ncs, nl, b, cc, r);
    fwd_summary_item<W, S, TV, FIR, XIN, AV>(d, x, xi, bc, ac, j_first, nj, summ, phi, b,
                                             c_first + cc, r);
}

// ---------------------------------------------------------------- backward

// S adjoint recursions over [t0, t0 + L) in decreasing time, transposed
// (scatter) form.  Before processing time t, slot q's adjoint state s_k
// (the part of ybar[t-1+k] still to be added) is in ss[q][(k - t) mod W] and
// its FIR adjoint state r_k (the part of gx[t-1+k] still to be added) in
// rs[q][(k - t) mod W].  Per step:
//   ybar = wgt[q] gy[t] + s_1,  s_k <- s_{k+1} - a_k[t] ybar,
//   r_k <- r_{k+1} + b_k[t] ybar.
template <int W, int S, bool TV, bool FIR, bool GIN, bool AV, typename io_t>
__device__ __forceinline__ void bwd_solves(const Dims &d, int64_t t0, const Cursor<io_t> &gc,
                                           const Cursor<io_t> &acur, const Cursor<io_t> &bcur,
                                           double (&ss)[S][W], double (&rs)[S][W],
                                           const double (&wgt)[S], const double (&la)[W + 1],
                                           const double (&lb)[W])
{
    constexpr int m = W - 1;
    using PF = Prefetch<W, TV, FIR, io_t>;
    auto fetch = [&](int64_t t, PF &p) {
        if constexpr (TV)
            ld_raw<W, FIR, AV>(d, acur.at(t0, t), bcur.at(t0, t), p.ra, p.rb);
        if constexpr (GIN) {
            const io_t g = *gc.at(t0, t);
            p.s0 = t < d.T ? g : io_t(0);
        }
    };
    const int64_t thi = t0 + d.L - 1;
    // circular prefetch in decreasing time: the i-th step processed (time
    // thi - i) reads buf[i % P], fetched P steps earlier
    constexpr int P = kSummaryPrefetch;
    constexpr int U = W > P ? W : P;
    PF buf[P];
#pragma unroll
    for (int q = 0; q < P; ++q)
        fetch(thi - q, buf[q]);
    for (int64_t tb = t0 + d.L - U; tb >= t0; tb -= U) {
#pragma unroll
        for (int s = U - 1; s >= 0; --s) {
            const int64_t t = tb + s;
            const PF cur = buf[(U - 1 - s) % P];
            fetch(t - P, buf[(U - 1 - s) % P]);
            double ca[W + 1], cb[W];
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
            double g = 0.0;
            if constexpr (GIN)
                g = (double)cur.s0;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const double yb = (GIN ? wgt[q] * g : 0.0) + ss[q][(1 - s) & m];
                ss[q][(1 - s) & m] = -ca[W] * yb;
#pragma unroll
                for (int k = 1; k < W; ++k)
                    ss[q][(k + 1 - s) & m] -= ca[k] * yb;
                if constexpr (FIR) {
                    rs[q][(1 - s) & m] = 0.0;
#pragma unroll
                    for (int k = 1; k < W; ++k)
                        rs[q][(k + 1 - s) & m] += cb[k] * yb;
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Items (r, b, c) for chunks c = c_first + cc; slots as in the forward.
// j < N: unit state s_{j+1} = 1, gy = 0; j == N: zero state with the real gy.
// Outgoing (s, r) of the chunk, column j (SB = (N+1)(N+M) per chunk):
//   summ[base + i*N + j] = s_{i+1}                     (i < N)  Phi'
//   summ[base + N*N + i] = s0_{i+1}                    (particular)
//   summ[base + N*N + N + i*N + j] = r_{i+1}           (i < M)  R
//   summ[base + N*N + N + M*N + i] = r0_{i+1}          (particular)
// Time-invariant Phi' and R go to phi[b*(N*N + M*N) + ...].
// Before the first (highest) time and after the last, s_k sits in slot
// (k + 1) mod W.
template <int W, int S, bool TV, bool FIR, bool GIN, bool AV, typename io_t>
__device__ __forceinline__ void bwd_summary_item(const Dims &d, const io_t *__restrict__ gy,
                                                 const io_t *__restrict__ bc,
                                                 const io_t *__restrict__ ac, int j_first, int nj,
                                                 double *__restrict__ summ,
                                                 double *__restrict__ phi, int64_t b, int64_t c,
                                                 int r)
{
    constexpr int m = W - 1;
    const int64_t t0 = c * d.L;
    const int N = d.N, M = d.M;
    double la[W + 1], lb[W];
    if constexpr (!TV)
        ld_row_lti<W, FIR>(d, bc, ac, b, la, lb);
    const Cursor<io_t> gc = cursor(d, gy, b, t0, 1);
    const Cursor<io_t> acur = cursor(d, ac, b, t0, d.N);
    const Cursor<io_t> bcur = cursor(d, bc, b, t0, d.has_b ? d.M + 1 : 0);
    double ss[S][W], rs[S][W], wgt[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const int j = j_first + r * S + q;
        wgt[q] = (j == N) ? 1.0 : 0.0;
#pragma unroll
        for (int e = 0; e < W; ++e) {
            ss[q][e] = (j < N && e == ((j + 2) & m)) ? 1.0 : 0.0;
            rs[q][e] = 0.0;
        }
    }
    bwd_solves<W, S, TV, FIR, GIN, AV>(d, t0, gc, acur, bcur, ss, rs, wgt, la, lb);
    const int64_t SB = (int64_t)(N + 1) * (N + M);
    double *base = summ + (b * d.C + c) * SB;
#pragma unroll
    for (int q = 0; q < S; ++q) {
        const int j = j_first + r * S + q;
        if (j >= j_first + nj || j > N)
            continue;
        if (j == N) {
#pragma unroll
            for (int i = 0; i < W; ++i) {
                if (i < N)
                    base[(int64_t)N * N + i] = ss[q][(i + 2) & m];
                if (FIR && i < M)
                    base[(int64_t)N * N + N + (int64_t)M * N + i] = rs[q][(i + 2) & m];
            }
        } else {
            double *pm = TV ? base : phi + b * ((int64_t)N * N + (int64_t)M * N);
            double *rm = TV ? base + (int64_t)N * N + N : pm + (int64_t)N * N;
#pragma unroll
            for (int i = 0; i < W; ++i) {
                if (i < N)
                    pm[(int64_t)i * N + j] = ss[q][(i + 2) & m];
                if (FIR && i < M)
                    rm[(int64_t)i * N + j] = rs[q][(i + 2) & m];
            }
        }
    }
}

template <int W, int S, bool TV, bool FIR, bool GIN, bool AV, typename io_t>
__global__ void __launch_bounds__(kThreads)
k_bwd_summary(Dims d, const io_t *__restrict__ gy, const io_t *__restrict__ bc,
              const io_t *__restrict__ ac, int64_t c_first, int64_t ncs, int j_first, int nj,
              double *__restrict__ summ, double *__restrict__ phi)
{
    const int nl = (nj + S - 1) / S;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= d.B * ncs * nl)
        return;
    int64_t b, cc;
    int r;
    decode_lanes(d, idx, ncs, nl, b, cc, r);
    bwd_summary_item<W, S, TV, FIR, GIN, AV>(d, gy, bc, ac, j_first, nj, summ, phi, b,
                                             c_first + cc, r);
}

// ---------------------------------------------------------------- launch

template <int W, bool FIR, typename io_t>
filt_status fwd_summary_fir(const Dims &d, const io_t *x, const io_t *xi, const io_t *bc,
                            const io_t *ac, double *summ, double *phi, hipStream_t st)
{
    const int N = d.N;
    const int64_t ncs = d.C - 1;  // chunks with a successor
    if (d.tv) {
        constexpr int S = SummarySlots<W>::value;
        const int nl = (N + 1 + S - 1) / S;
        if (d.a_vec)
            FILT_LAUNCH("fwd_summary", (k_fwd_summary<W, S, true, FIR, true, true, io_t>),
                        dim3(blocks_for(d.B * ncs * nl)), dim3(block_for(d.B * ncs * nl)), 0, st, d, x, xi, bc, ac,
                        (int64_t)0, ncs, 0, N + 1, summ, phi);
        else
            FILT_LAUNCH("fwd_summary", (k_fwd_summary<W, S, true, FIR, true, false, io_t>),
                        dim3(blocks_for(d.B * ncs * nl)), dim3(block_for(d.B * ncs * nl)), 0, st, d, x, xi, bc, ac,
                        (int64_t)0, ncs, 0, N + 1, summ, phi);
    } else {
        FILT_LAUNCH("fwd_summary", (k_fwd_summary<W, 1, false, FIR, true, false, io_t>),
                    dim3(blocks_for(d.B * ncs)), dim3(block_for(d.B * ncs)), 0, st, d, x, xi, bc, ac,
                    (int64_t)0, ncs, N, 1, summ, phi);
        FILT_LAUNCH("fwd_summary_phi", (k_fwd_summary<W, 1, false, false, false, false, io_t>),
                    dim3(blocks_for(d.B * N)), dim3(block_for(d.B * N)), 0, st, d, x, xi, bc, ac, (int64_t)0,
                    (int64_t)1, 0, N, summ, phi);
    }
    return check_launch("forward summary");
}

template <int W, typename io_t>
filt_status fwd_summary_w(const Dims &d, const io_t *x, const io_t *xi, const io_t *bc,
                          const io_t *ac, double *summ, double *phi, hipStream_t st)
{
    if (d.M > 0)
        return fwd_summary_fir<W, true, io_t>(d, x, xi, bc, ac, summ, phi, st);
    return fwd_summary_fir<W, false, io_t>(d, x, xi, bc, ac, summ, phi, st);
}

template <int W, bool FIR, typename io_t>
filt_status bwd_summary_fir(const Dims &d, const io_t *gy, const io_t *bc, const io_t *ac,
                            double *summ, double *phi, hipStream_t st)
{
    const int N = d.N;
    const int64_t ncs = d.C - 1;  // chunks 1..C-1 pass a state to an earlier chunk
    if (d.tv) {
        constexpr int S = SummarySlots<W>::value;
        const int nl = (N + 1 + S - 1) / S;
        if (d.a_vec)
            FILT_LAUNCH("bwd_summary", (k_bwd_summary<W, S, true, FIR, true, true, io_t>),
                        dim3(blocks_for(d.B * ncs * nl)), dim3(block_for(d.B * ncs * nl)), 0, st, d, gy, bc, ac,
                        (int64_t)1, ncs, 0, N + 1, summ, phi);
        else
            FILT_LAUNCH("bwd_summary", (k_bwd_summary<W, S, true, FIR, true, false, io_t>),
                        dim3(blocks_for(d.B * ncs * nl)), dim3(block_for(d.B * ncs * nl)), 0, st, d, gy, bc, ac,
                        (int64_t)1, ncs, 0, N + 1, summ, phi);
    } else {
        FILT_LAUNCH("bwd_summary", (k_bwd_summary<W, 1, false, FIR, true, false, io_t>),
                    dim3(blocks_for(d.B * ncs)), dim3(block_for(d.B * ncs)), 0, st, d, gy, bc, ac, (int64_t)1,
                    ncs, N, 1, summ, phi);
        if (N > 0)
            FILT_LAUNCH("bwd_summary_phi", (k_bwd_summary<W, 1, false, FIR, false, false, io_t>),
                        dim3(blocks_for(d.B * N)), dim3(block_for(d.B * N)), 0, st, d, gy, bc, ac,
                        (int64_t)0, (int64_t)1, 0, N, summ, phi);
    }
    return check_launch("backward summary");
}

template <int W, typename io_t>
filt_status bwd_summary_w(const Dims &d, const io_t *gy, const io_t *bc, const io_t *ac,
                          double *summ, double *phi, hipStream_t st)
{
    if (d.M > 0)
        return bwd_summary_fir<W, true, io_t>(d, gy, bc, ac, summ, phi, st);
    return bwd_summary_fir<W, false, io_t>(d, gy, bc, ac, summ, phi, st);
}

}  // namespace filt_detail
