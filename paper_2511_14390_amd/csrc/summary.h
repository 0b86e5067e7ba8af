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
// Per-sample coefficients: every chunk needs N + 1 solves.  Orders up to 8:
// each lane runs S of them side by side, so one coefficient row fetched (and
// converted) per step feeds S recursions; nl = ceil((N + 1) / S) adjacent
// lanes cover one chunk, rows fetched a few steps ahead of their use.
// Orders 9..16: one 16-lane DPP row per chunk for the N homogeneous solves
// and a lane quad for the particular one (the row solves below).
// Time-invariant coefficients: one particular solve per chunk, and the N
// homogeneous solves once per channel (Phi is the same for every chunk).
//
// Register histories live in W registers addressed modulo W; the time loop
// is unrolled by W so every index is a compile-time constant.
#pragma once

#include "common.h"

namespace filt_detail {

// ---------------------------------------------------------------- forward

// S forward recursions over [t0, t0 + L).  h[q][t mod W] = y_q[t]; hx[t mod
// W] = x[t].  Slot q is driven by wgt[q] * (b * x)[t] (XIN) and its history.
// KT bounds the taps the loops visit (a_1..a_KT, b_0..b_KT): the bucket width
// W by default, the problem's max(N, M) for time-invariant coefficients of a
// narrower order than the bucket (the other taps are zero).
template <int W, int S, bool TV, bool FIR, bool XIN, bool AV, typename io_t, int KT = W>
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
                        if (k <= KT)
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
                    if (k > KT)
                        continue;
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
template <int W, int S, bool TV, bool FIR, bool XIN, bool AV, typename io_t, int KT = W>
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
    const Cursor<io_t> acur = row_cursor(d, ac, b, t0, d.N);
    const Cursor<io_t> bcur = row_cursor(d, bc, b, t0, d.has_b ? d.M + 1 : 0);
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
    fwd_solves<W, S, TV, FIR, XIN, AV, io_t, KT>(d, t0, xc, acur, bcur, h, hx, wgt, la, lb);
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

template <int W, int S, bool TV, bool FIR, bool XIN, bool AV, typename io_t, int KT = W>
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
    fwd_summary_item<W, S, TV, FIR, XIN, AV, io_t, KT>(d, x, xi, bc, ac, j_first, nj, summ, phi,
                                                       b, c_first + cc, r);
}

// ---------------------------------------------------------------- backward

// S adjoint recursions over [t0, t0 + L) in decreasing time, transposed
// (scatter) form.  Before processing time t, slot q's adjoint state s_k
// (the part of ybar[t-1+k] still to be added) is in ss[q][(k - t) mod W] and
// its FIR adjoint state r_k (the part of gx[t-1+k] still to be added) in
// rs[q][(k - t) mod W].  Per step:
//   ybar = wgt[q] gy[t] + s_1,  s_k <- s_{k+1} - a_k[t] ybar,
//   r_k <- r_{k+1} + b_k[t] ybar.
// KT bounds the taps as in fwd_solves (s_k, r_k for k > KT stay zero).
template <int W, int S, bool TV, bool FIR, bool GIN, bool AV, typename io_t, int KT = W>
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
                ss[q][(1 - s) & m] = KT < W ? 0.0 : -ca[W] * yb;
#pragma unroll
                for (int k = 1; k < W; ++k)
                    if (k <= KT)
                        ss[q][(k + 1 - s) & m] -= ca[k] * yb;
                if constexpr (FIR) {
                    rs[q][(1 - s) & m] = 0.0;
#pragma unroll
                    for (int k = 1; k < W; ++k)
                        if (k <= KT)
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
template <int W, int S, bool TV, bool FIR, bool GIN, bool AV, typename io_t, int KT = W>
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
    const Cursor<io_t> acur = row_cursor(d, ac, b, t0, d.N);
    const Cursor<io_t> bcur = row_cursor(d, bc, b, t0, d.has_b ? d.M + 1 : 0);
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
    bwd_solves<W, S, TV, FIR, GIN, AV, io_t, KT>(d, t0, gc, acur, bcur, ss, rs, wgt, la, lb);
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

template <int W, int S, bool TV, bool FIR, bool GIN, bool AV, typename io_t, int KT = W>
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
    bwd_summary_item<W, S, TV, FIR, GIN, AV, io_t, KT>(d, gy, bc, ac, j_first, nj, summ, phi, b,
                                                       c_first + cc, r);
}

// ---------------------------------------------------------------- row solves
//
// Per-sample coefficients of order 9..16 (the W = 16 bucket): the N
// homogeneous solves of a chunk (the columns of Phi_c) run on one 16-lane
// DPP row, lane j solving column j.  Lane j also loads and converts the one
// coefficient -a_{j+1}[t] of step t; the other lanes read it through a
// row_newbcast broadcast folded into the FMA (v_fmac_f64 takes a DPP source
// on CDNA3/4), so a lane converts one coefficient per step instead of a whole
// row and every FP64 instruction of the step is an FMA.  The particular solve
// (zero state, real input) has a coefficient row of its own per lane and runs
// as in fwd_summary_item / bwd_summary_item, on lanes of the same launch.
//
// The broadcast source is written by a VALU instruction shortly before each
// step's FMAs; DPP needs 2 wait states after such a write (5 after a VALU
// write of EXEC), hence the s_nop 4 that opens each step.  All 16 lanes of a
// row stay active for the whole chunk (lanes j >= N carry zero coefficients).

#define FILT_ROW_FMAC(lane, acc, src, mul)                                                         \
    "v_fmac_f64_dpp %" #acc ", %" #src ", %" #mul " row_newbcast:" #lane                          \
    " row_mask:0xf bank_mask:0xf\n"

// One forward step of a row: returns sum_k c_k * h[s - k] (k = 1..16) where
// c_k sits in lane k - 1 of the row and h[s - k] = h[(s - k) & 15].
template <int s>
__device__ __forceinline__ double row_fwd_step(double c, const double (&h)[16])
{
    double acc = 0.0;
    asm("s_nop 4\n"
        FILT_ROW_FMAC(15, 0, 1, 2) FILT_ROW_FMAC(14, 0, 1, 3) FILT_ROW_FMAC(13, 0, 1, 4)
        FILT_ROW_FMAC(12, 0, 1, 5) FILT_ROW_FMAC(11, 0, 1, 6) FILT_ROW_FMAC(10, 0, 1, 7)
        FILT_ROW_FMAC(9, 0, 1, 8) FILT_ROW_FMAC(8, 0, 1, 9) FILT_ROW_FMAC(7, 0, 1, 10)
        FILT_ROW_FMAC(6, 0, 1, 11) FILT_ROW_FMAC(5, 0, 1, 12) FILT_ROW_FMAC(4, 0, 1, 13)
        FILT_ROW_FMAC(3, 0, 1, 14) FILT_ROW_FMAC(2, 0, 1, 15) FILT_ROW_FMAC(1, 0, 1, 16)
        FILT_ROW_FMAC(0, 0, 1, 17)
        : "+v"(acc)
        : "v"(c), "v"(h[(s + 0) & 15]), "v"(h[(s + 1) & 15]), "v"(h[(s + 2) & 15]),
          "v"(h[(s + 3) & 15]), "v"(h[(s + 4) & 15]), "v"(h[(s + 5) & 15]),
          "v"(h[(s + 6) & 15]), "v"(h[(s + 7) & 15]), "v"(h[(s + 8) & 15]),
          "v"(h[(s + 9) & 15]), "v"(h[(s + 10) & 15]), "v"(h[(s + 11) & 15]),
          "v"(h[(s + 12) & 15]), "v"(h[(s + 13) & 15]), "v"(h[(s + 14) & 15]),
          "v"(h[(s + 15) & 15]));
    return acc;
}

// One adjoint step of a row (transposed form, as in bwd_solves with no
// input): ybar = s_1; s_k <- s_{k+1} + c_k ybar (s_17 = 0), with s_k in
// ss[(k - s) & 15] before the step and c_k in lane k - 1.
template <int s>
__device__ __forceinline__ void row_bwd_step(double c, double (&ss)[16])
{
    const double yb = ss[(1 - s) & 15];
    double nw = 0.0;
    asm("s_nop 4\n"
        FILT_ROW_FMAC(15, 0, 16, 17) FILT_ROW_FMAC(0, 1, 16, 17) FILT_ROW_FMAC(1, 2, 16, 17)
        FILT_ROW_FMAC(2, 3, 16, 17) FILT_ROW_FMAC(3, 4, 16, 17) FILT_ROW_FMAC(4, 5, 16, 17)
        FILT_ROW_FMAC(5, 6, 16, 17) FILT_ROW_FMAC(6, 7, 16, 17) FILT_ROW_FMAC(7, 8, 16, 17)
        FILT_ROW_FMAC(8, 9, 16, 17) FILT_ROW_FMAC(9, 10, 16, 17) FILT_ROW_FMAC(10, 11, 16, 17)
        FILT_ROW_FMAC(11, 12, 16, 17) FILT_ROW_FMAC(12, 13, 16, 17)
        FILT_ROW_FMAC(13, 14, 16, 17) FILT_ROW_FMAC(14, 15, 16, 17)
        : "+v"(nw), "+v"(ss[(2 - s) & 15]), "+v"(ss[(3 - s) & 15]), "+v"(ss[(4 - s) & 15]),
          "+v"(ss[(5 - s) & 15]), "+v"(ss[(6 - s) & 15]), "+v"(ss[(7 - s) & 15]),
          "+v"(ss[(8 - s) & 15]), "+v"(ss[(9 - s) & 15]), "+v"(ss[(10 - s) & 15]),
          "+v"(ss[(11 - s) & 15]), "+v"(ss[(12 - s) & 15]), "+v"(ss[(13 - s) & 15]),
          "+v"(ss[(14 - s) & 15]), "+v"(ss[(15 - s) & 15]), "+v"(ss[(16 - s) & 15])
        : "v"(c), "v"(yb));
    ss[(1 - s) & 15] = nw;
}

#undef FILT_ROW_FMAC

// Coefficient stream of one row lane: -a_{j+1}[t] for the chunk's steps in
// increasing (forward) or decreasing (adjoint) time, 16 steps ahead of use.
// Lanes j >= N read tap N - 1 and zero it.  Chunks with a successor (and, in
// the adjoint, chunks 1..C-1) are whole, so every step read lies in the chunk
// and the reads stop at its end.
template <typename io_t, bool FULL>
struct RowCoef {
    RowWalk<io_t> w; // this lane's tap: at(r) is its value's address at step r
    bool live;       // j < N

    __device__ __forceinline__ const io_t *at(int r) const { return w.at(r); }

    __device__ __forceinline__ double cvt(io_t raw) const
    {
        if constexpr (!FULL)
            raw = live ? raw : io_t(0);
        return -(double)raw;
    }
};

template <typename io_t, bool FULL>
__device__ __forceinline__ RowCoef<io_t, FULL> row_coef(const Dims &d, const io_t *ac, int64_t b,
                                                        int64_t c, int j)
{
    RowCoef<io_t, FULL> r;
    const int64_t t0 = c * d.L;
    const int jj = j < d.N ? j : d.N - 1;
    r.w = row_walk(d, ac, b, t0, d.N);
    r.w.p += jj;
    r.live = j < d.N;
    return r;
}

// Column j of Phi_c (unit state y(t0 - 1 - j) = 1, no input) on a row lane.
template <bool FULL, typename io_t>
__device__ __forceinline__ void fwd_row_item(const Dims &d, const io_t *__restrict__ ac,
                                             double *__restrict__ summ, int64_t b, int64_t c,
                                             int j)
{
    const RowCoef<io_t, FULL> rc = row_coef<io_t, FULL>(d, ac, b, c, j);
    double h[16];
#pragma unroll
    for (int e = 0; e < 16; ++e)
        h[e] = (rc.live && e == ((-1 - j) & 15)) ? 1.0 : 0.0;
    io_t buf[16];
#pragma unroll
    for (int s = 0; s < 16; ++s)
        buf[s] = *rc.at(s);
    for (int rel = 0; rel < d.L; rel += 16) {
        static_for<16>([&](auto I) {
            constexpr int s = decltype(I)::value;
            const double cf = rc.cvt(buf[s]);
            // step rel + 16 + s; the last block re-reads the chunk's last row
            // (unconditional loads keep the ring free of merges and waits)
            buf[s] = *rc.at(min(rel + 16 + s, (int)d.L - 1));
            h[s] = row_fwd_step<s>(cf, h);
            __builtin_amdgcn_sched_barrier(0);
        });
    }
    // the chunk length is a multiple of 16: y(t_end - 1 - i) sits in h[15 - i]
    if (rc.live) {
        double *o = summ + (b * d.C + c) * ((int64_t)d.N * d.N + d.N) + j;
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (i < d.N)
                o[(int64_t)i * d.N] = h[15 - i];
    }
}

// Column j of the adjoint chunk map (unit state s_{j+1} = 1, no input).
template <bool FULL, typename io_t>
__device__ __forceinline__ void bwd_row_item(const Dims &d, const io_t *__restrict__ ac,
                                             double *__restrict__ summ, int64_t b, int64_t c,
                                             int j)
{
    const RowCoef<io_t, FULL> rc = row_coef<io_t, FULL>(d, ac, b, c, j);
    double *o = summ + (b * d.C + c) * ((int64_t)(d.N + 1) * d.N) + j;
    if (c * d.L + d.L > d.T) {
        // a last chunk cut short by the signal's end: no adjoint state enters
        // it from above, so its map only ever multiplies zero; store zero
        // rather than reading coefficients past T
        if (rc.live)
            for (int i = 0; i < d.N; ++i)
                o[(int64_t)i * d.N] = 0.0;
        return;
    }
    // s_k in ss[(k - s) & 15] before relative step s; the first step is
    // s = L - 1 = 15 (mod 16)
    double ss[16];
#pragma unroll
    for (int e = 0; e < 16; ++e)
        ss[e] = (rc.live && e == ((j + 2) & 15)) ? 1.0 : 0.0;
    io_t buf[16];
#pragma unroll
    for (int s = 0; s < 16; ++s)
        buf[s] = *rc.at((int)d.L - 16 + s);
    for (int rel = d.L - 16; rel >= 0; rel -= 16) {
        static_for<16>([&](auto I) {
            constexpr int s = 15 - decltype(I)::value;
            const double cf = rc.cvt(buf[s]);
            // step rel - 16 + s; the last block re-reads the chunk's first row
            buf[s] = *rc.at(max(rel - 16 + s, 0));
            row_bwd_step<s>(cf, ss);
            __builtin_amdgcn_sched_barrier(0);
        });
    }
    // after the chunk's first step s_k sits in ss[(k + 1) & 15]
    if (rc.live) {
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (i < d.N)
                o[(int64_t)i * d.N] = ss[(i + 2) & 15];
    }
}

// Particular solves on quads.  The zero-state solve driven by the input (the
// s_c part of a summary) is one recursion per chunk; it runs on 4 adjacent
// lanes, lane q owning taps k = 4q + 1 .. 4q + 4 (one 16-byte load of the
// coefficient row per step).  Forward: lane q keeps w[i] = y[t - 4q - 1 - i],
// forms its part of sum_k a_k[t] y[t - k], and a quad butterfly adds the four
// parts (every lane ends with the same sum: FP64 addition is commutative);
// the window then moves by one sample, lane q taking lane q - 1's oldest.
// Adjoint (transposed form): lane q keeps st[i] = s_{4q+1+i}; ybar = g + s_1
// comes from lane 0 and s_k <- s_{k+1} - a_k ybar shifts within the lane,
// s_{4q+5} arriving from lane q + 1 (zero past the last lane).

// Workgroups of the row summaries: kRowGroupChunks items, waves 0-3 their
// rows, wave 4 their particular solves.
constexpr int kRowGroupChunks = 16;
constexpr int kRowGroupThreads = 16 * kRowGroupChunks + 64;

constexpr int kQuadPrefetch = 4;  // steps in flight (chunk lengths are multiples of 32)

// Forward summaries of one workgroup's items, reading the coefficient rows
// once.  The row lanes park every raw coefficient they consume in LDS (hand:
// two buffers of kHandSteps steps x 16 items x 16 taps) and the quad wave
// takes its taps from there, kHandSteps steps behind the rows, instead of
// loading the rows from HBM a second time.  Per 16-step block each wave
// passes two barriers (rows: write buffer 0, barrier, write buffer 1,
// barrier; quad: read buffer 1 of the block before, barrier, read buffer 0,
// barrier), L / 16 + 1 blocks in all, so L must be the same for every item
// of the workgroup.  The roles are wave-uniform; (b, c) is the item of this
// lane's row (threads below 16 kRowGroupChunks) or quad, and a lane whose
// item does not exist (act false) still runs every barrier, computing on a
// valid chunk and storing nothing.  Every chunk summarised here is whole.
constexpr int kHandSteps = 8;

template <bool FULL, bool HASB, typename io_t>
__device__ __forceinline__ void fwd_rows_group(const Dims &d, const io_t *__restrict__ x,
                                               const io_t *__restrict__ bc,
                                               const io_t *__restrict__ ac,
                                               double *__restrict__ summ, int64_t b,
                                               int64_t c, bool act,
                                               io_t (*hand)[kHandSteps][16][16])
{
    using H0 = std::integral_constant<int, 0>;
    using H1 = std::integral_constant<int, 1>;
    const int t = threadIdx.x;
    const int nblk = (int)(d.L / 16);
    const int N = d.N;
    if (t < 16 * kRowGroupChunks) {
        const int row = t >> 4, j = t & 15;
        const RowCoef<io_t, FULL> rc = row_coef<io_t, FULL>(d, ac, b, c, j);
        double h[16];
#pragma unroll
        for (int e = 0; e < 16; ++e)
            h[e] = (rc.live && e == ((-1 - j) & 15)) ? 1.0 : 0.0;
        io_t buf[16];
#pragma unroll
        for (int s = 0; s < 16; ++s)
            buf[s] = *rc.at(s);
        // steps 8 HH .. 8 HH + 7 of the block at rel; raw values to hand[HH]
        auto half = [&](auto HH, int rel) {
            static_for<kHandSteps>([&](auto I) {
                constexpr int s = decltype(HH)::value * kHandSteps + decltype(I)::value;
                hand[decltype(HH)::value][decltype(I)::value][row][j] = buf[s];
                const double cf = rc.cvt(buf[s]);
                buf[s] = *rc.at(min(rel + 16 + s, (int)d.L - 1));
                h[s] = row_fwd_step<s>(cf, h);
                __builtin_amdgcn_sched_barrier(0);
            });
        };
        for (int kb = 0; kb <= nblk; ++kb) {
            if (kb < nblk)
                half(H0{}, 16 * kb);
            __syncthreads();
            if (kb < nblk)
                half(H1{}, 16 * kb);
            __syncthreads();
        }
        if (act && rc.live) {
            double *o = summ + (b * d.C + c) * ((int64_t)N * N + N) + j;
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (i < N)
                    o[(int64_t)i * N] = h[15 - i];
        }
        return;
    }
    const int u = t - 16 * kRowGroupChunks;
    const int k = u >> 2, q = u & 3;
    const bool tb = d.layout == FILT_LAYOUT_TB;
    const int64_t e0 = tb ? c * d.L * d.B + b : b * d.T + c * d.L;
    const int64_t es = tb ? d.B : 1;
    const io_t *xp = x + e0;
    // order-0 FIR part: one tap per row (b_0)
    const RowWalk<io_t> bw = row_walk(d, HASB ? bc : x, b, c * d.L, HASB ? 1 : 0);
    io_t xb[16], gb[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        xb[s] = xp[s * es];
        if constexpr (HASB)
            gb[s] = *bw.at(s);
    }
    double w[4] = {0.0, 0.0, 0.0, 0.0};  // w[i] = y[t - 4q - 1 - i]
    // steps 8 HH .. 8 HH + 7 of the block at rel, taps from hand[HH]
    auto qhalf = [&](auto HH, int rel) {
        static_for<kHandSteps>([&](auto I) {
            constexpr int s = decltype(HH)::value * kHandSteps + decltype(I)::value;
            const io_t *hp = &hand[decltype(HH)::value][decltype(I)::value][k][4 * q];
            io_t a4[4];
            if constexpr (sizeof(io_t) == 4) {
                const float4 f = *reinterpret_cast<const float4 *>(hp);
                a4[0] = f.x;
                a4[1] = f.y;
                a4[2] = f.z;
                a4[3] = f.w;
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    a4[i] = hp[i];
            }
            const double xv = (double)xb[s];
            const double gv = HASB ? (double)gb[s] : 1.0;
            const int nx = min(rel + 16 + s, (int)d.L - 1);
            xb[s] = xp[nx * es];
            if constexpr (HASB)
                gb[s] = *bw.at(nx);
            double p = 0.0;
#pragma unroll
            for (int i = 3; i >= 0; --i)
                p = __builtin_fma((FULL || 4 * q + i < N) ? -(double)a4[i] : 0.0, w[i], p);
            double tot = p + quad_dpp<kQuadXor1>(p);
            tot = tot + quad_dpp<kQuadXor2>(tot);
            const double y = HASB ? __builtin_fma(gv, xv, tot) : xv + tot;
            const double prev = quad_dpp<kQuadFromPrev>(w[3]);
            w[3] = w[2];
            w[2] = w[1];
            w[1] = w[0];
            w[0] = q == 0 ? y : prev;
        });
    };
    for (int kb = 0; kb <= nblk; ++kb) {
        if (kb > 0)
            qhalf(H1{}, 16 * (kb - 1));
        __syncthreads();
        if (kb < nblk)
            qhalf(H0{}, 16 * kb);
        __syncthreads();
    }
    if (act) {
        double *o = summ + (b * d.C + c) * ((int64_t)N * N + N) + (int64_t)N * N;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (4 * q + i < N)
                o[4 * q + i] = w[i];
    }
}

// Particular part of the adjoint map of chunk c (zero state at its top, the
// real gy).  CLAMP: a last chunk cut short by the signal's end; its steps
// past T read clamped rows and a zero gy, leaving the state zero.
template <bool AV, bool CLAMP, typename io_t>
__device__ __forceinline__ void bwd_part_quad(const Dims &d, const io_t *__restrict__ gy,
                                              const io_t *__restrict__ ac,
                                              double *__restrict__ summ, int64_t b, int64_t c,
                                              int q)
{
    constexpr int P = kQuadPrefetch;
    const int N = d.N;
    const bool tb = d.layout == FILT_LAYOUT_TB;
    const int64_t e0 = tb ? c * d.L * d.B + b : b * d.T + c * d.L;
    const int64_t es = tb ? d.B : 1;
    const int last = CLAMP ? (int)min<int64_t>(d.T - 1 - c * d.L, d.L - 1) : d.L - 1;
    const io_t *gp = gy + e0;
    const RowWalk<io_t> aw = row_walk(d, ac, b, c * d.L, N);
    auto fetch = [&](int rel, QuadRaw<io_t> &r) {
        const int rc = CLAMP ? min(rel, last) : rel;
        quad_taps<AV>(aw.at(rc), q, N, r.a);
        const io_t g = gp[rc * es];
        r.s = (!CLAMP || rel <= last) ? g : io_t(0);
    };
    QuadRaw<io_t> buf[P];
    static_for<P>([&](auto I) {
        fetch(d.L - P + decltype(I)::value, buf[decltype(I)::value]);
    });
    double st[4] = {0.0, 0.0, 0.0, 0.0};
    for (int rel = d.L - P; rel >= 0; rel -= P) {
        static_for<P>([&](auto I) {
            constexpr int s = P - 1 - decltype(I)::value;
            const QuadRaw<io_t> r = buf[s];
            fetch(max(rel - P + s, 0), buf[s]);  // unconditional, clamped into the chunk
            const double yb = (double)r.s + quad_dpp<kQuadLane0>(st[0]);
            const double nx = quad_dpp<kQuadFromNext>(st[0]);
            st[0] = __builtin_fma(quad_coef<AV>(r.a, 0, q, N), yb, st[1]);
            st[1] = __builtin_fma(quad_coef<AV>(r.a, 1, q, N), yb, st[2]);
            st[2] = __builtin_fma(quad_coef<AV>(r.a, 2, q, N), yb, st[3]);
            st[3] = __builtin_fma(quad_coef<AV>(r.a, 3, q, N), yb, q == 3 ? 0.0 : nx);
        });
    }
    double *o = summ + (b * d.C + c) * ((int64_t)(N + 1) * N) + (int64_t)N * N;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (4 * q + i < N)
            o[4 * q + i] = st[i];
}

// Workgroups of kRowGroupThreads threads cover kRowGroupChunks consecutive
// items (b, chunk): waves 0-3 hold one 16-lane row per item, wave 4 the
// items' particular solves (a quad each, fed through LDS in the forward; with
// an FIR part, one lane each).  In the adjoint the quads load the coefficient
// rows themselves (a last chunk cut short needs clamped rows), and sharing
// the workgroup with the rows keeps part of that second read in cache.

template <bool FIR, bool AV, bool FULL, typename io_t>
__global__ void __launch_bounds__(kRowGroupThreads, FIR ? 1 : 5)
k_fwd_summary_rows(Dims d, const io_t *__restrict__ x, const io_t *__restrict__ xi,
                   const io_t *__restrict__ bc, const io_t *__restrict__ ac, int64_t ncs,
                   double *__restrict__ summ)
{
    const int64_t n = d.B * ncs;
    const int64_t first = (int64_t)blockIdx.x * kRowGroupChunks;
    const int t = threadIdx.x;
    if constexpr (!FIR) {
        __shared__ io_t hand[2][kHandSteps][16][16];
        // this lane's item: its row's, or its quad's
        const int k = t >= 16 * kRowGroupChunks ? (t - 16 * kRowGroupChunks) >> 2 : t >> 4;
        const bool act = first + k < n;
        int64_t b = 0, cc = 0;
        int r;
        if (act)
            decode_lanes(d, first + k, ncs, 1, b, cc, r);
        if (d.has_b)
            fwd_rows_group<FULL, true>(d, x, bc, ac, summ, b, cc, act, hand);
        else
            fwd_rows_group<FULL, false>(d, x, bc, ac, summ, b, cc, act, hand);
        return;
    }
    // with an FIR part: one lane per chunk for the particular solve, rows
    // and particular lanes each reading the coefficient rows
    int64_t b, cc;
    int r;
    if (t >= 16 * kRowGroupChunks) {
        const int u = t - 16 * kRowGroupChunks;
        if (u >= kRowGroupChunks || first + u >= n)
            return;
        decode_lanes(d, first + u, ncs, 1, b, cc, r);
        fwd_summary_item<16, 1, true, FIR, true, AV>(d, x, xi, bc, ac, d.N, 1, summ, nullptr, b,
                                                     cc, 0);
        return;
    }
    if (first + (t >> 4) >= n)  // whole rows only
        return;
    decode_lanes(d, first + (t >> 4), ncs, 1, b, cc, r);
    fwd_row_item<FULL>(d, ac, summ, b, cc, t & 15);
}

template <bool AV, bool FULL, typename io_t>
__global__ void __launch_bounds__(kRowGroupThreads, 5)
k_bwd_summary_rows(Dims d, const io_t *__restrict__ gy, const io_t *__restrict__ ac, int64_t ncs,
                   double *__restrict__ summ)
{
    const int64_t n = d.B * ncs;
    const int64_t first = (int64_t)blockIdx.x * kRowGroupChunks;
    const int t = threadIdx.x;
    int64_t b, cc;
    int r;
    if (t >= 16 * kRowGroupChunks) {
        const int u = t - 16 * kRowGroupChunks;
        if (first + (u >> 2) >= n)
            return;
        decode_lanes(d, first + (u >> 2), ncs, 1, b, cc, r);
        if ((cc + 2) * d.L > d.T)
            bwd_part_quad<AV, true>(d, gy, ac, summ, b, cc + 1, u & 3);
        else
            bwd_part_quad<AV, false>(d, gy, ac, summ, b, cc + 1, u & 3);
        return;
    }
    if (first + (t >> 4) >= n)
        return;
    decode_lanes(d, first + (t >> 4), ncs, 1, b, cc, r);
    bwd_row_item<FULL>(d, ac, summ, b, cc + 1, t & 15);
}

// ---------------------------------------------------------------- launch

template <int W, bool FIR, typename io_t>
filt_status fwd_summary_fir(const Dims &d, const io_t *x, const io_t *xi, const io_t *bc,
                            const io_t *ac, double *summ, double *phi, hipStream_t st)
{
    const int N = d.N;
    const int64_t ncs = d.C - 1;  // chunks with a successor
    if constexpr (W == 16) {
        if (d.tv) {
            const unsigned gr = (unsigned)((d.B * ncs + kRowGroupChunks - 1) / kRowGroupChunks);
#define FILT_ROWS(AV, FULL)                                                                        \
    FILT_LAUNCH("fwd_summary", (k_fwd_summary_rows<FIR, AV, FULL, io_t>), dim3(gr),               \
                dim3(kRowGroupThreads), 0, st, d, x, xi, bc, ac, ncs, summ)
            if (d.a_vec) {
                if (N == 16)
                    FILT_ROWS(true, true);
                else
                    FILT_ROWS(true, false);
            } else {
                FILT_ROWS(false, false);
            }
#undef FILT_ROWS
            return check_launch("forward summary");
        }
    }
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
        lti_tap_bound<W, FIR, io_t, double>(d, [&](auto kt) {
            constexpr int KT = decltype(kt)::value;
            FILT_LAUNCH("fwd_summary", (k_fwd_summary<W, 1, false, FIR, true, false, io_t, KT>),
                        dim3(blocks_for(d.B * ncs)), dim3(block_for(d.B * ncs)), 0, st, d, x, xi,
                        bc, ac, (int64_t)0, ncs, N, 1, summ, phi);
        });
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
    if constexpr (W == 16 && !FIR) {
        if (d.tv) {
            const unsigned gr = (unsigned)((d.B * ncs + kRowGroupChunks - 1) / kRowGroupChunks);
#define FILT_ROWS(AV, FULL)                                                                        \
    FILT_LAUNCH("bwd_summary", (k_bwd_summary_rows<AV, FULL, io_t>), dim3(gr),                    \
                dim3(kRowGroupThreads), 0, st, d, gy, ac, ncs, summ)
            if (d.a_vec) {
                if (N == 16)
                    FILT_ROWS(true, true);
                else
                    FILT_ROWS(true, false);
            } else {
                FILT_ROWS(false, false);
            }
#undef FILT_ROWS
            return check_launch("backward summary");
        }
    }
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
        lti_tap_bound<W, FIR, io_t, double>(d, [&](auto kt) {
            constexpr int KT = decltype(kt)::value;
            FILT_LAUNCH("bwd_summary", (k_bwd_summary<W, 1, false, FIR, true, false, io_t, KT>),
                        dim3(blocks_for(d.B * ncs)), dim3(block_for(d.B * ncs)), 0, st, d, gy, bc,
                        ac, (int64_t)1, ncs, N, 1, summ, phi);
        });
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
