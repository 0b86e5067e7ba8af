// chunk.h -- per-chunk forward / backward kernels (internal; included by
// the chunk_w*.hip translation units only).
#pragma once

#include "common.h"

namespace filt_detail {

// ---------------------------------------------------------------- forward

// Runs the forward recursion over [t0, t0 + L).  hy[t mod W] holds y[t] for
// the last W times, hx[t mod W] holds x[t].  PART: driven by x (else zero
// input, the homogeneous solve).  t0 and L are multiples of W.
template <int W, bool TV, bool PART, bool WRITE, typename io_t, typename acc_t>
__device__ __forceinline__ void fwd_chunk(const Dims &d, int64_t b, int64_t t0, const io_t *x,
                                          const io_t *bc, const io_t *ac, acc_t (&hy)[W],
                                          acc_t (&hx)[W], const acc_t (&la)[W + 1],
                                          const acc_t (&lb)[W], io_t *y)
{
    constexpr int m = W - 1;
    const int64_t tend = t0 + d.L;
    for (int64_t tb = t0; tb < tend; tb += W) {
#pragma unroll
        for (int s = 0; s < W; ++s) {
            const int64_t t = tb + s;
            acc_t ca[W + 1], cb[W];
            if (TV) {
                ld_coef<W>(d, bc, ac, b, t, ca, cb);
            } else {
#pragma unroll
                for (int k = 0; k <= W; ++k)
                    ca[k] = la[k];
#pragma unroll
                for (int k = 0; k < W; ++k)
                    cb[k] = lb[k];
            }
            acc_t acc = acc_t(0);
            if (PART) {
                hx[s & m] = t < d.T ? (acc_t)x[sig_at(d, b, t)] : acc_t(0);
#pragma unroll
                for (int k = W - 1; k >= 0; --k)
                    acc += cb[k] * hx[(s - k) & m];
            }
            // oldest taps first so the newest output is the last dependency
#pragma unroll
            for (int k = W; k >= 1; --k)
                acc -= ca[k] * hy[(s - k) & m];
            hy[s & m] = acc;
            if (WRITE && t < d.T)
                y[sig_at(d, b, t)] = (io_t)acc;
        }
    }
}

template <int W, typename io_t, typename acc_t>
__device__ __forceinline__ void lti_coef(const Dims &d, const io_t *bc, const io_t *ac, int64_t b,
                                         acc_t (&la)[W + 1], acc_t (&lb)[W])
{
    // time-invariant rows do not depend on t; t = 0 is always in range here
    ld_coef<W>(d, bc, ac, b, 0, la, lb);
}

// Phase 1 (forward), always in FP64: the companion-form transition of a chunk
// has entries far above 1 when poles cluster near the unit circle, so an FP32
// Phi would lose the digits the carry needs.  Items (b, c, j): j < N solves chunk c from the unit
// state e_j (column j of Phi_c), j == N solves it from zero state with the
// real input (s_c).  summ[(b*C + c)*SS + i*N + j] = Phi_c[i][j],
// summ[(b*C + c)*SS + N*N + i] = s_c[i]; state index i = 0..N-1 is y(t-1-i).
// For time-invariant filters Phi is written to phi[b*N*N + ...] (chunk 0 only).
template <int W, bool TV, bool PART, typename io_t, typename acc_t>
__global__ void __launch_bounds__(kThreads)
k_fwd_summary(Dims d, const io_t *__restrict__ x, const io_t *__restrict__ xi,
              const io_t *__restrict__ bc, const io_t *__restrict__ ac, int64_t c_first,
              int64_t ncs, int j_first, int nj, double *__restrict__ summ,
              double *__restrict__ phi)
{
    constexpr int m = W - 1;
    const int64_t total = d.B * ncs * nj;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total)
        return;
    int64_t b, cc, jj;
    decode(d, idx, ncs, b, cc, jj);
    const int64_t c = c_first + cc;
    const int j = j_first + (int)jj;
    const int64_t t0 = c * d.L;
    const int N = d.N;

    acc_t la[W + 1], lb[W];
    if (!TV)
        lti_coef<W>(d, bc, ac, b, la, lb);
    acc_t hy[W], hx[W];
#pragma unroll
    for (int q = 0; q < W; ++q) {
        hy[q] = acc_t(0);
        hx[q] = acc_t(0);
    }
    if (PART) {
#pragma unroll
        for (int k = 1; k < W; ++k)
            hx[(-k) & m] = ld_x<io_t, acc_t>(d, x, xi, b, t0 - k);
    } else {
        // unit state: y(t0 - 1 - j) = 1
#pragma unroll
        for (int q = 0; q < W; ++q)
            hy[q] = (q == ((-(j + 1)) & m)) ? acc_t(1) : acc_t(0);
    }
    fwd_chunk<W, TV, PART, false>(d, b, t0, x, bc, ac, hy, hx, la, lb, (io_t *)nullptr);
    const int64_t SS = (int64_t)N * N + N;
    if (PART) {
        double *o = summ + (b * d.C + c) * SS + (int64_t)N * N;
#pragma unroll
        for (int i = 0; i < W; ++i)
            if (i < N)
                o[i] = (double)hy[(-(i + 1)) & m];
    } else {
        double *o = TV ? summ + (b * d.C + c) * SS : phi + b * (int64_t)N * N;
#pragma unroll
        for (int i = 0; i < W; ++i)
            if (i < N)
                o[(int64_t)i * N + j] = (double)hy[(-(i + 1)) & m];
    }
}

// Phase 3 (forward): rerun each chunk from its exact entering state.
template <int W, bool TV, typename io_t, typename acc_t>
__global__ void __launch_bounds__(kThreads)
k_fwd_apply(Dims d, const io_t *__restrict__ x, const io_t *__restrict__ xi,
            const io_t *__restrict__ bc, const io_t *__restrict__ ac,
            const io_t *__restrict__ yi, const double *__restrict__ hin, io_t *__restrict__ y)
{
    constexpr int m = W - 1;
    const int64_t total = d.B * d.C;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total)
        return;
    int64_t b, c, jj;
    decode(d, idx, d.C, b, c, jj);
    const int64_t t0 = c * d.L;
    acc_t la[W + 1], lb[W];
    if (!TV)
        lti_coef<W>(d, bc, ac, b, la, lb);
    acc_t hy[W], hx[W];
#pragma unroll
    for (int q = 0; q < W; ++q)
        hy[q] = acc_t(0);
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
    hx[0] = acc_t(0);
#pragma unroll
    for (int k = 1; k < W; ++k)
        hx[(-k) & m] = ld_x<io_t, acc_t>(d, x, xi, b, t0 - k);
    fwd_chunk<W, TV, true, true>(d, b, t0, x, bc, ac, hy, hx, la, lb, y);
}

// ---------------------------------------------------------------- backward

// Runs the adjoint over [t0, t0 + L) in decreasing time, in transposed
// (scatter) form.  Before processing time t, the adjoint state
// s_k = -sum_{i>=k} a_i[t+i-k+1]... (the partial sums still owed to ybar[t-1+k])
// lives in ss[(k - t) mod W] and the FIR adjoint state r_k (partial sums owed to
// gx[t-1+k]) in rs[(k - t) mod W].  Per step:
//   ybar = gy[t] + s_1,  gx[t] = b_0 ybar + r_1,
//   s_k <- s_{k+1} - a_k[t] ybar,  r_k <- r_{k+1} + b_k[t] ybar.
// COEF: also form gb_k[t] = ybar x[t-k] and ga_k[t] = -ybar y[t-k]; the
// windows wx[t mod W] = x[t], wy[t mod W] = y[t] slide downward in time.
template <int W, bool TV, bool PART, bool APPLY, bool COEF, typename io_t, typename acc_t>
__device__ __forceinline__ void bwd_chunk(const Dims &d, int64_t b, int64_t t0, const io_t *gy,
                                          const io_t *x, const io_t *xi, const io_t *y,
                                          const io_t *yi, const io_t *bc, const io_t *ac,
                                          acc_t (&ss)[W], acc_t (&rs)[W],
                                          const acc_t (&la)[W + 1], const acc_t (&lb)[W],
                                          io_t *gx, io_t *gb, io_t *ga, double (&sga)[W + 1],
                                          double (&sgb)[W])
{
    constexpr int m = W - 1;
    acc_t wx[W], wy[W];
    const int64_t thi = t0 + d.L - 1;
    if (COEF) {
#pragma unroll
        for (int q = 0; q < W; ++q) {
            wx[q] = acc_t(0);
            wy[q] = acc_t(0);
        }
        if (gb != nullptr) {
#pragma unroll
            for (int k = 0; k < W - 1; ++k)
                wx[(thi - k) & m] = ld_x<io_t, acc_t>(d, x, xi, b, thi - k);
        }
        if (ga != nullptr) {
#pragma unroll
            for (int k = 1; k < W; ++k)
                wy[(thi - k) & m] = ld_y<io_t, acc_t>(d, y, yi, b, thi - k);
        }
    }
    for (int64_t tb = t0 + d.L - W; tb >= t0; tb -= W) {
#pragma unroll
        for (int s = W - 1; s >= 0; --s) {
            const int64_t t = tb + s;
            const bool in = t < d.T;
            acc_t ca[W + 1], cb[W];
            if (TV) {
                ld_coef<W>(d, bc, ac, b, t, ca, cb);
            } else {
#pragma unroll
                for (int k = 0; k <= W; ++k)
                    ca[k] = la[k];
#pragma unroll
                for (int k = 0; k < W; ++k)
                    cb[k] = lb[k];
            }
            const acc_t g = (PART && in) ? (acc_t)gy[sig_at(d, b, t)] : acc_t(0);
            const acc_t yb = g + ss[(1 - s) & m];
            if (APPLY) {
                const acc_t gxv = cb[0] * yb + rs[(1 - s) & m];
                if (gx != nullptr && in)
                    gx[sig_at(d, b, t)] = (io_t)gxv;
            }
            ss[(1 - s) & m] = -ca[W] * yb;
#pragma unroll
            for (int k = 1; k < W; ++k)
                ss[(k + 1 - s) & m] -= ca[k] * yb;
            rs[(1 - s) & m] = acc_t(0);
#pragma unroll
            for (int k = 1; k < W; ++k)
                rs[(k + 1 - s) & m] += cb[k] * yb;
            if (COEF) {
                if (gb != nullptr) {
                    wx[(s + 1) & m] = ld_x<io_t, acc_t>(d, x, xi, b, t - (W - 1));
                    if (TV) {
                        if (in) {
                            io_t *o = gb + row_at(d, b, t, d.M + 1);
#pragma unroll
                            for (int k = 0; k < W; ++k)
                                if (k <= d.M)
                                    o[k] = (io_t)(yb * wx[(s - k) & m]);
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < W; ++k)
                            sgb[k] += (double)(yb * wx[(s - k) & m]);
                    }
                }
                if (ga != nullptr) {
                    wy[s & m] = ld_y<io_t, acc_t>(d, y, yi, b, t - W);
                    if (TV) {
                        if (in) {
                            io_t *o = ga + row_at(d, b, t, d.N);
#pragma unroll
                            for (int k = 1; k <= W; ++k)
                                if (k <= d.N)
                                    o[k - 1] = (io_t)(-yb * wy[(s - k) & m]);
                        }
                    } else {
#pragma unroll
                        for (int k = 1; k <= W; ++k)
                            sga[k] -= (double)(yb * wy[(s - k) & m]);
                    }
                }
            }
        }
    }
}

// Phase 1 (backward), always in FP64 (see the forward summary).  Items (b, c, j) for chunks c = c_first.. : j < N runs
// the adjoint over chunk c from the unit state s_{j+1} = 1 (gy = 0), j == N
// from zero state with the real gy.  The chunk's outgoing (s, r) is written
// as column j: summ[(b*C+c)*SB + i*N + j] = s_{i+1} (i < N),
// summ[... + N*N + i] = s0 (particular), summ[... + N*N + N + i*N + j] = r_{i+1}
// (i < M), summ[... + N*N + N + M*N + i] = r0.  Time-invariant Phi/R go to
// phi[b*(N*N + M*N) + ...].
template <int W, bool TV, bool PART, typename io_t, typename acc_t>
__global__ void __launch_bounds__(kThreads)
k_bwd_summary(Dims d, const io_t *__restrict__ gy, const io_t *__restrict__ bc,
              const io_t *__restrict__ ac, int64_t c_first, int64_t ncs, int j_first, int nj,
              double *__restrict__ summ, double *__restrict__ phi)
{
    constexpr int m = W - 1;
    const int64_t total = d.B * ncs * nj;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total)
        return;
    int64_t b, cc, jj;
    decode(d, idx, ncs, b, cc, jj);
    const int64_t c = c_first + cc;
    const int j = j_first + (int)jj;
    const int64_t t0 = c * d.L;
    const int N = d.N, M = d.M;
    acc_t la[W + 1], lb[W];
    if (!TV)
        lti_coef<W>(d, bc, ac, b, la, lb);
    acc_t ss[W], rs[W];
#pragma unroll
    for (int q = 0; q < W; ++q) {
        ss[q] = acc_t(0);
        rs[q] = acc_t(0);
    }
    if (!PART) {
        // s_{j+1} = 1; before the first (highest) time, s_k is in slot (k+1) mod W
#pragma unroll
        for (int q = 0; q < W; ++q)
            ss[q] = (q == ((j + 2) & m)) ? acc_t(1) : acc_t(0);
    }
    double sga[W + 1], sgb[W];
    bwd_chunk<W, TV, PART, false, false>(d, b, t0, gy, (const io_t *)nullptr,
                                         (const io_t *)nullptr, (const io_t *)nullptr,
                                         (const io_t *)nullptr, bc, ac, ss, rs, la, lb,
                                         (io_t *)nullptr, (io_t *)nullptr, (io_t *)nullptr, sga,
                                         sgb);
    const int64_t SB = (int64_t)(N + 1) * (N + M);
    double *base = summ + (b * d.C + c) * SB;
    if (PART) {
#pragma unroll
        for (int i = 0; i < W; ++i) {
            if (i < N)
                base[(int64_t)N * N + i] = (double)ss[(i + 2) & m];
            if (i < M)
                base[(int64_t)N * N + N + (int64_t)M * N + i] = (double)rs[(i + 2) & m];
        }
    } else {
        double *pm = TV ? base : phi + b * ((int64_t)N * N + (int64_t)M * N);
        double *rm = TV ? base + (int64_t)N * N + N : pm + (int64_t)N * N;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            if (i < N)
                pm[(int64_t)i * N + j] = (double)ss[(i + 2) & m];
            if (i < M)
                rm[(int64_t)i * N + j] = (double)rs[(i + 2) & m];
        }
    }
}

// Phase 3 (backward).  gin[(b*C+c)*(N+M)] holds the (s, r) state entering
// chunk c from the future (zero for the last chunk).  Writes gx, per-sample
// ga/gb, or per-(b, c) FP64 partial sums of the time-invariant ga/gb into
// part[(b*C+c)*(N+M+1)] (ga_1..ga_N, gb_0..gb_M); chunk 0 writes gyi, gxi.
template <int W, bool TV, bool COEF, typename io_t, typename acc_t>
__global__ void __launch_bounds__(kThreads)
k_bwd_apply(Dims d, const io_t *__restrict__ gy, const io_t *__restrict__ x,
            const io_t *__restrict__ xi, const io_t *__restrict__ y,
            const io_t *__restrict__ yi, const io_t *__restrict__ bc,
            const io_t *__restrict__ ac, const double *__restrict__ gin, io_t *__restrict__ gx,
            io_t *__restrict__ gb, io_t *__restrict__ ga, io_t *__restrict__ gxi,
            io_t *__restrict__ gyi, double *__restrict__ part)
{
    constexpr int m = W - 1;
    const int64_t total = d.B * d.C;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total)
        return;
    int64_t b, c, jj;
    decode(d, idx, d.C, b, c, jj);
    const int64_t t0 = c * d.L;
    const int N = d.N, M = d.M;
    acc_t la[W + 1], lb[W];
    if (!TV)
        lti_coef<W>(d, bc, ac, b, la, lb);
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
            if (i < M)
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
    bwd_chunk<W, TV, true, true, COEF>(d, b, t0, gy, x, xi, y, yi, bc, ac, ss, rs, la, lb, gx,
                                       gb, ga, sga, sgb);
    if (!TV && COEF) {
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
            if (gxi != nullptr && i < M)
                gxi[b * M + i] = (io_t)rs[(i + 2) & m];
        }
    }
}


template <int W, bool TV, typename io_t, typename acc_t>
filt_status forward_impl(const Dims &d, const io_t *x, const io_t *bc, const io_t *ac,
                         const io_t *xi, const io_t *yi, io_t *y, char *ws, hipStream_t st)
{
    const WsPlan w = ws_plan(d);
    double *summ = (double *)(ws + w.summ);
    double *phi = (double *)(ws + w.phi);
    double *states = (double *)(ws + w.states);
    const int N = d.N;
    if (d.C > 1 && N > 0) {
        const int64_t ncs = d.C - 1;  // chunks with a successor
        FILT_LAUNCH("fwd_summary_part", (k_fwd_summary<W, TV, true, io_t, double>), dim3(grid_for(d.B * ncs)),
                           dim3(kThreads), 0, st, d, x, xi, bc, ac, (int64_t)0, ncs, N, 1, summ,
                           phi);
        if (TV)
            FILT_LAUNCH("fwd_summary_homog", (k_fwd_summary<W, TV, false, io_t, double>),
                               dim3(grid_for(d.B * ncs * N)), dim3(kThreads), 0, st, d, x, xi,
                               bc, ac, (int64_t)0, ncs, 0, N, summ, phi);
        else
            FILT_LAUNCH("fwd_summary_homog", (k_fwd_summary<W, TV, false, io_t, double>),
                               dim3(grid_for(d.B * N)), dim3(kThreads), 0, st, d, x, xi, bc, ac,
                               (int64_t)0, (int64_t)1, 0, N, summ, phi);
        filt_status s = check_launch("forward summary");
        if (s != FILT_OK)
            return s;
        CarryArgs a{};
        a.summ = summ;
        a.phi = phi;
        a.SS = (int64_t)N * N + N;
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
    FILT_LAUNCH("fwd_apply", (k_fwd_apply<W, TV, io_t, acc_t>), dim3(grid_for(d.B * d.C)),
                       dim3(kThreads), 0, st, d, x, xi, bc, ac, yi, states, y);
    return check_launch("forward apply");
}

template <int W, bool TV, typename io_t, typename acc_t>
filt_status backward_impl(const Dims &d, const io_t *gy, const io_t *x, const io_t *y,
                          const io_t *bc, const io_t *ac, const io_t *xi, const io_t *yi,
                          io_t *gx, io_t *gb, io_t *ga, io_t *gxi, io_t *gyi, char *ws,
                          hipStream_t st)
{
    const WsPlan w = ws_plan(d);
    double *summ = (double *)(ws + w.summ);
    double *phi = (double *)(ws + w.phi);
    double *states = (double *)(ws + w.states);
    double *part = (double *)(ws + w.part);
    const int N = d.N, M = d.M;
    if (d.C > 1 && N + M > 0) {
        const int64_t ncs = d.C - 1;  // chunks 1..C-1 pass a state to an earlier chunk
        FILT_LAUNCH("bwd_summary_part", (k_bwd_summary<W, TV, true, io_t, double>), dim3(grid_for(d.B * ncs)),
                           dim3(kThreads), 0, st, d, gy, bc, ac, (int64_t)1, ncs, N, 1, summ,
                           phi);
        if (N > 0) {
            if (TV)
                FILT_LAUNCH("bwd_summary_homog", (k_bwd_summary<W, TV, false, io_t, double>),
                                   dim3(grid_for(d.B * ncs * N)), dim3(kThreads), 0, st, d, gy,
                                   bc, ac, (int64_t)1, ncs, 0, N, summ, phi);
            else
                FILT_LAUNCH("bwd_summary_homog", (k_bwd_summary<W, TV, false, io_t, double>),
                                   dim3(grid_for(d.B * N)), dim3(kThreads), 0, st, d, gy, bc, ac,
                                   (int64_t)0, (int64_t)1, 0, N, summ, phi);
        }
        filt_status s = check_launch("backward summary");
        if (s != FILT_OK)
            return s;
        if (N > 0) {
            CarryArgs a{};
            a.summ = summ;
            a.phi = phi;
            a.SS = (int64_t)(N + 1) * (N + M);
            a.D = N;
            a.R = M;
            a.bwd = 1;
            a.agg = (double *)(ws + w.agg);
            a.bstart = (double *)(ws + w.bstart);
            a.states = states;
            s = carry_run(d, a, nullptr, false, st);
            if (s != FILT_OK)
                return s;
        } else {
            s = fir_states_run(d, summ, states, st);
            if (s != FILT_OK)
                return s;
        }
    }
    const bool coef = (ga != nullptr) || (gb != nullptr);
    if (coef)
        FILT_LAUNCH("bwd_apply", (k_bwd_apply<W, TV, true, io_t, acc_t>), dim3(grid_for(d.B * d.C)),
                           dim3(kThreads), 0, st, d, gy, x, xi, y, yi, bc, ac, states, gx, gb, ga,
                           gxi, gyi, part);
    else
        FILT_LAUNCH("bwd_apply", (k_bwd_apply<W, TV, false, io_t, acc_t>), dim3(grid_for(d.B * d.C)),
                           dim3(kThreads), 0, st, d, gy, x, xi, y, yi, bc, ac, states, gx, gb, ga,
                           gxi, gyi, part);
    filt_status s = check_launch("backward apply");
    if (s != FILT_OK)
        return s;
    if (!TV && coef) {
        s = reduce_lti_run(d, part, ga, gb, sizeof(io_t) == 8, st);
    }
    return s;
}


template <int W, typename io_t, typename acc_t>
filt_status forward_w(const Dims &d, const io_t *x, const io_t *bc, const io_t *ac,
                      const io_t *xi, const io_t *yi, io_t *y, char *ws, hipStream_t st)
{
    return d.tv ? forward_impl<W, true, io_t, acc_t>(d, x, bc, ac, xi, yi, y, ws, st)
                : forward_impl<W, false, io_t, acc_t>(d, x, bc, ac, xi, yi, y, ws, st);
}

template <int W, typename io_t, typename acc_t>
filt_status backward_w(const Dims &d, const io_t *gy, const io_t *x, const io_t *y,
                       const io_t *bc, const io_t *ac, const io_t *xi, const io_t *yi, io_t *gx,
                       io_t *gb, io_t *ga, io_t *gxi, io_t *gyi, char *ws, hipStream_t st)
{
    return d.tv ? backward_impl<W, true, io_t, acc_t>(d, gy, x, y, bc, ac, xi, yi, gx, gb, ga,
                                                      gxi, gyi, ws, st)
                : backward_impl<W, false, io_t, acc_t>(d, gy, x, y, bc, ac, xi, yi, gx, gb, ga,
                                                       gxi, gyi, ws, st);
}

}  // namespace filt_detail
