// carry.h -- device bodies of the carry scan (phase 2) for per-sample
// coefficients, shared by the dense kernels in carry.hip and the batched
// kernels in batched.hip (time-invariant filters use the log-depth scan in
// carry.hip).
//
// Chunk summaries (Phi_c, s_c) combine with the operator of Sec. 3.2,
// (Phi, s) then (Phi', s') = (Phi' Phi, Phi' s + s').  The scan is blocked:
//   (1) carry_agg    every block of G consecutive steps is reduced to one
//                    affine map (one wavefront per block, the running
//                    [P | q] in MFMA registers);
//   (2) carry_blocks one pass per channel over the blocks gives the state at
//                    every block start (one workgroup per channel);
//   (3) carry_fill   every block replays its steps from that state and writes
//                    the state entering each chunk (one workgroup per block).
// Steps (2) and (3) are chains of matrix-vector products: a workgroup first
// copies the records of a run of steps from HBM into LDS with every thread
// loading (many loads in flight, one memory latency per run) and then walks
// the steps out of LDS.  All arithmetic is FP64.  D = the filter order N
// (<= 16).
#pragma once

#include "common.h"

namespace filt_detail {

constexpr int kMaxD = 16;

// LDS budget of one staged run of step records, in doubles (36 KiB: 16
// steps of an order-16 summary).
constexpr int kStageDoubles = 4608;

// Steps per staged run for records of `rec` doubles, out of `steps`.
__host__ __device__ inline int stage_steps(int rec, int64_t steps)
{
    int k = rec > 0 ? kStageDoubles / rec : kStageDoubles;
    if (k < 1)
        k = 1;
    return (int)((int64_t)k < steps ? (int64_t)k : steps);
}

// Record layout of the chunk summaries as the carry reads them: per chunk
// (stride SS) Phi [D x D], the vector s at offset soff and, for the backward
// with M > 0, R [M x D] and r0 [M] after it.  The fill stages whole records.
struct CarryRec {
    int fill_len;  // doubles of one chunk record
    int blk_len;   // one block aggregate [P | q]
};

__host__ __device__ inline CarryRec carry_rec(int D, int64_t SS)
{
    CarryRec r;
    r.fill_len = (int)SS;
    r.blk_len = D * D + D;
    return r;
}

// Workgroup copy of k records into LDS: record r (0 <= r < k) is the doubles
// [off, off + rec) of entry r_lo + r of an array with entry stride `stride`;
// it lands at lds[r * rec].  Each thread keeps up to 8 loads in flight.
__device__ __forceinline__ void stage_records(const double *__restrict__ base, int64_t stride,
                                              int64_t r_lo, int k, int off, int rec,
                                              double *lds)
{
    constexpr int U = 8;
    const unsigned n = (unsigned)k * (unsigned)rec;
    const unsigned nt = blockDim.x;
    if (stride == rec && off == 0) {
        // whole records back to back: one linear run, in rounds of U * nt
        // elements without per-element tests, then one guarded round
        const double *src = base + r_lo * stride;
        const unsigned full = n / (U * nt) * (U * nt);
        for (unsigned b0 = 0; b0 < full; b0 += U * nt) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                v[u] = src[b0 + threadIdx.x + u * nt];
#pragma unroll
            for (int u = 0; u < U; ++u)
                lds[b0 + threadIdx.x + u * nt] = v[u];
        }
        if (full < n) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const unsigned e = full + threadIdx.x + u * nt;
                if (e < n)
                    v[u] = src[e];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const unsigned e = full + threadIdx.x + u * nt;
                if (e < n)
                    lds[e] = v[u];
            }
        }
        return;
    }
    // (record, word) of element e kept up to date by additions: e advances
    // by nt, i.e. by dq records and dr words with a carry
    const unsigned urec = (unsigned)rec;
    const unsigned dq = nt / urec, dr = nt - dq * urec;
    unsigned r = threadIdx.x / urec, w = threadIdx.x - (threadIdx.x / urec) * urec;
    for (unsigned e0 = threadIdx.x; e0 < n; e0 += U * nt) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const unsigned e = e0 + u * nt;
            if (e < n)
                v[u] = base[(r_lo + r) * stride + off + w];
            w += dr;
            r += dq;
            if (w >= urec) {
                w -= urec;
                ++r;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const unsigned e = e0 + u * nt;
            if (e < n)
                lds[e] = v[u];
        }
    }
}

typedef double doublex4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ doublex4 mfma_f64(double a, double b, doublex4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// (1) Block aggregates of per-sample transitions, on the FP64 matrix cores.
// One wavefront per (b, blk).  The running [P | q] is held as two 16 x 16
// tiles (zero-padded past D; q in column 0 of the second) in the output
// layout of the FP64 16x16x4 MFMA: lane l has rows 4 r + l / 16 (r < 4) of
// column l % 16.  A step multiplies both by Phi_c with four 16x16x4 products
// each; product s takes k = 4 s + l / 16, so its B operand is register r = s
// of the same lane and the chain never leaves registers.  The operands of the
// next steps are fetched kCarryPrefetch steps ahead.
// agg[(b*NB + blk)*(D*D + D) + i*D + j] = P[i][j], [... + D*D + i] = q[i].
constexpr int kCarryPrefetch = 4;

struct CarryOps {
    double f[4];  // Phi_c[l % 16][4 s + l / 16]
    double s[4];  // s_c[4 r + l / 16] in column 0, else 0
};

__device__ __forceinline__ void carry_agg_body(const Dims &d, const CarryArgs &a, int64_t b,
                                               int64_t blk)
{
    constexpr int PD = kCarryPrefetch;
    const int D = a.D;
    const int l = threadIdx.x & 63;
    const int j = l & 15, g = l >> 4;
    doublex4 P, q;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        P[r] = (4 * r + g == j && j < D) ? 1.0 : 0.0;
        q[r] = 0.0;
    }
    const int64_t i0 = blk * d.G;
    const int64_t i1 = min(i0 + d.G, d.C - 1);
    auto fetch = [&](int64_t st, CarryOps &o) {
        const int64_t c = a.bwd ? d.C - 1 - st : st;
        const double *base = a.summ + (b * d.C + c) * a.SS;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = 4 * t + g;
            o.f[t] = (j < D && k < D) ? base[j * D + k] : 0.0;
            o.s[t] = (j == 0 && k < D) ? base[a.soff + k] : 0.0;
        }
    };
    CarryOps buf[PD];
#pragma unroll
    for (int t = 0; t < PD; ++t)
        if (i0 + t < i1)
            fetch(i0 + t, buf[t]);
    for (int64_t base = i0; base < i1; base += PD) {
#pragma unroll
        for (int t = 0; t < PD; ++t) {
            const int64_t st = base + t;
            if (st < i1) {
                const CarryOps o = buf[t];
                if (st + PD < i1)
                    fetch(st + PD, buf[t]);
                doublex4 Pn = {0.0, 0.0, 0.0, 0.0};
                doublex4 qn = {o.s[0], o.s[1], o.s[2], o.s[3]};
                Pn = mfma_f64(o.f[0], P[0], Pn);
                qn = mfma_f64(o.f[0], q[0], qn);
                Pn = mfma_f64(o.f[1], P[1], Pn);
                qn = mfma_f64(o.f[1], q[1], qn);
                Pn = mfma_f64(o.f[2], P[2], Pn);
                qn = mfma_f64(o.f[2], q[2], qn);
                Pn = mfma_f64(o.f[3], P[3], Pn);
                qn = mfma_f64(o.f[3], q[3], qn);
                P = Pn;
                q = qn;
            }
        }
    }
    double *o = a.agg + (b * d.NB + blk) * (int64_t)(D * D + D);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = 4 * r + g;
        if (i < D && j < D)
            o[i * D + j] = P[r];
        if (i < D && j == 0)
            o[D * D + i] = q[r];
    }
}

// (2) Sequential pass over blocks; one workgroup per channel, thread i < D
// holds state entry i.  init: [B][D] state before the first step (float or
// double), or null for zero.  bstart[(b*NB + blk)*D + i] = state at the block
// start.  stage: stage_steps(D*D + D, NB) * (D*D + D) doubles.
template <int DB>
__device__ __forceinline__ void carry_blocks_body(const Dims &d, const CarryArgs &a,
                                                  const void *init, int init_f64, int64_t b,
                                                  double *stage)
{
    __shared__ double v[2][kMaxD];
    const int D = a.D;
    const int DD = D * D;
    const int rec = DD + D;
    const int i = threadIdx.x;
    const bool act = i < D;
    if (act) {
        double x0 = 0.0;
        if (init != nullptr)
            x0 = init_f64 ? ((const double *)init)[b * D + i]
                          : (double)((const float *)init)[b * D + i];
        v[0][i] = x0;
    }
    const int K = stage_steps(rec, d.NB);
    const double *ab = a.agg + b * d.NB * rec;
    int cur = 0;
    for (int64_t t0 = 0; t0 < d.NB; t0 += K) {
        const int k = (int)min<int64_t>(K, d.NB - t0);
        __syncthreads();
        stage_records(ab, rec, t0, k, 0, rec, stage);
        __syncthreads();
        for (int q = 0; q < k; ++q) {
            if (act) {
                const double *r = stage + q * rec;
                a.bstart[(b * d.NB + t0 + q) * D + i] = v[cur][i];
                double acc0 = r[DD + i];
                double acc1 = 0.0;
#pragma unroll
                for (int k2 = 0; k2 < DB; k2 += 2) {
                    if (k2 < D)
                        acc0 += r[i * D + k2] * v[cur][k2];
                    if (k2 + 1 < D)
                        acc1 += r[i * D + k2 + 1] * v[cur][k2 + 1];
                }
                v[cur ^ 1][i] = acc0 + acc1;
            }
            cur ^= 1;
            __syncthreads();
        }
    }
}

// (3) States inside each block; one workgroup per (b, blk).  Threads i < D
// advance the state; for the backward, threads D <= i < D + R also form the
// FIR adjoint state R S + r0 carried across the same chunk boundary (R, r0 of
// the chunk the step crosses, S the state entering that chunk).  Writes
// states[(b*C + cn)*(D + R)] for the chunk cn entered after each step.
// stage: stage_steps(fill_len, G) * fill_len doubles.
template <int DB>
__device__ __forceinline__ void carry_fill_body(const Dims &d, const CarryArgs &a, int64_t b,
                                                int64_t blk, double *stage)
{
    __shared__ double v[2][kMaxD];
    const int D = a.D;
    const int R = a.R;
    const int SD = D + R;
    const int DD = D * D;
    const CarryRec cr = carry_rec(D, a.SS);
    const int i = threadIdx.x;
    const bool act = i < SD;
    if (i < D)
        v[0][i] = a.bstart[(b * d.NB + blk) * D + i];
    // thread i < D: row i of Phi and s[i]; thread D + q: row q of R and r0[q]
    // (offsets within a staged record)
    const int so = (int)a.soff;
    const int row_at = i < D ? i * D : so + D + (i - D) * D;
    const int s_at = i < D ? so + i : so + D + R * D + (i - D);
    const int64_t i0 = blk * d.G;
    const int64_t i1 = min(i0 + d.G, d.C - 1);
    const int K = stage_steps(cr.fill_len, d.G);
    const double *sb = a.summ + b * d.C * a.SS;
    double *ob = a.states + b * d.C * SD + i;
    int cur = 0;
    for (int64_t t0 = i0; t0 < i1; t0 += K) {
        const int k = (int)min<int64_t>(K, i1 - t0);
        const int64_t c_lo = a.bwd ? d.C - t0 - k : t0;
        __syncthreads();
        stage_records(sb, a.SS, c_lo, k, 0, cr.fill_len, stage);
        __syncthreads();
        for (int q = 0; q < k; ++q) {
            if (act) {
                const double *rec = stage + (a.bwd ? k - 1 - q : q) * cr.fill_len;
                double acc0 = rec[s_at];
                double acc1 = 0.0;
#pragma unroll
                for (int k2 = 0; k2 < DB; k2 += 2) {
                    if (k2 < D)
                        acc0 += rec[row_at + k2] * v[cur][k2];
                    if (k2 + 1 < D)
                        acc1 += rec[row_at + k2 + 1] * v[cur][k2 + 1];
                }
                const double acc = acc0 + acc1;
                const int64_t st = t0 + q;
                const int64_t cn = a.bwd ? d.C - 2 - st : st + 1;
                ob[cn * SD] = acc;
                if (i < D)
                    v[cur ^ 1][i] = acc;
            }
            cur ^= 1;
            __syncthreads();
        }
    }
}

// Threads for a staged carry workgroup: enough to load a run with about 16
// loads per thread, at least `active`, a multiple of 64, at most 256.
inline unsigned carry_threads(int64_t stage_doubles, int active)
{
    int64_t t = (stage_doubles + 15) / 16;
    t = std::max<int64_t>(t, active);
    t = std::min<int64_t>(std::max<int64_t>(t, 64), 256);
    return (unsigned)((t + 63) / 64 * 64);
}

// Dispatch on the order bucket (rows of 4, 8 or 16 doubles).
#define FILT_CARRY_DB(D, CALL)                                                                     \
    do {                                                                                           \
        if ((D) <= 4) {                                                                            \
            CALL(4);                                                                               \
        } else if ((D) <= 8) {                                                                     \
            CALL(8);                                                                               \
        } else {                                                                                   \
            CALL(16);                                                                              \
        }                                                                                          \
    } while (0)

}  // namespace filt_detail
