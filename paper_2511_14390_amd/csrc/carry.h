// carry.h -- device bodies of the carry scan (phase 2), shared by the
// dense kernels in carry.hip and the batched kernels in batched.hip.
//
// Chunk summaries (Phi_c, s_c) combine with the operator of Sec. 3.2,
// (Phi, s) then (Phi', s') = (Phi' Phi, Phi' s + s').  The scan is blocked:
//   (1) carry_agg    every block of G consecutive steps is reduced to one
//                    affine map (one workgroup per block, the running
//                    D x (D+1) matrix in LDS, one thread per entry);
//   (2) carry_blocks one pass per channel over the blocks gives the state at
//                    every block start (one workgroup per channel);
//   (3) carry_fill   every block replays its steps from that state and writes
//                    the state entering each chunk (one workgroup per block).
// Each step is a short dependent chain, so a workgroup first copies the
// records of a run of steps from HBM into LDS with every thread loading
// (many loads in flight, one memory latency per run) and then walks the steps
// out of LDS.  For a time-invariant filter Phi (and R) are the same for every
// chunk and stay in registers; only the vectors are staged.
// All arithmetic is FP64.  D = the filter order N (<= 16).
#pragma once

#include "common.h"

namespace filt_detail {

constexpr int kMaxD = 16;

// LDS budget of one staged run of step records, in doubles (32 KiB).
constexpr int kStageDoubles = 4096;

// Steps per staged run for records of `rec` doubles, out of `steps`.
__host__ __device__ inline int stage_steps(int rec, int64_t steps)
{
    int k = rec > 0 ? kStageDoubles / rec : kStageDoubles;
    if (k < 1)
        k = 1;
    return (int)((int64_t)k < steps ? (int64_t)k : steps);
}

// Record layout of the chunk summaries as the carry reads them: per chunk
// (stride SS) Phi [D x D] (per-sample filters), the vector s at offset soff
// and, for the backward with M > 0, R [M x D] and r0 [M] after it.
// Time-invariant filters keep Phi (and R) once per channel, so only the part
// from s on is staged.
struct CarryRec {
    int agg_off, agg_len;    // what the block aggregation reads
    int fill_off, fill_len;  // what the in-block fill reads
    int blk_len;             // one block aggregate [P | q]
};

__host__ __device__ inline CarryRec carry_rec(int tv, int D, int64_t SS, int64_t soff)
{
    CarryRec r;
    r.agg_off = tv ? 0 : (int)soff;
    r.agg_len = tv ? (int)soff + D : D;
    r.fill_off = r.agg_off;
    r.fill_len = (int)SS - r.fill_off;
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
    const unsigned urec = (unsigned)rec;
    for (unsigned e0 = threadIdx.x; e0 < n; e0 += U * nt) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const unsigned e = e0 + u * nt;
            if (e < n) {
                const unsigned r = e / urec;
                const unsigned w = e - r * urec;
                v[u] = base[(r_lo + r) * stride + off + w];
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

// Row `row` (D entries, zero padded to DB) of a constant matrix, in registers.
template <int DB>
__device__ __forceinline__ void const_row(const double *row, int D, double (&r)[DB])
{
#pragma unroll
    for (int k = 0; k < DB; ++k)
        r[k] = (row != nullptr && k < D) ? row[k] : 0.0;
}

// (1) Block aggregates.  Workgroup (b, blk); thread e = i*(D+1) + j holds
// entry (i, j) of [P | q]: column j < D of the block's matrix, column D its
// vector.  agg[(b*NB + blk)*(D*D + D) + i*D + j] = P[i][j], [... + D*D + i] = q[i].
// stage: dynamic LDS of stage_steps(agg_len, G) * agg_len doubles.
template <int DB, bool TV>
__device__ __forceinline__ void carry_agg_body(const Dims &d, const CarryArgs &a, int64_t b,
                                               int64_t blk, double *stage)
{
    __shared__ double Pm[2][kMaxD][kMaxD + 1];
    const int D = a.D;
    const int DD = D * D;
    const CarryRec cr = carry_rec(TV, D, a.SS, a.soff);
    const int e = threadIdx.x;
    const bool act = e < D * (D + 1);
    const int i = act ? e / (D + 1) : 0;
    const int j = act ? e % (D + 1) : 0;
    if (act)
        Pm[0][i][j] = (j == i) ? 1.0 : 0.0;
    double fixed[DB];
    const_row<DB>(TV ? nullptr : a.phi + b * (DD + (int64_t)a.R * D) + i * D, D, fixed);
    const int64_t i0 = blk * d.G;
    const int64_t i1 = min(i0 + d.G, d.C - 1);
    const int K = stage_steps(cr.agg_len, d.G);
    const double *sb = a.summ + b * d.C * a.SS;
    // within a record: row i of Phi at i*D (per-sample), s[i] after the offset
    const int s_at = (int)a.soff + i - cr.agg_off;
    int cur = 0;
    for (int64_t t0 = i0; t0 < i1; t0 += K) {
        const int k = (int)min<int64_t>(K, i1 - t0);
        const int64_t c_lo = a.bwd ? d.C - t0 - k : t0;
        __syncthreads();
        stage_records(sb, a.SS, c_lo, k, cr.agg_off, cr.agg_len, stage);
        __syncthreads();
        for (int q = 0; q < k; ++q) {
            if (act) {
                const double *rec = stage + (a.bwd ? k - 1 - q : q) * cr.agg_len;
                double acc0 = (j == D) ? rec[s_at] : 0.0;
                double acc1 = 0.0;
#pragma unroll
                for (int k2 = 0; k2 < DB; k2 += 2) {
                    if (k2 < D)
                        acc0 += (TV ? rec[i * D + k2] : fixed[k2]) * Pm[cur][k2][j];
                    if (k2 + 1 < D)
                        acc1 += (TV ? rec[i * D + k2 + 1] : fixed[k2 + 1]) * Pm[cur][k2 + 1][j];
                }
                Pm[cur ^ 1][i][j] = acc0 + acc1;
            }
            cur ^= 1;
            __syncthreads();
        }
    }
    if (act) {
        double *o = a.agg + (b * d.NB + blk) * (int64_t)(DD + D);
        if (j < D)
            o[i * D + j] = Pm[cur][i][j];
        else
            o[DD + i] = Pm[cur][i][D];
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
template <int DB, bool TV>
__device__ __forceinline__ void carry_fill_body(const Dims &d, const CarryArgs &a, int64_t b,
                                                int64_t blk, double *stage)
{
    __shared__ double v[2][kMaxD];
    const int D = a.D;
    const int R = a.R;
    const int SD = D + R;
    const int DD = D * D;
    const CarryRec cr = carry_rec(TV, D, a.SS, a.soff);
    const int i = threadIdx.x;
    const bool act = i < SD;
    if (i < D)
        v[0][i] = a.bstart[(b * d.NB + blk) * D + i];
    // thread i < D: row i of Phi and s[i]; thread D + q: row q of R and r0[q]
    // (offsets within a staged record)
    const int so = (int)a.soff;
    const int row_at = i < D ? i * D : so + D + (i - D) * D;
    const int s_at = (i < D ? so + i : so + D + R * D + (i - D)) - cr.fill_off;
    double fixed[DB];
    {
        const double *pb = a.phi + b * (DD + (int64_t)R * D);
        const double *row = i < D ? pb + i * D : pb + DD + (i - D) * D;
        const_row<DB>((!TV && act) ? row : nullptr, D, fixed);
    }
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
        stage_records(sb, a.SS, c_lo, k, cr.fill_off, cr.fill_len, stage);
        __syncthreads();
        for (int q = 0; q < k; ++q) {
            if (act) {
                const double *rec = stage + (a.bwd ? k - 1 - q : q) * cr.fill_len;
                double acc0 = rec[s_at];
                double acc1 = 0.0;
#pragma unroll
                for (int k2 = 0; k2 < DB; k2 += 2) {
                    if (k2 < D)
                        acc0 += (TV ? rec[row_at + k2] : fixed[k2]) * v[cur][k2];
                    if (k2 + 1 < D)
                        acc1 += (TV ? rec[row_at + k2 + 1] : fixed[k2 + 1]) * v[cur][k2 + 1];
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
