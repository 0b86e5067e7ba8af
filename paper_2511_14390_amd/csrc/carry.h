// carry.h -- device bodies of the carry scan (phase 2), shared by the
// dense kernels in carry.hip and the batched kernels in batched.hip.
//
// Chunk summaries (Phi_c, s_c) combine with the operator of Sec. 3.2,
// (Phi, s) then (Phi', s') = (Phi' Phi, Phi' s + s').  The scan is blocked:
//   (1) carry_agg    every block of G consecutive steps is reduced to one
//                    affine map (one workgroup per block, the running
//                    D x (D+1) matrix in LDS, one thread per entry);
//   (2) carry_blocks one pass per channel over the blocks gives the state at
//                    every block start (one wavefront per channel);
//   (3) carry_fill   every block replays its steps from that state and writes
//                    the state entering each chunk (one wavefront per block).
// All arithmetic is FP64.  D = the filter order N (<= 16).
#pragma once

#include "common.h"

namespace filt_detail {

constexpr int kMaxD = 16;

__device__ __forceinline__ int64_t step_chunk(const Dims &d, const CarryArgs &a, int64_t i)
{
    return a.bwd ? d.C - 1 - i : i;
}

// Phi (D x D, row-major) and s of scan step i.
__device__ __forceinline__ void step_ops(const Dims &d, const CarryArgs &a, int64_t b, int64_t i,
                                         const double *&P, const double *&s)
{
    const int64_t c = step_chunk(d, a, i);
    const double *base = a.summ + (b * d.C + c) * a.SS;
    const int64_t DD = (int64_t)a.D * a.D;
    P = d.tv ? base : a.phi + b * (DD + (int64_t)a.R * a.D);
    s = base + DD;
}

// (1) Block aggregates.  Workgroup (b, blk); thread e = i*(D+1) + j holds
// entry (i, j) of [P | q]: column j < D of the block's matrix, column D its
// vector.  agg[(b*NB + blk)*(D*D + D) + i*D + j] = P[i][j], [... + D*D + i] = q[i].
__device__ __forceinline__ void carry_agg_body(const Dims &d, const CarryArgs &a, int64_t b,
                                               int64_t blk)
{
    __shared__ double Pm[2][kMaxD][kMaxD + 1];
    const int D = a.D;
    const int e = threadIdx.x;
    const bool act = e < D * (D + 1);
    const int i = act ? e / (D + 1) : 0;
    const int j = act ? e % (D + 1) : 0;
    if (act)
        Pm[0][i][j] = (j == i) ? 1.0 : 0.0;
    __syncthreads();
    const int64_t i0 = blk * d.G;
    const int64_t i1 = min(i0 + d.G, d.C - 1);
    int cur = 0;
    for (int64_t st = i0; st < i1; ++st) {
        const double *P, *s;
        step_ops(d, a, b, st, P, s);
        if (act) {
            double acc = (j == D) ? s[i] : 0.0;
            for (int k = 0; k < D; ++k)
                acc += P[i * D + k] * Pm[cur][k][j];
            Pm[cur ^ 1][i][j] = acc;
        }
        cur ^= 1;
        __syncthreads();
    }
    if (act) {
        double *o = a.agg + (b * d.NB + blk) * (int64_t)(D * D + D);
        if (j < D)
            o[i * D + j] = Pm[cur][i][j];
        else
            o[D * D + i] = Pm[cur][i][D];
    }
}

// (2) Sequential pass over blocks; one wavefront per channel, lane i holds
// state entry i.  init: [B][D] state before the first step (float or double),
// or null for zero.  bstart[(b*NB + blk)*D + i] = state at the block start.
__device__ __forceinline__ void carry_blocks_body(const Dims &d, const CarryArgs &a,
                                                  const void *init, int init_f64, int64_t b)
{
    __shared__ double v[2][kMaxD];
    const int D = a.D;
    const int i = threadIdx.x;
    const bool act = i < D;
    if (act) {
        double x0 = 0.0;
        if (init != nullptr)
            x0 = init_f64 ? ((const double *)init)[b * D + i]
                          : (double)((const float *)init)[b * D + i];
        v[0][i] = x0;
    }
    __syncthreads();
    int cur = 0;
    for (int64_t blk = 0; blk < d.NB; ++blk) {
        if (act) {
            a.bstart[(b * d.NB + blk) * D + i] = v[cur][i];
            const double *o = a.agg + (b * d.NB + blk) * (int64_t)(D * D + D);
            double acc = o[D * D + i];
            for (int k = 0; k < D; ++k)
                acc += o[i * D + k] * v[cur][k];
            v[cur ^ 1][i] = acc;
        }
        cur ^= 1;
        __syncthreads();
    }
}

// (3) States inside each block; one wavefront per (b, blk).  Lanes i < D
// advance the state; for the backward, lanes D <= i < D + R also form the FIR
// adjoint state R S + r0 carried across the same chunk boundary (R, r0 of the
// chunk the step crosses, S the state entering that chunk).  Writes
// states[(b*C + cn)*(D + R)] for the chunk cn entered after each step.
__device__ __forceinline__ void carry_fill_body(const Dims &d, const CarryArgs &a, int64_t b,
                                                int64_t blk)
{
    __shared__ double v[2][kMaxD];
    const int D = a.D;
    const int R = a.R;
    const int SD = D + R;
    const int64_t DD = (int64_t)D * D;
    const int i = threadIdx.x;
    if (i < D)
        v[0][i] = a.bstart[(b * d.NB + blk) * D + i];
    __syncthreads();
    const int64_t i0 = blk * d.G;
    const int64_t i1 = min(i0 + d.G, d.C - 1);
    int cur = 0;
    for (int64_t st = i0; st < i1; ++st) {
        const double *P, *s;
        step_ops(d, a, b, st, P, s);
        const int64_t cn = a.bwd ? d.C - 2 - st : st + 1;
        double *o = a.states + (b * d.C + cn) * SD;
        if (i < D) {
            double acc = s[i];
            for (int k = 0; k < D; ++k)
                acc += P[i * D + k] * v[cur][k];
            v[cur ^ 1][i] = acc;
            o[i] = acc;
        } else if (i < SD) {
            const int q = i - D;
            const int64_t c = step_chunk(d, a, st);
            const double *base = a.summ + (b * d.C + c) * a.SS;
            const double *Rm = d.tv ? base + DD + D : a.phi + b * (DD + (int64_t)R * D) + DD;
            const double *r0 = base + DD + D + (int64_t)R * D;
            double acc = r0[q];
            for (int k = 0; k < D; ++k)
                acc += Rm[q * D + k] * v[cur][k];
            o[D + q] = acc;
        }
        cur ^= 1;
        __syncthreads();
    }
}

}  // namespace filt_detail
