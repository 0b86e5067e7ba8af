// carry.hip -- the scan over chunk summaries, and the small reduction
// kernels of the backward.
//
// The chunk summaries (Phi_c, s_c) combine with the operator of Sec. 3.2,
// (Phi, s) then (Phi', s') = (Phi' Phi, Phi' s + s').  The scan is blocked:
// (1) every block of G consecutive steps is reduced to one affine map,
// (2) one sequential pass per channel over the blocks gives the state at
// every block start, (3) every block replays its G steps from that state and
// writes the state entering each chunk.  All arithmetic is FP64.
//
// State vectors use a compile-time bucket DB >= D (D = the filter order) so a
// few kernels cover every order; matrices keep their true row stride D.
#include "common.h"

namespace filt_detail {
namespace {

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

template <int DB>
__device__ __forceinline__ void matvec(const double *P, const double *s, int D,
                                       const double (&v)[DB], double (&nv)[DB])
{
#pragma unroll
    for (int q = 0; q < DB; ++q) {
        double acc = 0.0;
        if (q < D) {
            acc = (s != nullptr) ? s[q] : 0.0;
#pragma unroll
            for (int k = 0; k < DB; ++k)
                if (k < D)
                    acc += P[q * D + k] * v[k];
        }
        nv[q] = acc;
    }
}

// (1) Block aggregates.  Item (b, blk, j): j < D propagates e_j (column j of
// the block's matrix), j == D propagates 0 with the offsets (its vector).
// agg[(b*NB + blk)*(D*D + D) + r*D + j] = P[r][j], agg[... + D*D + r] = q[r].
template <int DB>
__global__ void __launch_bounds__(kThreads) k_carry_agg(Dims d, CarryArgs a)
{
    const int D = a.D;
    const int64_t total = d.B * d.NB * (D + 1);
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total)
        return;
    const int j = (int)(idx % (D + 1));
    const int64_t r = idx / (D + 1);
    const int64_t blk = r % d.NB;
    const int64_t b = r / d.NB;
    const int64_t i0 = blk * d.G;
    const int64_t i1 = min(i0 + d.G, d.C - 1);
    double v[DB];
#pragma unroll
    for (int q = 0; q < DB; ++q)
        v[q] = (q == j) ? 1.0 : 0.0;
    for (int64_t i = i0; i < i1; ++i) {
        const double *P, *s;
        step_ops(d, a, b, i, P, s);
        double nv[DB];
        matvec<DB>(P, j == D ? s : nullptr, D, v, nv);
#pragma unroll
        for (int q = 0; q < DB; ++q)
            v[q] = nv[q];
    }
    double *o = a.agg + (b * d.NB + blk) * (int64_t)(D * D + D);
#pragma unroll
    for (int q = 0; q < DB; ++q) {
        if (q < D) {
            if (j < D)
                o[q * D + j] = v[q];
            else
                o[D * D + q] = v[q];
        }
    }
}

// (2) Sequential pass over blocks, one thread per channel.  init: [B][D]
// state before the first step (float or double), or null for zero.
template <int DB>
__global__ void __launch_bounds__(kThreads)
k_carry_blocks(Dims d, CarryArgs a, const void *init, int init_f64)
{
    const int D = a.D;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= d.B)
        return;
    double v[DB];
#pragma unroll
    for (int q = 0; q < DB; ++q) {
        double x0 = 0.0;
        if (init != nullptr && q < D)
            x0 = init_f64 ? ((const double *)init)[b * D + q]
                          : (double)((const float *)init)[b * D + q];
        v[q] = x0;
    }
    for (int64_t blk = 0; blk < d.NB; ++blk) {
        double *bs = a.bstart + (b * d.NB + blk) * D;
#pragma unroll
        for (int q = 0; q < DB; ++q)
            if (q < D)
                bs[q] = v[q];
        const double *o = a.agg + (b * d.NB + blk) * (int64_t)(D * D + D);
        double nv[DB];
        matvec<DB>(o, o + D * D, D, v, nv);
#pragma unroll
        for (int q = 0; q < DB; ++q)
            v[q] = nv[q];
    }
}

// (3) States inside each block, one thread per (b, blk).  Writes the state
// after every step, i.e. the state entering the next chunk in scan order;
// backward also writes the FIR adjoint state R S + r0 carried across the same
// chunk boundary (R, r0 of the chunk the step crosses, S the state entering
// that chunk).
template <int DB>
__global__ void __launch_bounds__(kThreads) k_carry_fill(Dims d, CarryArgs a)
{
    const int D = a.D;
    const int64_t total = d.B * d.NB;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total)
        return;
    const int64_t blk = idx % d.NB;
    const int64_t b = idx / d.NB;
    const int64_t i0 = blk * d.G;
    const int64_t i1 = min(i0 + d.G, d.C - 1);
    const int SD = D + a.R;
    const int64_t DD = (int64_t)D * D;
    double v[DB];
    const double *bs = a.bstart + (b * d.NB + blk) * D;
#pragma unroll
    for (int q = 0; q < DB; ++q)
        v[q] = (q < D) ? bs[q] : 0.0;
    for (int64_t i = i0; i < i1; ++i) {
        const double *P, *s;
        step_ops(d, a, b, i, P, s);
        double nv[DB];
        matvec<DB>(P, s, D, v, nv);
        const int64_t cn = a.bwd ? d.C - 2 - i : i + 1;
        double *o = a.states + (b * d.C + cn) * SD;
        if (a.R > 0) {
            const int64_t c = step_chunk(d, a, i);
            const double *base = a.summ + (b * d.C + c) * a.SS;
            const double *Rm = d.tv ? base + DD + D : a.phi + b * (DD + (int64_t)a.R * D) + DD;
            const double *r0 = base + DD + D + (int64_t)a.R * D;
            for (int q = 0; q < a.R; ++q) {
                double acc = r0[q];
#pragma unroll
                for (int k = 0; k < DB; ++k)
                    if (k < D)
                        acc += Rm[q * D + k] * v[k];
                o[D + q] = acc;
            }
        }
#pragma unroll
        for (int q = 0; q < DB; ++q) {
            v[q] = nv[q];
            if (q < D)
                o[q] = v[q];
        }
    }
}

template <int DB>
filt_status run_carry(const Dims &d, const CarryArgs &a, const void *init, bool init_f64,
                      hipStream_t st)
{
    FILT_LAUNCH("carry_agg", (k_carry_agg<DB>), dim3(grid_for(d.B * d.NB * (a.D + 1))),
                       dim3(kThreads), 0, st, d, a);
    FILT_LAUNCH("carry_blocks", (k_carry_blocks<DB>), dim3(grid_for(d.B)), dim3(kThreads), 0, st, d, a,
                       init, (int)init_f64);
    FILT_LAUNCH("carry_fill", (k_carry_fill<DB>), dim3(grid_for(d.B * d.NB)), dim3(kThreads), 0, st, d,
                       a);
    return check_launch("carry");
}

// Pure FIR backward (N == 0): the FIR adjoint state entering chunk c is the
// zero-state outgoing state r0 of chunk c+1 (no feedback to carry).
__global__ void __launch_bounds__(kThreads)
k_fir_states(Dims d, const double *__restrict__ summ, double *__restrict__ states)
{
    const int M = d.M;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= d.B * (d.C - 1) * M)
        return;
    const int q = (int)(idx % M);
    const int64_t r = idx / M;
    const int64_t c = r % (d.C - 1);
    const int64_t b = r / (d.C - 1);
    states[(b * d.C + c) * M + q] = summ[(b * d.C + c + 1) * M + q];
}

// Sum the per-chunk partials of time-invariant ga / gb over chunks (FP64,
// fixed order).
template <typename io_t>
__global__ void __launch_bounds__(kThreads)
k_reduce_lti(Dims d, const double *__restrict__ part, io_t *__restrict__ ga,
             io_t *__restrict__ gb)
{
    const int K = d.N + d.M + 1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= d.B * K)
        return;
    const int64_t b = idx / K;
    const int k = (int)(idx % K);
    double acc = 0.0;
    for (int64_t c = 0; c < d.C; ++c)
        acc += part[(b * d.C + c) * K + k];
    if (k < d.N) {
        if (ga != nullptr)
            ga[b * d.N + k] = (io_t)acc;
    } else if (gb != nullptr) {
        gb[b * (d.M + 1) + (k - d.N)] = (io_t)acc;
    }
}

}  // namespace

filt_status carry_run(const Dims &d, const CarryArgs &a, const void *init, bool init_f64,
                      hipStream_t st)
{
    if (d.C < 2)
        return FILT_OK;
    if (a.D <= 1)
        return run_carry<1>(d, a, init, init_f64, st);
    if (a.D <= 2)
        return run_carry<2>(d, a, init, init_f64, st);
    if (a.D <= 4)
        return run_carry<4>(d, a, init, init_f64, st);
    if (a.D <= 8)
        return run_carry<8>(d, a, init, init_f64, st);
    if (a.D <= 16)
        return run_carry<16>(d, a, init, init_f64, st);
    return fail(FILT_EUNSUPPORTED, "carry order %d", a.D);
}

filt_status fir_states_run(const Dims &d, const double *summ, double *states, hipStream_t st)
{
    if (d.C < 2 || d.M == 0)
        return FILT_OK;
    FILT_LAUNCH("fir_states", k_fir_states, dim3(grid_for(d.B * (d.C - 1) * d.M)), dim3(kThreads), 0, st,
                       d, summ, states);
    return check_launch("fir states");
}

filt_status reduce_lti_run(const Dims &d, const double *part, void *ga, void *gb, bool f64,
                           hipStream_t st)
{
    const int64_t n = d.B * (d.N + d.M + 1);
    if (f64)
        FILT_LAUNCH("reduce_lti", (k_reduce_lti<double>), dim3(grid_for(n)), dim3(kThreads), 0, st, d,
                           part, (double *)ga, (double *)gb);
    else
        FILT_LAUNCH("reduce_lti", (k_reduce_lti<float>), dim3(grid_for(n)), dim3(kThreads), 0, st, d,
                           part, (float *)ga, (float *)gb);
    return check_launch("reduce");
}

}  // namespace filt_detail
