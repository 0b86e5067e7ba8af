// carry.hip -- dense launches of the carry scan (device bodies in carry.h)
// and the small reduction kernels of the backward.
#include "carry.h"

namespace filt_detail {
namespace {

__global__ void __launch_bounds__(320) k_carry_agg(Dims d, CarryArgs a)
{
    extern __shared__ double carry_stage[];
    const int64_t b = blockIdx.x / d.NB, blk = blockIdx.x % d.NB;
#define CALL(DB)                                                                                   \
    (d.tv ? carry_agg_body<DB, true>(d, a, b, blk, carry_stage)                                    \
          : carry_agg_body<DB, false>(d, a, b, blk, carry_stage))
    FILT_CARRY_DB(a.D, CALL);
#undef CALL
}

__global__ void __launch_bounds__(256)
k_carry_blocks(Dims d, CarryArgs a, const void *init, int init_f64)
{
    extern __shared__ double carry_stage[];
#define CALL(DB) carry_blocks_body<DB>(d, a, init, init_f64, blockIdx.x, carry_stage)
    FILT_CARRY_DB(a.D, CALL);
#undef CALL
}

__global__ void __launch_bounds__(256) k_carry_fill(Dims d, CarryArgs a)
{
    extern __shared__ double carry_stage[];
    const int64_t b = blockIdx.x / d.NB, blk = blockIdx.x % d.NB;
#define CALL(DB)                                                                                   \
    (d.tv ? carry_fill_body<DB, true>(d, a, b, blk, carry_stage)                                   \
          : carry_fill_body<DB, false>(d, a, b, blk, carry_stage))
    FILT_CARRY_DB(a.D, CALL);
#undef CALL
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

// Sum the per-chunk partials of time-invariant ga / gb over chunks: one
// workgroup per (channel, tap), strided partial sums then a fixed-shape tree
// in LDS (FP64, deterministic order).
template <typename io_t>
__global__ void __launch_bounds__(256)
k_reduce_lti(Dims d, const double *__restrict__ part, io_t *__restrict__ ga,
             io_t *__restrict__ gb)
{
    __shared__ double red[256];
    const int K = d.N + d.M + 1;
    const int64_t b = blockIdx.x / K;
    const int k = (int)(blockIdx.x % K);
    double acc = 0.0;
    for (int64_t c = threadIdx.x; c < d.C; c += blockDim.x)
        acc += part[(b * d.C + c) * K + k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (k < d.N) {
            if (ga != nullptr)
                ga[b * d.N + k] = (io_t)red[0];
        } else if (gb != nullptr) {
            gb[b * (d.M + 1) + (k - d.N)] = (io_t)red[0];
        }
    }
}

}  // namespace

filt_status carry_run(const Dims &d, const CarryArgs &a, const void *init, bool init_f64,
                      hipStream_t st)
{
    if (d.C < 2)
        return FILT_OK;
    if (a.D < 1 || a.D > kMaxD || a.D + a.R > 64)
        return fail(FILT_EUNSUPPORTED, "carry order %d (+%d)", a.D, a.R);
    const CarryRec cr = carry_rec(d.tv, a.D, a.R, a.SS);
    const int64_t agg_lds = (int64_t)stage_steps(cr.agg_len, d.G) * cr.agg_len;
    const int64_t blk_lds = (int64_t)stage_steps(cr.blk_len, d.NB) * cr.blk_len;
    const int64_t fill_lds = (int64_t)stage_steps(cr.fill_len, d.G) * cr.fill_len;
    const int agg_threads = ((a.D * (a.D + 1) + 63) / 64) * 64;
    FILT_LAUNCH("carry_agg", k_carry_agg, dim3((unsigned)(d.B * d.NB)), dim3(agg_threads),
                agg_lds * sizeof(double), st, d, a);
    FILT_LAUNCH("carry_blocks", k_carry_blocks, dim3((unsigned)d.B),
                dim3(carry_threads(blk_lds, a.D)), blk_lds * sizeof(double), st, d, a, init,
                (int)init_f64);
    FILT_LAUNCH("carry_fill", k_carry_fill, dim3((unsigned)(d.B * d.NB)),
                dim3(carry_threads(fill_lds, a.D + a.R)), fill_lds * sizeof(double), st, d, a);
    return check_launch("carry");
}

filt_status fir_states_run(const Dims &d, const double *summ, double *states, hipStream_t st)
{
    if (d.C < 2 || d.M == 0)
        return FILT_OK;
    FILT_LAUNCH("fir_states", k_fir_states, dim3(blocks_for(d.B * (d.C - 1) * d.M)), dim3(block_for(d.B * (d.C - 1) * d.M)),
                0, st, d, summ, states);
    return check_launch("fir states");
}

filt_status reduce_lti_run(const Dims &d, const double *part, void *ga, void *gb, bool f64,
                           hipStream_t st)
{
    const unsigned n = (unsigned)(d.B * (d.N + d.M + 1));
    const unsigned t = d.C >= 256 ? 256u : 64u;
    if (f64)
        FILT_LAUNCH("reduce_lti", (k_reduce_lti<double>), dim3(n), dim3(t), 0, st, d, part,
                    (double *)ga, (double *)gb);
    else
        FILT_LAUNCH("reduce_lti", (k_reduce_lti<float>), dim3(n), dim3(t), 0, st, d, part,
                    (float *)ga, (float *)gb);
    return check_launch("reduce");
}

}  // namespace filt_detail
