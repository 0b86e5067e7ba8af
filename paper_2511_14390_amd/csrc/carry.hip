// carry.hip -- dense launches of the carry scan (device bodies in carry.h)
// and the small reduction kernels of the backward.
#include "carry.h"

namespace filt_detail {
namespace {

__global__ void __launch_bounds__(64) k_carry_agg(Dims d, CarryArgs a)
{
    carry_agg_body(d, a, blockIdx.x / d.NB, blockIdx.x % d.NB);
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
#define CALL(DB) carry_fill_body<DB>(d, a, b, blk, carry_stage)
    FILT_CARRY_DB(a.D, CALL);
#undef CALL
}

// ---------------------------------------------------------------------------
// Time-invariant carry: Phi is the same at every step, so the scan
// S_{c+1} = Phi S_c + s_c is a prefix sum under the operator of Sec. 3.2 with
// a fixed matrix, done Kogge-Stone style in log2 depth: at level l every
// step adds Phi^(2^l) times the running sum of the step 2^l before it.
// Steps are tiled 256 per workgroup (one thread per step):
//   (1) lti_agg    the sum over each tile (from a zero state);
//   (2) lti_tiles  the state at every tile start, one workgroup per channel,
//                  the same scan over tiles with Phi^256 (groups of 256 tiles
//                  one after another);
//   (3) lti_fill   each tile again from its start state, writing every state.
// The powers Phi^(2^l) are squared up in LDS by each workgroup (FP64).
// ---------------------------------------------------------------------------
constexpr int kLtiTile = 256;
constexpr int kLtiLevels = 8;  // log2(kLtiTile)

__host__ __device__ inline int64_t lti_tiles(const Dims &d) { return (d.C - 1 + kLtiTile - 1) / kLtiTile; }

template <int DB>
struct LtiShared {
    double pw[kLtiLevels][DB][DB];  // Phi^(2^(first + l))
    double tmp[DB][DB];
    double ex[DB][kLtiTile];        // exchange, component-major
    double st[DB];                  // state handed in
};

// pw[l] = Phi^(2^(first + l)), l < kLtiLevels; all threads take part.
template <int DB>
__device__ __forceinline__ void lti_powers(const double *phi, int D, int first, LtiShared<DB> &sh)
{
    const int e = threadIdx.x;
    const int i = e / DB, k = e % DB;
    const bool act = e < DB * DB;
    if (act)
        sh.tmp[i][k] = (i < D && k < D) ? phi[i * D + k] : 0.0;
    __syncthreads();
    for (int l = 0; l < first + kLtiLevels; ++l) {
        if (l >= first && act)
            sh.pw[l - first][i][k] = sh.tmp[i][k];
        if (l + 1 == first + kLtiLevels)
            break;
        double v = 0.0;
        if (act)
#pragma unroll
            for (int m = 0; m < DB; ++m)
                v += sh.tmp[i][m] * sh.tmp[m][k];
        __syncthreads();
        if (act)
            sh.tmp[i][k] = v;
        __syncthreads();
    }
    __syncthreads();
}

// Inclusive Kogge-Stone scan over the workgroup's 256 elements v (one per
// thread) with v_j += pw[l] v_{j - 2^l} at level l.
template <int DB>
__device__ __forceinline__ void lti_ks(LtiShared<DB> &sh, double (&v)[DB])
{
    const int j = threadIdx.x;
#pragma unroll 1
    for (int l = 0; l < kLtiLevels; ++l) {
        const int dist = 1 << l;
#pragma unroll
        for (int k = 0; k < DB; ++k)
            sh.ex[k][j] = v[k];
        __syncthreads();
        if (j >= dist) {
            double w[DB];
#pragma unroll
            for (int k = 0; k < DB; ++k)
                w[k] = sh.ex[k][j - dist];
#pragma unroll
            for (int i = 0; i < DB; ++i) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < DB; ++k)
                    acc += sh.pw[l][i][k] * w[k];
                v[i] += acc;
            }
        }
        __syncthreads();
    }
}

// s of the chunk crossed at step st (zero beyond the last step).
template <int DB>
__device__ __forceinline__ void lti_load_s(const Dims &d, const CarryArgs &a, int64_t b,
                                           int64_t st, double (&v)[DB])
{
    const int64_t steps = d.C - 1;
    const int64_t c = a.bwd ? d.C - 1 - st : st;
    const double *s = a.summ + (b * d.C + c) * a.SS + a.soff;
#pragma unroll
    for (int k = 0; k < DB; ++k)
        v[k] = (st < steps && k < a.D) ? s[k] : 0.0;
}

template <int DB>
__device__ __forceinline__ const double *lti_phi(const CarryArgs &a, int64_t b)
{
    return a.phi + b * ((int64_t)a.D * a.D + (int64_t)a.R * a.D);
}

template <int DB>
__global__ void __launch_bounds__(kLtiTile) k_lti_agg(Dims d, CarryArgs a)
{
    __shared__ LtiShared<DB> sh;
    const int64_t nt = lti_tiles(d);
    const int64_t b = blockIdx.x / nt, tile = blockIdx.x % nt;
    lti_powers<DB>(lti_phi<DB>(a, b), a.D, 0, sh);
    double v[DB];
    lti_load_s<DB>(d, a, b, tile * kLtiTile + threadIdx.x, v);
    lti_ks<DB>(sh, v);
    // only full tiles are summed (the last tile's sum is never needed)
    if (threadIdx.x == kLtiTile - 1)
        for (int k = 0; k < a.D; ++k)
            a.agg[(b * nt + tile) * a.D + k] = v[k];
}

template <int DB>
__global__ void __launch_bounds__(kLtiTile)
k_lti_tiles(Dims d, CarryArgs a, const void *init, int init_f64)
{
    __shared__ LtiShared<DB> sh;
    const int64_t nt = lti_tiles(d);
    const int64_t b = blockIdx.x;
    const int j = threadIdx.x;
    lti_powers<DB>(lti_phi<DB>(a, b), a.D, kLtiLevels, sh);  // Phi^(256 * 2^l)
    if (j < a.D) {
        double x0 = 0.0;
        if (init != nullptr)
            x0 = init_f64 ? ((const double *)init)[b * a.D + j]
                          : (double)((const float *)init)[b * a.D + j];
        sh.st[j] = x0;
        a.bstart[(b * nt) * a.D + j] = x0;
    }
    __syncthreads();
    for (int64_t g0 = 0; g0 + 1 < nt; g0 += kLtiTile) {
        // element j: the sum of tile g0 + j, plus Phi^256 times the state
        // entering the group for j = 0; the scan gives the state after it
        const int64_t t = g0 + j;
        double v[DB];
#pragma unroll
        for (int k = 0; k < DB; ++k)
            v[k] = (t + 1 < nt && k < a.D) ? a.agg[(b * nt + t) * a.D + k] : 0.0;
        if (j == 0) {
#pragma unroll
            for (int i = 0; i < DB; ++i) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < DB; ++k)
                    acc += sh.pw[0][i][k] * sh.st[k];
                v[i] += acc;
            }
        }
        lti_ks<DB>(sh, v);
        if (t + 1 < nt)
            for (int k = 0; k < a.D; ++k)
                a.bstart[(b * nt + t + 1) * a.D + k] = v[k];
        if (j == kLtiTile - 1)
            for (int k = 0; k < a.D; ++k)
                sh.st[k] = v[k];
        __syncthreads();
    }
}

template <int DB>
__global__ void __launch_bounds__(kLtiTile) k_lti_fill(Dims d, CarryArgs a, const void *init,
                                                       int init_f64)
{
    __shared__ LtiShared<DB> sh;
    __shared__ double Rm[kMaxD][DB];
    const int64_t nt = lti_tiles(d);
    const int64_t b = blockIdx.x / nt, tile = blockIdx.x % nt;
    const int j = threadIdx.x;
    const int D = a.D, R = a.R, SD = D + R;
    const double *phi = lti_phi<DB>(a, b);
    lti_powers<DB>(phi, D, 0, sh);
    if (j < D) {
        // the state entering the tile: from the tile pass, or the initial
        // state when the steps fit one tile
        double x0 = 0.0;
        if (nt > 1)
            x0 = a.bstart[(b * nt + tile) * D + j];
        else if (init != nullptr)
            x0 = init_f64 ? ((const double *)init)[b * D + j]
                          : (double)((const float *)init)[b * D + j];
        sh.st[j] = x0;
    }
    if (R > 0 && j < R * DB) {
        const int q = j / DB, k = j % DB;
        Rm[q][k] = k < D ? phi[D * D + q * D + k] : 0.0;
    }
    __syncthreads();
    const int64_t st = tile * kLtiTile + j;
    double v[DB];
    lti_load_s<DB>(d, a, b, st, v);
    if (j == 0) {
#pragma unroll
        for (int i = 0; i < DB; ++i) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < DB; ++k)
                acc += sh.pw[0][i][k] * sh.st[k];
            v[i] += acc;
        }
    }
    lti_ks<DB>(sh, v);
    const int64_t steps = d.C - 1;
    const int64_t cn = a.bwd ? d.C - 2 - st : st + 1;
    if (st < steps)
        for (int k = 0; k < D; ++k)
            a.states[(b * d.C + cn) * SD + k] = v[k];
    if (R > 0) {
        // FIR adjoint state across the same boundary: R S_in + r0, S_in the
        // state entering the chunk crossed at this step
#pragma unroll
        for (int k = 0; k < DB; ++k)
            sh.ex[k][j] = v[k];
        __syncthreads();
        if (st < steps) {
            double sin[DB];
#pragma unroll
            for (int k = 0; k < DB; ++k)
                sin[k] = j == 0 ? sh.st[k] : sh.ex[k][j - 1];
            const int64_t c = a.bwd ? d.C - 1 - st : st;
            const double *r0 = a.summ + (b * d.C + c) * a.SS + a.soff + D + (int64_t)R * D;
            for (int q = 0; q < R; ++q) {
                double acc = r0[q];
#pragma unroll
                for (int k = 0; k < DB; ++k)
                    acc += Rm[q][k] * sin[k];
                a.states[(b * d.C + cn) * SD + D + q] = acc;
            }
        }
    }
}

filt_status lti_carry_run(const Dims &d, const CarryArgs &a, const void *init, bool init_f64,
                          hipStream_t st)
{
    const int64_t nt = lti_tiles(d);
#define LTI_LAUNCH(DB)                                                                             \
    do {                                                                                           \
        if (nt > 1) {                                                                              \
            FILT_LAUNCH("carry_lti_agg", k_lti_agg<DB>, dim3((unsigned)(d.B * nt)),                \
                        dim3(kLtiTile), 0, st, d, a);                                              \
            FILT_LAUNCH("carry_lti_tiles", k_lti_tiles<DB>, dim3((unsigned)d.B), dim3(kLtiTile),   \
                        0, st, d, a, init, (int)init_f64);                                         \
        }                                                                                          \
        FILT_LAUNCH("carry_lti_fill", k_lti_fill<DB>, dim3((unsigned)(d.B * nt)), dim3(kLtiTile),  \
                    0, st, d, a, init, (int)init_f64);                                             \
    } while (0)
    FILT_CARRY_DB(a.D, LTI_LAUNCH);
#undef LTI_LAUNCH
    return check_launch("time-invariant carry");
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
    if (!d.tv)
        return lti_carry_run(d, a, init, init_f64, st);
    const CarryRec cr = carry_rec(a.D, a.SS);
    const int64_t blk_lds = (int64_t)stage_steps(cr.blk_len, d.NB) * cr.blk_len;
    const int64_t fill_lds = (int64_t)stage_steps(cr.fill_len, d.G) * cr.fill_len;
    FILT_LAUNCH("carry_agg", k_carry_agg, dim3((unsigned)(d.B * d.NB)), dim3(64), 0, st, d, a);
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
