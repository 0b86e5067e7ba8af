// mr.hip -- the matrix recurrence v(n+1) = A v(n) + z(n), v(0) = v0, per
// channel: the state-space recursion of Sec. 2 Eq. 4 with the input already
// in state space (the operator of App. B), and its backward (Sec. 3.1 Eqs. 7
// and 9): the adjoint gz(n) = gv(n) + A^T gz(n+1) runs the same recursion
// with A transposed in reverse time; gv0 = A^T gz(0) and
// gA = sum_n gz(n) v(n)^T.
//
// One recurrence runs on one 16-lane DPP row: lane i owns state component
// v_i and row i of A (of A^T in the backward) in FP64 registers, and each
// step forms sum_j A_ij v_j with v_j broadcast from lane j of the row by
// row_newbcast inside v_fmac_f64_dpp, so a step is K FMAs per lane and the K^2
// work of the matrix-vector product is spread over the row.  The time axis is
// cut into chunks (the scan of Sec. 3.2): each row first solves its chunk
// from a zero state (the summary s_c), the time-invariant carry of the
// library (Kogge-Stone over chunks with powers of Phi = A^L) gives the state
// entering every chunk, and a second pass reruns each chunk from its
// entering state writing the output.  The backward runs the same kernels on
// the time-reversed signal with A^T; its apply pass also accumulates gA
// (each lane its row, v(n) broadcast across the row) into per-chunk FP64
// partial sums, and the chunk holding time 0 forms gv0.
#include "common.h"

namespace filt_detail {
namespace {

constexpr int kMrRow = 16;  // lanes per recurrence
constexpr int kMrBlk = 16;  // steps loaded per block (double-buffered)

struct MrDims {
    int64_t B, T, L, C;
    int K, layout;
};

// Element (b, t, i) of a [layout] state signal ([B][T][K] or [T][B][K]).
__device__ __forceinline__ int64_t mr_at(const MrDims &d, int64_t b, int64_t t, int i)
{
    return (d.layout == FILT_LAYOUT_TB ? t * d.B + b : b * d.T + t) * d.K + i;
}

#define MR_FMAC(j, acc, src, mul)                                                                  \
    "v_fmac_f64_dpp %" #acc ", %" #src ", %" #mul " row_newbcast:" #j                              \
    " row_mask:0xf bank_mask:0xf\n"

// sum_{j < KB} m[j] * src(lane j of the row), two interleaved accumulators.
// The DPP source is written by a VALU instruction just before: 2 wait states
// are required, hence the s_nop.  All 16 lanes of the row are active.
template <int KB>
__device__ __forceinline__ double row_dot(double src, const double (&m)[kMrRow])
{
    double a0 = 0.0, a1 = 0.0;
    if constexpr (KB == 4) {
        asm("s_nop 4\n" MR_FMAC(0, 0, 2, 3) MR_FMAC(1, 1, 2, 4) MR_FMAC(2, 0, 2, 5)
                MR_FMAC(3, 1, 2, 6)
            : "+v"(a0), "+v"(a1)
            : "v"(src), "v"(m[0]), "v"(m[1]), "v"(m[2]), "v"(m[3]));
    } else if constexpr (KB == 8) {
        asm("s_nop 4\n" MR_FMAC(0, 0, 2, 3) MR_FMAC(1, 1, 2, 4) MR_FMAC(2, 0, 2, 5)
                MR_FMAC(3, 1, 2, 6) MR_FMAC(4, 0, 2, 7) MR_FMAC(5, 1, 2, 8) MR_FMAC(6, 0, 2, 9)
                    MR_FMAC(7, 1, 2, 10)
            : "+v"(a0), "+v"(a1)
            : "v"(src), "v"(m[0]), "v"(m[1]), "v"(m[2]), "v"(m[3]), "v"(m[4]), "v"(m[5]),
              "v"(m[6]), "v"(m[7]));
    } else {
        static_assert(KB == 16, "row width");
        asm("s_nop 4\n" MR_FMAC(0, 0, 2, 3) MR_FMAC(1, 1, 2, 4) MR_FMAC(2, 0, 2, 5)
                MR_FMAC(3, 1, 2, 6) MR_FMAC(4, 0, 2, 7) MR_FMAC(5, 1, 2, 8) MR_FMAC(6, 0, 2, 9)
                    MR_FMAC(7, 1, 2, 10) MR_FMAC(8, 0, 2, 11) MR_FMAC(9, 1, 2, 12)
                        MR_FMAC(10, 0, 2, 13) MR_FMAC(11, 1, 2, 14) MR_FMAC(12, 0, 2, 15)
                            MR_FMAC(13, 1, 2, 16) MR_FMAC(14, 0, 2, 17) MR_FMAC(15, 1, 2, 18)
            : "+v"(a0), "+v"(a1)
            : "v"(src), "v"(m[0]), "v"(m[1]), "v"(m[2]), "v"(m[3]), "v"(m[4]), "v"(m[5]),
              "v"(m[6]), "v"(m[7]), "v"(m[8]), "v"(m[9]), "v"(m[10]), "v"(m[11]), "v"(m[12]),
              "v"(m[13]), "v"(m[14]), "v"(m[15]));
    }
    return a0 + a1;
}

// acc[j] += src(lane j of the row) * mul for j < KB (each lane a row of an
// outer product).
template <int KB>
__device__ __forceinline__ void row_outer(double src, double mul, double (&acc)[kMrRow])
{
    if constexpr (KB == 4) {
        asm("s_nop 4\n" MR_FMAC(0, 0, 4, 5) MR_FMAC(1, 1, 4, 5) MR_FMAC(2, 2, 4, 5)
                MR_FMAC(3, 3, 4, 5)
            : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3])
            : "v"(src), "v"(mul));
    } else if constexpr (KB == 8) {
        asm("s_nop 4\n" MR_FMAC(0, 0, 8, 9) MR_FMAC(1, 1, 8, 9) MR_FMAC(2, 2, 8, 9)
                MR_FMAC(3, 3, 8, 9) MR_FMAC(4, 4, 8, 9) MR_FMAC(5, 5, 8, 9) MR_FMAC(6, 6, 8, 9)
                    MR_FMAC(7, 7, 8, 9)
            : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]),
              "+v"(acc[5]), "+v"(acc[6]), "+v"(acc[7])
            : "v"(src), "v"(mul));
    } else {
        asm("s_nop 4\n" MR_FMAC(0, 0, 16, 17) MR_FMAC(1, 1, 16, 17) MR_FMAC(2, 2, 16, 17)
                MR_FMAC(3, 3, 16, 17) MR_FMAC(4, 4, 16, 17) MR_FMAC(5, 5, 16, 17)
                    MR_FMAC(6, 6, 16, 17) MR_FMAC(7, 7, 16, 17) MR_FMAC(8, 8, 16, 17)
                        MR_FMAC(9, 9, 16, 17) MR_FMAC(10, 10, 16, 17) MR_FMAC(11, 11, 16, 17)
                            MR_FMAC(12, 12, 16, 17) MR_FMAC(13, 13, 16, 17)
                                MR_FMAC(14, 14, 16, 17) MR_FMAC(15, 15, 16, 17)
            : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]),
              "+v"(acc[5]), "+v"(acc[6]), "+v"(acc[7]), "+v"(acc[8]), "+v"(acc[9]),
              "+v"(acc[10]), "+v"(acc[11]), "+v"(acc[12]), "+v"(acc[13]), "+v"(acc[14]),
              "+v"(acc[15])
            : "v"(src), "v"(mul));
    }
}

#undef MR_FMAC

// Lane i's matrix row: row i of A, or row i of A^T (column i of A); zero
// past K (so lanes i >= K keep a zero state).
__device__ __forceinline__ void mr_load_row(const MrDims &d, const float *A, int trans,
                                            int64_t b, int i, double (&m)[kMrRow])
{
    const float *Ab = A + b * (int64_t)d.K * d.K;
#pragma unroll
    for (int j = 0; j < kMrRow; ++j) {
        double v = 0.0;
        if (i < d.K && j < d.K)
            v = (double)(trans ? Ab[j * d.K + i] : Ab[i * d.K + j]);
        m[j] = v;
    }
}

// Row -> (channel, chunk): channels fastest in [T][B][K] (neighbouring rows
// read neighbouring K-rows), chunks fastest in [B][T][K].
__device__ __forceinline__ void mr_decode(const MrDims &d, int64_t row, int64_t nc, int64_t &b,
                                          int64_t &c)
{
    if (d.layout == FILT_LAYOUT_TB) {
        b = row % d.B;
        c = row / d.B;
    } else {
        c = row % nc;
        b = row / nc;
    }
}

// Run chunk c of the (REV: time-reversed) signal `in` from state v (lane i's
// component).  OUT: write each step's state to `out`.  GA: accumulate
// ga[j] += vprev_j(t) * v_i(t), vprev(t) the forward state before physical
// time t (vsig at t - 1, or v0 at t = 0).
template <int KB, bool REV, bool OUT, bool GA>
__device__ __forceinline__ void mr_chunk(const MrDims &d, int64_t b, int64_t c, int i,
                                         const double (&m)[kMrRow], double &v,
                                         const float *__restrict__ in, float *__restrict__ out,
                                         const float *__restrict__ vsig,
                                         const float *__restrict__ v0, double (&ga)[kMrRow])
{
    const int64_t t0 = c * d.L;
    const int64_t n = d.L < d.T - t0 ? d.L : d.T - t0;
    const bool own = i < d.K;
    auto phys = [&](int64_t t) { return REV ? d.T - 1 - t : t; };
    auto ld_in = [&](int64_t t) { return own ? in[mr_at(d, b, phys(t), i)] : 0.f; };
    auto ld_prev = [&](int64_t t) {
        const int64_t tp = phys(t);
        if (!own)
            return 0.f;
        if (tp > 0)
            return vsig[mr_at(d, b, tp - 1, i)];
        return v0 != nullptr ? v0[b * d.K + i] : 0.f;
    };
    auto step = [&](int64_t t, float xin, float xprev) {
        v = row_dot<KB>(v, m) + (double)xin;
        if constexpr (OUT) {
            if (own)
                out[mr_at(d, b, phys(t), i)] = (float)v;
        }
        if constexpr (GA)
            row_outer<KB>((double)xprev, v, ga);
    };
    const int64_t nb = n / kMrBlk;
    float cur[kMrBlk], curp[kMrBlk];
    if (nb > 0) {
#pragma unroll
        for (int s = 0; s < kMrBlk; ++s) {
            cur[s] = ld_in(t0 + s);
            curp[s] = GA ? ld_prev(t0 + s) : 0.f;
        }
    }
    for (int64_t k = 0; k < nb; ++k) {
        const int64_t tb = t0 + k * kMrBlk;
        float nxt[kMrBlk], nxtp[kMrBlk];
        const bool more = k + 1 < nb;
#pragma unroll
        for (int s = 0; s < kMrBlk; ++s) {
            nxt[s] = more ? ld_in(tb + kMrBlk + s) : 0.f;
            nxtp[s] = (GA && more) ? ld_prev(tb + kMrBlk + s) : 0.f;
        }
#pragma unroll
        for (int s = 0; s < kMrBlk; ++s)
            step(tb + s, cur[s], curp[s]);
#pragma unroll
        for (int s = 0; s < kMrBlk; ++s) {
            cur[s] = nxt[s];
            curp[s] = nxtp[s];
        }
    }
    for (int64_t t = t0 + nb * kMrBlk; t < t0 + n; ++t)
        step(t, ld_in(t), GA ? ld_prev(t) : 0.f);
}

// Zero-state summary of every chunk with a successor:
// summ[(b*C + c)*K + i] = state leaving chunk c from a zero entering state.
template <int KB, bool REV>
__global__ void __launch_bounds__(256)
k_mr_summary(MrDims d, const float *__restrict__ A, int trans, const float *__restrict__ in,
             double *__restrict__ summ)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = g / kMrRow;
    const int i = (int)(g % kMrRow);
    const int64_t nc = d.C - 1;
    if (row >= d.B * nc)
        return;
    int64_t b, c;
    mr_decode(d, row, nc, b, c);
    double m[kMrRow], ga[kMrRow];
    mr_load_row(d, A, trans, b, i, m);
    double v = 0.0;
    mr_chunk<KB, REV, false, false>(d, b, c, i, m, v, in, nullptr, nullptr, nullptr, ga);
    if (i < d.K)
        summ[(b * d.C + c) * d.K + i] = v;
}

// Phi = M^L (M = A or A^T): row (b, j) runs L steps from the unit state e_j;
// phi[(b*K + i)*K + j] = Phi_ij.
template <int KB>
__global__ void __launch_bounds__(256)
k_mr_phi(MrDims d, const float *__restrict__ A, int trans, double *__restrict__ phi)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = g / kMrRow;
    const int i = (int)(g % kMrRow);
    if (row >= d.B * d.K)
        return;
    const int64_t b = row / d.K;
    const int j = (int)(row % d.K);
    double m[kMrRow];
    mr_load_row(d, A, trans, b, i, m);
    double v = (i == j) ? 1.0 : 0.0;
    for (int64_t t = 0; t < d.L; ++t)
        v = row_dot<KB>(v, m);
    if (i < d.K)
        phi[(b * d.K + i) * d.K + j] = v;
}

// Output pass.  Forward (GA = false): chunk c from its entering state (v0
// for chunk 0), writing v.  Backward (REV, GA): the adjoint of the reversed
// chunk from its entering state (zero for the last physical chunk), writing
// gz, accumulating gA partials part[((b*C + c)*K + i)*K + j], and for the
// chunk holding time 0, gv0 = A^T gz(0).
template <int KB, bool REV, bool GA>
__global__ void __launch_bounds__(256)
k_mr_apply(MrDims d, const float *__restrict__ A, int trans, const float *__restrict__ in,
           const float *__restrict__ v0, const double *__restrict__ states,
           float *__restrict__ out, const float *__restrict__ vsig, double *__restrict__ part,
           float *__restrict__ gv0)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = g / kMrRow;
    const int i = (int)(g % kMrRow);
    if (row >= d.B * d.C)
        return;
    int64_t b, c;
    mr_decode(d, row, d.C, b, c);
    double m[kMrRow];
    mr_load_row(d, A, trans, b, i, m);
    double v = 0.0;
    if (i < d.K) {
        if (c > 0)
            v = states[(b * d.C + c) * d.K + i];
        else if (!GA && v0 != nullptr)
            v = (double)v0[b * d.K + i];
    }
    double ga[kMrRow];
#pragma unroll
    for (int j = 0; j < kMrRow; ++j)
        ga[j] = 0.0;
    mr_chunk<KB, REV, true, GA>(d, b, c, i, m, v, in, out, vsig, v0, ga);
    if constexpr (GA) {
        if (i < d.K) {
            double *o = part + ((b * d.C + c) * d.K + i) * d.K;
#pragma unroll
            for (int j = 0; j < kMrRow; ++j)
                if (j < d.K)
                    o[j] = ga[j];
        }
        if (c == d.C - 1 && gv0 != nullptr) {
            const double w = row_dot<KB>(v, m);  // A^T gz(0)
            if (i < d.K)
                gv0[b * d.K + i] = (float)w;
        }
    }
}

// gA[b][i][j] = sum over chunks of the partials: one workgroup per element,
// strided FP64 partial sums and a fixed-shape tree in LDS (deterministic).
__global__ void __launch_bounds__(256)
k_mr_reduce(MrDims d, const double *__restrict__ part, float *__restrict__ gA)
{
    __shared__ double red[256];
    const int64_t KK = (int64_t)d.K * d.K;
    const int64_t b = blockIdx.x / KK, e = blockIdx.x % KK;
    double s = 0.0;
    for (int64_t c = threadIdx.x; c < d.C; c += blockDim.x)
        s += part[(b * d.C + c) * KK + e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        gA[blockIdx.x] = (float)red[0];
}

__global__ void __launch_bounds__(256) k_mr_zero(float *__restrict__ p, int64_t n)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n)
        p[g] = 0.f;
}

filt_status mr_check(const filt_problem *p)
{
    if (p == nullptr)
        return fail(FILT_EINVAL, "problem is NULL");
    if (p->B < 0 || p->T < 0)
        return fail(FILT_EINVAL, "B and T must be >= 0");
    if (p->N < 1 || p->N > kMrRow)
        return fail(FILT_EUNSUPPORTED, "state size N must be 1..16 (got %d)", p->N);
    if (p->M != 0 || p->time_varying != 0)
        return fail(FILT_EINVAL, "the matrix recurrence takes M = 0 and time_varying = 0");
    if (p->layout != FILT_LAYOUT_TB && p->layout != FILT_LAYOUT_BT)
        return fail(FILT_EINVAL, "layout must be FILT_LAYOUT_TB or FILT_LAYOUT_BT");
    if (p->chunk < 0 || (p->chunk % 32) != 0)
        return fail(FILT_EINVAL, "chunk must be 0 or a positive multiple of 32 (got %d)",
                    p->chunk);
    return FILT_OK;
}

MrDims mr_dims(const filt_problem *p)
{
    MrDims d{};
    d.B = p->B;
    d.T = p->T;
    d.K = p->N;
    d.layout = p->layout;
    int64_t L = p->chunk;
    if (L == 0) {
        // about 16384 recurrences (rows of 16 lanes) over the whole problem:
        // a row's step waits on its loads, so short chunks (more rows in
        // flight) win until the carry over chunks dominates
        const int64_t want = std::max<int64_t>(1, (16384 + d.B - 1) / std::max<int64_t>(d.B, 1));
        L = (d.T + want - 1) / want;
        L = std::min<int64_t>(8192, std::max<int64_t>(32, (L + 31) / 32 * 32));
    }
    d.L = L;
    d.C = d.T > 0 ? (d.T + L - 1) / L : 0;
    return d;
}

struct MrWs {
    size_t summ, phi, agg, bstart, states, part, total;
};

MrWs mr_ws(const MrDims &d)
{
    MrWs w{};
    const int64_t nt = (d.C - 1 + 255) / 256;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    w.summ = take((size_t)(d.B * d.C * d.K) * sizeof(double));
    w.phi = take((size_t)(d.B * d.K * d.K) * sizeof(double));
    w.agg = take((size_t)(d.B * std::max<int64_t>(nt, 1) * d.K) * sizeof(double));
    w.bstart = take((size_t)(d.B * std::max<int64_t>(nt, 1) * d.K) * sizeof(double));
    w.states = take((size_t)(d.B * d.C * d.K) * sizeof(double));
    w.part = take((size_t)(d.B * d.C * d.K * d.K) * sizeof(double));
    w.total = 256 + off;
    return w;
}

unsigned rows_grid(int64_t rows)
{
    return (unsigned)((rows * kMrRow + 255) / 256);
}

// One direction: summaries, Phi, carry, then the output pass.
template <int KB, bool REV>
filt_status mr_run(const MrDims &d, const float *A, const float *in, const float *v0,
                   float *out, const float *vsig, float *gA, float *gv0, char *ws,
                   hipStream_t st)
{
    const MrWs w = mr_ws(d);
    double *summ = (double *)(ws + w.summ);
    double *phi = (double *)(ws + w.phi);
    double *states = (double *)(ws + w.states);
    double *part = (double *)(ws + w.part);
    const int trans = REV ? 1 : 0;
    if (d.C > 1) {
        FILT_LAUNCH("mr_summary", (k_mr_summary<KB, REV>), dim3(rows_grid(d.B * (d.C - 1))),
                    dim3(256), 0, st, d, A, trans, in, summ);
        FILT_LAUNCH("mr_phi", k_mr_phi<KB>, dim3(rows_grid(d.B * d.K)), dim3(256), 0, st, d, A,
                    trans, phi);
        filt_status s = check_launch("matrix recurrence summaries");
        if (s != FILT_OK)
            return s;
        Dims cd{};
        cd.B = d.B;
        cd.T = d.T;
        cd.L = d.L;
        cd.C = d.C;
        cd.N = d.K;
        cd.tv = false;
        CarryArgs a{};
        a.summ = summ;
        a.phi = phi;
        a.SS = d.K;
        a.soff = 0;
        a.D = d.K;
        a.R = 0;
        a.bwd = 0;
        a.agg = (double *)(ws + w.agg);
        a.bstart = (double *)(ws + w.bstart);
        a.states = states;
        s = carry_run(cd, a, REV ? nullptr : (const void *)v0, false, st);
        if (s != FILT_OK)
            return s;
    }
    FILT_LAUNCH("mr_apply", (k_mr_apply<KB, REV, REV>), dim3(rows_grid(d.B * d.C)), dim3(256),
                0, st, d, A, trans, in, v0, states, out, vsig, part, gv0);
    filt_status s = check_launch("matrix recurrence apply");
    if (s != FILT_OK || !REV || gA == nullptr)
        return s;
    FILT_LAUNCH("mr_reduce", k_mr_reduce, dim3((unsigned)(d.B * d.K * d.K)), dim3(256), 0, st,
                d, part, gA);
    return check_launch("matrix recurrence gA");
}

template <bool REV>
filt_status mr_dispatch(const MrDims &d, const float *A, const float *in, const float *v0,
                        float *out, const float *vsig, float *gA, float *gv0, char *ws,
                        hipStream_t st)
{
    if (d.K <= 4)
        return mr_run<4, REV>(d, A, in, v0, out, vsig, gA, gv0, ws, st);
    if (d.K <= 8)
        return mr_run<8, REV>(d, A, in, v0, out, vsig, gA, gv0, ws, st);
    return mr_run<16, REV>(d, A, in, v0, out, vsig, gA, gv0, ws, st);
}

filt_status mr_zero(float *p, int64_t n, hipStream_t st)
{
    if (p == nullptr || n <= 0)
        return FILT_OK;
    FILT_LAUNCH("mr_zero", k_mr_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    return check_launch("zero fill");
}

}  // namespace
}  // namespace filt_detail

using namespace filt_detail;

extern "C" {

filt_status filt_mr_workspace_bytes(const filt_problem *p, size_t *bytes)
{
    filt_status s = mr_check(p);
    if (s != FILT_OK)
        return s;
    if (bytes == nullptr)
        return fail(FILT_EINVAL, "bytes is NULL");
    if (p->B == 0 || p->T == 0) {
        *bytes = 0;
        return FILT_OK;
    }
    *bytes = mr_ws(mr_dims(p)).total;
    return FILT_OK;
}

filt_status filt_mr_forward(const filt_problem *p, const float *A, const float *v0,
                            const float *z, float *v, void *ws, size_t ws_bytes, void *stream)
{
    filt_status s = mr_check(p);
    if (s != FILT_OK)
        return s;
    if (p->B == 0 || p->T == 0)
        return FILT_OK;
    if (A == nullptr || z == nullptr || v == nullptr)
        return fail(FILT_EINVAL, "A, z and v are required");
    const MrDims d = mr_dims(p);
    const MrWs w = mr_ws(d);
    if (ws == nullptr || ws_bytes < w.total)
        return fail(FILT_EWORKSPACE, "workspace of %zu bytes needed, %zu given", w.total,
                    ws == nullptr ? (size_t)0 : ws_bytes);
    char *base = (char *)(((uintptr_t)ws + 255) & ~uintptr_t(255));
    return mr_dispatch<false>(d, A, z, v0, v, nullptr, nullptr, nullptr, base,
                              (hipStream_t)stream);
}

filt_status filt_mr_backward(const filt_problem *p, const float *A, const float *v0,
                             const float *v, const float *gv, float *gz, float *gA, float *gv0,
                             void *ws, size_t ws_bytes, void *stream)
{
    filt_status s = mr_check(p);
    if (s != FILT_OK)
        return s;
    hipStream_t st = (hipStream_t)stream;
    if (p->B == 0)
        return FILT_OK;
    if (p->T == 0) {
        s = mr_zero(gA, p->B * (int64_t)p->N * p->N, st);
        if (s == FILT_OK)
            s = mr_zero(gv0, p->B * (int64_t)p->N, st);
        return s;
    }
    if (A == nullptr || gv == nullptr || v == nullptr)
        return fail(FILT_EINVAL, "A, v and gv are required");
    const MrDims d = mr_dims(p);
    const MrWs w = mr_ws(d);
    if (ws == nullptr || ws_bytes < w.total)
        return fail(FILT_EWORKSPACE, "workspace of %zu bytes needed, %zu given", w.total,
                    ws == nullptr ? (size_t)0 : ws_bytes);
    char *base = (char *)(((uintptr_t)ws + 255) & ~uintptr_t(255));
    // the adjoint pass writes gz as it goes, so gz is always an output
    if (gz == nullptr)
        return fail(FILT_EINVAL, "gz is required (the adjoint pass writes it)");
    return mr_dispatch<true>(d, A, gv, v0, gz, v, gA, gv0, base, st);
}

}  // extern "C"
