// batched.h -- batched ragged filtering: many independent all-pole filters of
// different lengths and orders (per-sample coefficients, M = 0) in one pass.
//
// Segments are grouped by register bucket W (the orders N <= W share one
// kernel instantiation).  Every launch walks a device-side item list -- the
// (segment, chunk[, lane]) work of one bucket -- with a grid-stride loop over
// an occupancy-sized grid, so one launch per phase and bucket covers every
// filter whatever its length.  The per-item arithmetic is the same device
// code as the dense path (summary.h, carry.h, apply.h) applied to a
// one-channel [B, T] problem at the segment's offsets.
#pragma once

#include "apply.h"
#include "carry.h"
#include "stream.h"
#include "summary.h"

namespace filt_detail {

// Device-side description of one segment (offsets in elements / doubles).
struct SegDesc {
    int64_t x_off, T, a_off, ic_off;
    int64_t L, C, G, NB;
    int64_t summ_off, states_off, agg_off, bstart_off;
    int64_t tile_base, ntile;  // single-pass buckets: first tile record, tiles
    int32_t N, a_vec;
    int64_t hop;               // samples per coefficient row (1: per sample)
    FrameDiv fd;               // frame-held rows when fd.m != 0
};

// One unit of work: a chunk of a segment (and, for the summaries, one of the
// lanes that share that chunk's solves).
struct Item {
    int32_t seg, chunk, lane, pad;
};

}  // namespace filt_detail

// staged order-16 applies: need SegDesc and Item
#include "quadstage.h"

namespace filt_detail {

__device__ __forceinline__ Dims seg_dims(const SegDesc &s)
{
    Dims d{};
    d.B = 1;
    d.T = s.T;
    d.M = 0;
    d.N = s.N;
    d.tv = 1;
    d.hop = s.hop;
    d.fd = s.fd;
    d.F = s.fd.m != 0 ? (s.T + s.hop - 1) / s.hop : s.T;
    d.layout = FILT_LAYOUT_BT;
    d.has_b = 0;
    d.L = s.L;
    d.C = s.C;
    d.G = s.G;
    d.NB = s.NB;
    d.a_vec = s.a_vec;
    d.ga_vec = s.a_vec;
    return d;
}

__device__ __forceinline__ CarryArgs seg_carry(const SegDesc &s, double *ws, int bwd)
{
    CarryArgs a{};
    a.summ = ws + s.summ_off;
    a.phi = nullptr;
    a.SS = (int64_t)s.N * s.N + s.N;
    a.soff = (int64_t)s.N * s.N;
    a.D = s.N;
    a.R = 0;
    a.bwd = bwd;
    a.agg = ws + s.agg_off;
    a.bstart = ws + s.bstart_off;
    a.states = ws + s.states_off;
    return a;
}

#define FILT_GRID_STRIDE(g, n)                                                                     \
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < (n);                      \
         g += (int64_t)gridDim.x * blockDim.x)

// Forward summaries: items (seg, chunk, lane) for chunks 0..C-2.
template <int W, bool AV>
__global__ void __launch_bounds__(kThreads)
kb_fwd_summary(const SegDesc *__restrict__ segs, const Item *__restrict__ items, int64_t n,
               const float *__restrict__ x, const float *__restrict__ a, double *__restrict__ ws)
{
    constexpr int S = SummarySlots<W>::value;
    FILT_GRID_STRIDE(g, n)
    {
        const Item it = items[g];
        const SegDesc sd = segs[it.seg];
        const Dims d = seg_dims(sd);
        const float *ap = a + sd.a_off;
        fwd_summary_item<W, S, true, false, true, AV, float>(d, x + sd.x_off, nullptr, ap, ap, 0,
                                                             sd.N + 1, ws + sd.summ_off, nullptr,
                                                             0, it.chunk, it.lane);
    }
}

// Backward summaries: items (seg, chunk, lane); the chunk summarised is
// chunk + 1 (chunks 1..C-1 pass a state to an earlier chunk).
template <int W, bool AV>
__global__ void __launch_bounds__(kThreads)
kb_bwd_summary(const SegDesc *__restrict__ segs, const Item *__restrict__ items, int64_t n,
               const float *__restrict__ gy, const float *__restrict__ a, double *__restrict__ ws)
{
    constexpr int S = SummarySlots<W>::value;
    FILT_GRID_STRIDE(g, n)
    {
        const Item it = items[g];
        const SegDesc sd = segs[it.seg];
        const Dims d = seg_dims(sd);
        const float *ap = a + sd.a_off;
        bwd_summary_item<W, S, true, false, true, AV, float>(d, gy + sd.x_off, ap, ap, 0,
                                                             sd.N + 1, ws + sd.summ_off, nullptr,
                                                             0, it.chunk + 1, it.lane);
    }
}

// Forward apply: items (seg, chunk) for every chunk.
template <int W, bool AV>
__global__ void __launch_bounds__(kThreads)
kb_fwd_apply(const SegDesc *__restrict__ segs, const Item *__restrict__ items, int64_t n,
             const float *__restrict__ x, const float *__restrict__ a,
             const float *__restrict__ yi, const double *__restrict__ ws, float *__restrict__ y)
{
    FILT_GRID_STRIDE(g, n)
    {
        const Item it = items[g];
        const SegDesc sd = segs[it.seg];
        const Dims d = seg_dims(sd);
        const float *ap = a + sd.a_off;
        fwd_apply_item<W, true, false, AV, float, double>(
            d, x + sd.x_off, nullptr, ap, ap, yi != nullptr ? yi + sd.ic_off : nullptr,
            ws + sd.states_off, y + sd.x_off, 0, it.chunk);
    }
}

// Backward apply: items (seg, chunk); writes gx, the per-sample ga rows (GA)
// and, from chunk 0, gyi.
template <int W, bool AV, bool GA>
__global__ void __launch_bounds__(kThreads)
kb_bwd_apply(const SegDesc *__restrict__ segs, const Item *__restrict__ items, int64_t n,
             const float *__restrict__ gy, const float *__restrict__ y,
             const float *__restrict__ a, const float *__restrict__ yi,
             const double *__restrict__ ws, float *__restrict__ gx, float *__restrict__ ga,
             float *__restrict__ gyi)
{
    FILT_GRID_STRIDE(g, n)
    {
        const Item it = items[g];
        const SegDesc sd = segs[it.seg];
        const Dims d = seg_dims(sd);
        const float *ap = a + sd.a_off;
        bwd_apply_item<W, true, false, GA, false, AV, float, double>(
            d, gy + sd.x_off, nullptr, nullptr, y + sd.x_off,
            yi != nullptr ? yi + sd.ic_off : nullptr, ap, ap, ws + sd.states_off,
            gx != nullptr ? gx + sd.x_off : nullptr, nullptr, GA ? ga + sd.a_off : nullptr, nullptr,
            gyi != nullptr ? gyi + sd.ic_off : nullptr, nullptr, nullptr, 0, it.chunk);
    }
}

// Order-16 bucket applies on lane quads (apply.h): four lanes per item.
// The backward writes ybar into gx (gx = ybar without b) and gyi from chunk 0.
template <bool AV>
__global__ void __launch_bounds__(kThreads)
kb_fwd_apply_quad(const SegDesc *__restrict__ segs, const Item *__restrict__ items, int64_t n,
                  const float *__restrict__ x, const float *__restrict__ a,
                  const float *__restrict__ yi, const double *__restrict__ ws,
                  float *__restrict__ y)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((idx >> 2) >= n)  // whole quads
        return;
    const Item it = items[idx >> 2];
    const SegDesc sd = segs[it.seg];
    const Dims d = seg_dims(sd);
    const float *yis = yi != nullptr ? yi + sd.ic_off : nullptr;
    if (((int64_t)it.chunk + 1) * d.L > d.T)
        fwd_apply_quad<AV, false, true>(d, x + sd.x_off, (const float *)nullptr, a + sd.a_off,
                                        yis, ws + sd.states_off, y + sd.x_off, 0, it.chunk,
                                        (int)(idx & 3));
    else
        fwd_apply_quad<AV, false, false>(d, x + sd.x_off, (const float *)nullptr, a + sd.a_off,
                                         yis, ws + sd.states_off, y + sd.x_off, 0, it.chunk,
                                         (int)(idx & 3));
}

template <bool AV>
__global__ void __launch_bounds__(kThreads)
kb_bwd_apply_quad(const SegDesc *__restrict__ segs, const Item *__restrict__ items, int64_t n,
                  const float *__restrict__ gy, const float *__restrict__ a,
                  const double *__restrict__ ws, float *gx, float *__restrict__ gyi)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((idx >> 2) >= n)
        return;
    const Item it = items[idx >> 2];
    const SegDesc sd = segs[it.seg];
    const Dims d = seg_dims(sd);
    float *gxs = gx + sd.x_off;
    float *gyis = gyi != nullptr ? gyi + sd.ic_off : nullptr;
    if (((int64_t)it.chunk + 1) * d.L > d.T)
        bwd_apply_quad<AV, false, true, false>(d, gy + sd.x_off, (const float *)nullptr,
                                               a + sd.a_off, ws + sd.states_off, gxs, gyis, gxs,
                                               (const float *)nullptr, (const float *)nullptr,
                                               (float *)nullptr, 0, it.chunk, (int)(idx & 3));
    else
        bwd_apply_quad<AV, false, false, false>(d, gy + sd.x_off, (const float *)nullptr,
                                                a + sd.a_off, ws + sd.states_off, gxs, gyis, gxs,
                                                (const float *)nullptr, (const float *)nullptr,
                                                (float *)nullptr, 0, it.chunk, (int)(idx & 3));
}

// Staged applies (stream.h) over the items (seg, chunk) of one bucket, one
// wavefront per 64 items; Lc is the bucket's chunk length.
template <int W, bool VEC>
__global__ void __launch_bounds__(64)
kb_stream_fwd(const SegDesc *__restrict__ segs, const Item *__restrict__ items, int64_t n,
              int64_t Lc, const float *__restrict__ x, const float *__restrict__ a,
              const float *__restrict__ yi, const double *__restrict__ ws, float *__restrict__ y)
{
    __shared__ StreamLds<W> L;
    const int i = threadIdx.x;
    const int64_t g = (int64_t)blockIdx.x * 64 + i;
    const bool act = g < n;
    SegDesc sd{};
    int64_t c = 0;
    if (act) {
        const Item it = items[g];
        sd = segs[it.seg];
        c = it.chunk;
    }
    const int64_t t0 = c * Lc;
    L.osig[i] = act ? sd.x_off + t0 : 0;
    L.oout[i] = L.osig[i];
    L.ocoef[i] = act ? sd.a_off + (sd.fd.m != 0 ? (int64_t)frame_of(sd.fd, (uint32_t)t0) : t0) *
                               sd.N
                     : 0;
    stream_set_rows(L, i, t0, sd.fd);
    L.ln[i] = act ? min(Lc, sd.T - t0) : 0;
    L.lN[i] = act ? sd.N : 0;
    double h0[W];
#pragma unroll
    for (int q = 0; q < W; ++q) {
        double v = 0.0;
        if (act && q < sd.N)
            v = c == 0 ? (yi != nullptr ? (double)yi[sd.ic_off + q] : 0.0)
                       : ws[sd.states_off + c * sd.N + q];
        h0[q] = v;
    }
    __syncthreads();
    stream_forward<W, VEC>(L, StreamPtrs{x, a, y}, Lc, h0);
}

// Writes ybar into gx (equal for b = [1]) and, from chunk 0, gyi.
template <int W, bool VEC>
__global__ void __launch_bounds__(64)
kb_stream_bwd(const SegDesc *__restrict__ segs, const Item *__restrict__ items, int64_t n,
              int64_t Lc, const float *__restrict__ gy, const float *__restrict__ a,
              const double *__restrict__ ws, float *__restrict__ gx, float *__restrict__ gyi)
{
    __shared__ StreamLds<W> L;
    const int i = threadIdx.x;
    const int64_t g = (int64_t)blockIdx.x * 64 + i;
    const bool act = g < n;
    SegDesc sd{};
    int64_t c = 0;
    if (act) {
        const Item it = items[g];
        sd = segs[it.seg];
        c = it.chunk;
    }
    const int64_t t0 = c * Lc;
    L.osig[i] = act ? sd.x_off + t0 : 0;
    L.oout[i] = L.osig[i];
    L.ocoef[i] = act ? sd.a_off + (sd.fd.m != 0 ? (int64_t)frame_of(sd.fd, (uint32_t)t0) : t0) *
                               sd.N
                     : 0;
    stream_set_rows(L, i, t0, sd.fd);
    L.ln[i] = act ? min(Lc, sd.T - t0) : 0;
    L.lN[i] = act ? sd.N : 0;
    double s0[W];
#pragma unroll
    for (int q = 0; q < W; ++q)
        s0[q] = (act && q < sd.N && c + 1 < sd.C) ? ws[sd.states_off + c * sd.N + q] : 0.0;
    __syncthreads();
    stream_backward<W, VEC>(L, StreamPtrs{gy, a, gx}, Lc, s0);
    if (act && c == 0 && gyi != nullptr)
#pragma unroll
        for (int q = 0; q < W; ++q)
            if (q < sd.N)
                gyi[sd.ic_off + q] = (float)s0[q];
}

// Per-sample ga from the stored adjoint, one workgroup per item:
// ga_k[t] = -ybar[t] y[t-k], y[-j] = yi[j-1] (Eq. 8 per sample).  One copy
// per order bucket (W) so each bucket's unit owns its kernel.
template <int W>
__global__ void __launch_bounds__(256)
kb_coef_grads(const SegDesc *__restrict__ segs, const Item *__restrict__ items, int64_t Lc,
              const float *__restrict__ ybar, const float *__restrict__ y,
              const float *__restrict__ yi, float *__restrict__ ga, int ga_aligned)
{
    const Item it = items[blockIdx.x];
    const SegDesc sd = segs[it.seg];
    const int N = sd.N;
    if (N == 0 || sd.fd.m != 0)
        return;  // frame-held rows take kb_frame_grads
    const int64_t t0 = (int64_t)it.chunk * Lc;
    const int64_t n = min(Lc, sd.T - t0);
    const int G = (N + 3) / 4;
    // whole float4 rows only when every row starts on a 16-byte boundary: a
    // 16-byte aligned ga base (checked on the host), N and a_off multiples of 4
    const bool vec = ga_aligned && (N % 4) == 0 && (sd.a_off % 4) == 0;
    for (int64_t u = threadIdx.x; u < n * G; u += blockDim.x) {
        const int64_t t = t0 + u / G;
        const int q = (int)(u % G);
        const float v = -ybar[sd.x_off + t];
        float r[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int k = 4 * q + jj + 1;
            float yv = 0.f;
            if (k <= N) {
                if (t - k >= 0)
                    yv = y[sd.x_off + t - k];
                else if (yi != nullptr)
                    yv = yi[sd.ic_off + (k - t - 1)];
            }
            r[jj] = v * yv;
        }
        float *o = ga + sd.a_off + t * N + 4 * q;
        // written once, not read again here: stream past the caches
        if (vec) {
            using f4 = float __attribute__((ext_vector_type(4)));
            const f4 v4 = {r[0], r[1], r[2], r[3]};
            __builtin_nontemporal_store(v4, reinterpret_cast<f4 *>(o));
        } else {
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
                if (4 * q + jj < N)
                    __builtin_nontemporal_store(r[jj], o + jj);
        }
    }
}

// Frame-held rows: ga of the bucket's frame-held segments from the stored
// adjoint, ga_k[f] = -sum_{t in f} ybar[t] y[t-k] (Sec. 3.1 Eq. 8 summed over
// the frame).  One wavefront (workgroup) per item (segment, first frame,
// frames <= 64).
static __global__ void __launch_bounds__(64)
kb_frame_grads(const SegDesc *__restrict__ segs, const Item *__restrict__ items,
               const float *__restrict__ ybar, const float *__restrict__ y,
               const float *__restrict__ yi, float *__restrict__ ga)
{
    __shared__ float lds[kFrameLds];
    const Item it = items[blockIdx.x];
    const SegDesc sd = segs[it.seg];
    frame_sums_wave(ybar + sd.x_off, y + sd.x_off, yi != nullptr ? yi + sd.ic_off : nullptr,
                    sd.N, 1, sd.N, -1.0, sd.T, sd.hop, (int64_t)it.chunk, it.lane,
                    ga + sd.a_off, lds, (int)threadIdx.x);
}

// Launch geometry of a grid-stride kernel over n items.
inline void persistent_grid(int64_t n, unsigned &blocks, unsigned &threads)
{
    threads = block_for(n);
    const int64_t want = (n + threads - 1) / threads;
    const int64_t cap = kCUs * (threads == 64 ? 16 : 4);
    blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, cap));
}

// acc + v * (lane s's xrow of the row), the broadcast folded into the FMA
// (row_newbcast); FIRST: xrow was written by the step's own block, so the
// two wait states a DPP read needs after a VALU write come first.
template <int s, bool FIRST>
__device__ __forceinline__ double row_bcast_fma(double acc, double xrow, double v)
{
#define FILT_XB_ASM(n) "v_fmac_f64_dpp %0, %1, %2 row_newbcast:" #n " row_mask:0xf bank_mask:0xf"
#define FILT_XB_CASE(n)                                                                            \
    if constexpr (s == n) {                                                                        \
        if constexpr (FIRST)                                                                       \
            asm("s_nop 1\n" FILT_XB_ASM(n) : "+v"(acc) : "v"(xrow), "v"(v));                      \
        else                                                                                       \
            asm(FILT_XB_ASM(n) : "+v"(acc) : "v"(xrow), "v"(v));                                   \
    }
    FILT_XB_CASE(0) FILT_XB_CASE(1) FILT_XB_CASE(2) FILT_XB_CASE(3) FILT_XB_CASE(4)
    FILT_XB_CASE(5) FILT_XB_CASE(6) FILT_XB_CASE(7) FILT_XB_CASE(8) FILT_XB_CASE(9)
    FILT_XB_CASE(10) FILT_XB_CASE(11) FILT_XB_CASE(12) FILT_XB_CASE(13) FILT_XB_CASE(14)
    FILT_XB_CASE(15)
#undef FILT_XB_CASE
#undef FILT_XB_ASM
    return acc;
}

// Order-16 bucket summaries by duality, one 16-lane DPP row per chunk and
// no driven solve (sixteen chunks per 256-thread workgroup, no LDS, no
// barriers).  Forward: row lane i runs the adjoint solve seeded with
// s_{i+1} = 1 at the chunk's end (the cotangent of the state component i
// leaving the chunk); its adjoint state at the chunk's start is row i of
// Phi_c, and sum_t ybar_i[t] x[t] is s_c[i].  Adjoint: row lane j runs the
// forward solve from the unit state e_j; its final state is row j of the
// chunk's adjoint map (Phi_c transposed) and sum_t gy[t] y_j[t] is that
// map's driven part.  Coefficients are read 16 steps ahead; the signal one
// 16-step block ahead, lane j holding step j of the block, its value
// broadcast to the row inside the accumulating FMA.
template <bool FULL>
__global__ void __launch_bounds__(256)
kb_fwd_summary_dual(const SegDesc *__restrict__ segs, const Item *__restrict__ items, int64_t n,
                    const float *__restrict__ x, const float *__restrict__ a,
                    double *__restrict__ ws)
{
    const int row = threadIdx.x >> 4, j = threadIdx.x & 15;
    for (int64_t first = (int64_t)blockIdx.x * 16; first < n; first += (int64_t)gridDim.x * 16) {
        const int64_t g = first + row;
        if (g >= n)
            continue;  // the whole row: its DPP broadcasts stay inside it
        const Item it = items[g];
        const SegDesc sd = segs[it.seg];
        const Dims d = seg_dims(sd);
        const int64_t c = it.chunk;  // chunks 0..C-2 are whole
        const RowCoef<float, FULL> rc = row_coef<float, FULL>(d, a + sd.a_off, 0, c, j);
        const float *xp = x + sd.x_off + c * d.L;
        const int L = (int)d.L;
        double ss[16];
#pragma unroll
        for (int e = 0; e < 16; ++e)
            ss[e] = (rc.live && e == ((j + 2) & 15)) ? 1.0 : 0.0;
        float cb[16];
#pragma unroll
        for (int s = 0; s < 16; ++s)
            cb[s] = *rc.at(L - 16 + s);
        // lane j holds x of step rel + j of the block; step s reads lane s's
        float xn = xp[L - 16 + j];
        double acc = 0.0;
        for (int rel = L - 16; rel >= 0; rel -= 16) {
            const double xrow = (double)xn;
            xn = xp[max(rel - 16, 0) + j];
            static_for<16>([&](auto I) {
                constexpr int s = 15 - decltype(I)::value;
                const double cf = rc.cvt(cb[s]);
                const int nx = max(rel - 16 + s, 0);
                cb[s] = *rc.at(nx);
                const double sv = ss[(1 - s) & 15];
                row_bwd_step<s>(cf, ss);
                acc = row_bcast_fma<s, s == 15>(acc, xrow, sv);
                __builtin_amdgcn_sched_barrier(0);
            });
        }
        if (rc.live) {
            const int N = d.N;
            double *o = ws + sd.summ_off + c * ((int64_t)N * N + N);
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (i < N)
                    o[j * N + i] = ss[(i + 2) & 15];
            o[(int64_t)N * N + j] = acc;
        }
    }
}

template <bool FULL>
__global__ void __launch_bounds__(256)
kb_bwd_summary_dual(const SegDesc *__restrict__ segs, const Item *__restrict__ items, int64_t n,
                    const float *__restrict__ gy, const float *__restrict__ a,
                    double *__restrict__ ws)
{
    const int row = threadIdx.x >> 4, j = threadIdx.x & 15;
    for (int64_t first = (int64_t)blockIdx.x * 16; first < n; first += (int64_t)gridDim.x * 16) {
        const int64_t g = first + row;
        if (g >= n)
            continue;
        const Item it = items[g];
        const SegDesc sd = segs[it.seg];
        const Dims d = seg_dims(sd);
        const int64_t c = it.chunk + 1;  // chunks 1..C-1 pass a state to an earlier chunk
        const RowCoef<float, FULL> rc = row_coef<float, FULL>(d, a + sd.a_off, 0, c, j);
        const float *gp = gy + sd.x_off + c * d.L;
        const int L = (int)d.L;
        // a last chunk cut short by the signal's end: steps past T take zero
        // coefficients and zero gy (reads clamped to its last sample)
        const int valid = (int)min<int64_t>(d.L, d.T - c * d.L);
        double h[16];
#pragma unroll
        for (int e = 0; e < 16; ++e)
            h[e] = (rc.live && e == ((-1 - j) & 15)) ? 1.0 : 0.0;
        float cb[16];
#pragma unroll
        for (int s = 0; s < 16; ++s)
            cb[s] = *rc.at(min(s, valid - 1));
        // lane j holds gy of step rel + j of the block (zero past the
        // signal's end); step s reads lane s's
        float gn = gp[min(j, valid - 1)];
        double acc = 0.0;
        for (int rel = 0; rel < L; rel += 16) {
            const double grow = rel + j < valid ? (double)gn : 0.0;
            gn = gp[min(rel + 16 + j, valid - 1)];
            static_for<16>([&](auto I) {
                constexpr int s = decltype(I)::value;
                const bool in = rel + s < valid;
                const double cf = in ? rc.cvt(cb[s]) : 0.0;
                const int nx = min(rel + 16 + s, valid - 1);
                cb[s] = *rc.at(nx);
                h[s] = row_fwd_step<s>(cf, h);
                acc = row_bcast_fma<s, s == 0>(acc, grow, h[s]);
                __builtin_amdgcn_sched_barrier(0);
            });
        }
        if (rc.live) {
            const int N = d.N;
            double *o = ws + sd.summ_off + c * ((int64_t)N * N + N);
            // a chunk cut short only ever sees a zero state from above
            const bool whole = valid == L;
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (i < N)
                    o[j * N + i] = whole ? h[15 - i] : 0.0;
            o[(int64_t)N * N + j] = acc;
        }
    }
}

inline unsigned dual_groups(int64_t n)
{
    const int64_t want = (n + 15) / 16;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, kCUs * 8));
}

// Launch names carry the order bucket ("..._w16"), so per-kernel timings
// and byte counts can be attributed to one bucket's samples.
#define FILT_BNAME(KIND, W)                                                                        \
    ((W) == 1 ? KIND "_w1" : (W) == 2 ? KIND "_w2" : (W) == 4 ? KIND "_w4" : (W) == 8 ? KIND "_w8" \
                                                                                : KIND "_w16")

// One bucket's launches (defined per bucket in generated units).
struct BucketArgs {
    const SegDesc *segs;
    const Item *sum_items;
    int64_t sum_n;
    const Item *app_items;
    int64_t app_n;
    int av;
};

template <int W>
filt_status batched_fwd_summary(const BucketArgs &b, const float *x, const float *a, double *ws,
                                hipStream_t st)
{
    if (b.sum_n == 0)
        return FILT_OK;
    if constexpr (W == 16) {
        if (b.av)
            FILT_LAUNCH(FILT_BNAME("batched_fwd_summary", W), kb_fwd_summary_dual<true>,
                        dim3(dual_groups(b.sum_n)), dim3(256), 0, st, b.segs, b.sum_items, b.sum_n,
                        x, a, ws);
        else
            FILT_LAUNCH(FILT_BNAME("batched_fwd_summary", W), kb_fwd_summary_dual<false>,
                        dim3(dual_groups(b.sum_n)), dim3(256), 0, st, b.segs, b.sum_items, b.sum_n,
                        x, a, ws);
        return check_launch("batched forward summary");
    }
    unsigned g, t;
    persistent_grid(b.sum_n, g, t);
    if (b.av)
        FILT_LAUNCH(FILT_BNAME("batched_fwd_summary", W), (kb_fwd_summary<W, true>), dim3(g), dim3(t), 0, st,
                    b.segs, b.sum_items, b.sum_n, x, a, ws);
    else
        FILT_LAUNCH(FILT_BNAME("batched_fwd_summary", W), (kb_fwd_summary<W, false>), dim3(g), dim3(t), 0, st,
                    b.segs, b.sum_items, b.sum_n, x, a, ws);
    return check_launch("batched forward summary");
}

template <int W>
filt_status batched_bwd_summary(const BucketArgs &b, const float *gy, const float *a, double *ws,
                                hipStream_t st)
{
    if (b.sum_n == 0)
        return FILT_OK;
    if constexpr (W == 16) {
        if (b.av)
            FILT_LAUNCH(FILT_BNAME("batched_bwd_summary", W), kb_bwd_summary_dual<true>,
                        dim3(dual_groups(b.sum_n)), dim3(256), 0, st, b.segs, b.sum_items, b.sum_n,
                        gy, a, ws);
        else
            FILT_LAUNCH(FILT_BNAME("batched_bwd_summary", W), kb_bwd_summary_dual<false>,
                        dim3(dual_groups(b.sum_n)), dim3(256), 0, st, b.segs, b.sum_items, b.sum_n,
                        gy, a, ws);
        return check_launch("batched backward summary");
    }
    unsigned g, t;
    persistent_grid(b.sum_n, g, t);
    if (b.av)
        FILT_LAUNCH(FILT_BNAME("batched_bwd_summary", W), (kb_bwd_summary<W, true>), dim3(g), dim3(t), 0, st,
                    b.segs, b.sum_items, b.sum_n, gy, a, ws);
    else
        FILT_LAUNCH(FILT_BNAME("batched_bwd_summary", W), (kb_bwd_summary<W, false>), dim3(g), dim3(t), 0, st,
                    b.segs, b.sum_items, b.sum_n, gy, a, ws);
    return check_launch("batched backward summary");
}

template <int W>
filt_status batched_fwd_apply(const BucketArgs &b, const float *x, const float *a,
                              const float *yi, const double *ws, float *y, hipStream_t st)
{
    if (b.app_n == 0)
        return FILT_OK;
    if constexpr (W == 16) {
        const dim3 grid((unsigned)((b.app_n * 4 + kThreads - 1) / kThreads));
        const dim3 sgrid((unsigned)((b.app_n + kQuadChains - 1) / kQuadChains));
        if (b.av)
            FILT_LAUNCH(FILT_BNAME("batched_fwd_apply", W), kb_fwd_apply_quad_staged, sgrid,
                        dim3(64), 0, st, b.segs, b.app_items, b.app_n, x, a, yi, ws, y);
        else
            FILT_LAUNCH(FILT_BNAME("batched_fwd_apply", W), kb_fwd_apply_quad<false>, grid, dim3(kThreads), 0,
                        st, b.segs, b.app_items, b.app_n, x, a, yi, ws, y);
        return check_launch("batched forward apply");
    }
    unsigned g, t;
    persistent_grid(b.app_n, g, t);
    if (b.av)
        FILT_LAUNCH(FILT_BNAME("batched_fwd_apply", W), (kb_fwd_apply<W, true>), dim3(g), dim3(t), 0, st, b.segs,
                    b.app_items, b.app_n, x, a, yi, ws, y);
    else
        FILT_LAUNCH(FILT_BNAME("batched_fwd_apply", W), (kb_fwd_apply<W, false>), dim3(g), dim3(t), 0, st,
                    b.segs, b.app_items, b.app_n, x, a, yi, ws, y);
    return check_launch("batched forward apply");
}

template <int W>
filt_status batched_bwd_apply(const BucketArgs &b, const float *gy, const float *y,
                              const float *a, const float *yi, const double *ws, float *gx,
                              float *ga, float *gyi, hipStream_t st)
{
    if (b.app_n == 0)
        return FILT_OK;
    unsigned g, t;
    persistent_grid(b.app_n, g, t);
#define FILT_KB_BWD(AVV, GAV)                                                                      \
    FILT_LAUNCH(FILT_BNAME("batched_bwd_apply", W), (kb_bwd_apply<W, AVV, GAV>), dim3(g), dim3(t), 0, st, b.segs, \
                b.app_items, b.app_n, gy, y, a, yi, ws, gx, ga, gyi)
    if (b.av) {
        if (ga != nullptr)
            FILT_KB_BWD(true, true);
        else
            FILT_KB_BWD(true, false);
    } else {
        if (ga != nullptr)
            FILT_KB_BWD(false, true);
        else
            FILT_KB_BWD(false, false);
    }
#undef FILT_KB_BWD
    return check_launch("batched backward apply");
}

// Buckets whose rows are at most 8 taps take the staged applies.
template <int W>
constexpr bool kStreamBucket = W <= 8;

template <int W>
filt_status batched_stream_fwd(const BucketArgs &b, int64_t Lc, const float *x, const float *a,
                               const float *yi, const double *ws, float *y, hipStream_t st)
{
    if (b.app_n == 0)
        return FILT_OK;
    const dim3 grid((unsigned)((b.app_n + 63) / 64));
    if (b.av && W % 4 == 0)
        FILT_LAUNCH(FILT_BNAME("batched_stream_fwd", W), (kb_stream_fwd<W, (W % 4 == 0)>), grid, dim3(64), 0, st,
                    b.segs, b.app_items, b.app_n, Lc, x, a, yi, ws, y);
    else
        FILT_LAUNCH(FILT_BNAME("batched_stream_fwd", W), (kb_stream_fwd<W, false>), grid, dim3(64), 0, st, b.segs,
                    b.app_items, b.app_n, Lc, x, a, yi, ws, y);
    return check_launch("batched staged forward apply");
}

template <int W>
filt_status batched_stream_bwd(const BucketArgs &b, int64_t Lc, const float *gy, const float *y,
                               const float *a, const float *yi, const double *ws, float *gx,
                               float *ga, float *gyi, hipStream_t st)
{
    if (b.app_n == 0)
        return FILT_OK;
    const dim3 grid((unsigned)((b.app_n + 63) / 64));
    if (b.av && W % 4 == 0)
        FILT_LAUNCH(FILT_BNAME("batched_stream_bwd", W), (kb_stream_bwd<W, (W % 4 == 0)>), grid, dim3(64), 0, st,
                    b.segs, b.app_items, b.app_n, Lc, gy, a, ws, gx, gyi);
    else
        FILT_LAUNCH(FILT_BNAME("batched_stream_bwd", W), (kb_stream_bwd<W, false>), grid, dim3(64), 0, st, b.segs,
                    b.app_items, b.app_n, Lc, gy, a, ws, gx, gyi);
    if (ga != nullptr)
        FILT_LAUNCH(FILT_BNAME("batched_coef_grads", W), kb_coef_grads<W>, dim3((unsigned)b.app_n), dim3(256), 0, st,
                    b.segs, b.app_items, Lc, gx, y, yi, ga, (int)((uintptr_t)ga % 16 == 0));
    return check_launch("batched staged backward apply");
}

// Order-16 bucket backward: the apply (quads) writes gx (= ybar); with
// full-width rows the staged adjoint also forms the per-sample ga rows,
// otherwise the per-item pass forms them from gx.
template <int W>
filt_status batched_bwd_split(const BucketArgs &b, int64_t Lc, const float *gy, const float *y,
                              const float *a, const float *yi, const double *ws, float *gx,
                              float *ga, float *gyi, hipStream_t st)
{
    filt_status s = FILT_OK;
    if (b.app_n == 0)
        return s;
    if constexpr (W == 16) {
        const dim3 grid((unsigned)((b.app_n * 4 + kThreads - 1) / kThreads));
        const dim3 sgrid((unsigned)((b.app_n + kQuadChains - 1) / kQuadChains));
        // full-width rows: the staged adjoint, forming the per-sample ga rows
        // itself when their base is 16-byte aligned
        const bool fused = ga != nullptr && (uintptr_t)ga % 16 == 0;
        if (b.av && fused) {
            FILT_LAUNCH(FILT_BNAME("batched_bwd_apply", W), kb_bwd_apply_quad_staged<true>, sgrid,
                        dim3(64), 0, st, b.segs, b.app_items, b.app_n, gy, a, ws, gx, gyi, y, yi,
                        ga);
            return check_launch("batched backward apply");
        }
        if (b.av)
            FILT_LAUNCH(FILT_BNAME("batched_bwd_apply", W), kb_bwd_apply_quad_staged<false>, sgrid,
                        dim3(64), 0, st, b.segs, b.app_items, b.app_n, gy, a, ws, gx, gyi,
                        (const float *)nullptr, (const float *)nullptr, (float *)nullptr);
        else
            FILT_LAUNCH(FILT_BNAME("batched_bwd_apply", W), kb_bwd_apply_quad<false>, grid, dim3(kThreads), 0,
                        st, b.segs, b.app_items, b.app_n, gy, a, ws, gx, gyi);
        s = check_launch("batched backward apply");
    } else {
        s = batched_bwd_apply<W>(b, gy, y, a, yi, ws, gx, nullptr, gyi, st);
    }
    if (s != FILT_OK || ga == nullptr)
        return s;
    FILT_LAUNCH(FILT_BNAME("batched_coef_grads", W), kb_coef_grads<W>, dim3((unsigned)b.app_n), dim3(256), 0, st,
                b.segs, b.app_items, Lc, gx, y, yi, ga, (int)((uintptr_t)ga % 16 == 0));
    return check_launch("batched coefficient gradients");
}

#define FILT_DECLARE_BATCHED(W, EXT)                                                               \
    EXT template filt_status batched_fwd_summary<W>(const BucketArgs &, const float *,             \
                                                    const float *, double *, hipStream_t);         \
    EXT template filt_status batched_bwd_summary<W>(const BucketArgs &, const float *,             \
                                                    const float *, double *, hipStream_t);         \
    EXT template filt_status batched_fwd_apply<W>(const BucketArgs &, const float *,               \
                                                  const float *, const float *, const double *,    \
                                                  float *, hipStream_t);                           \
    EXT template filt_status batched_bwd_apply<W>(const BucketArgs &, const float *,               \
                                                  const float *, const float *, const float *,     \
                                                  const double *, float *, float *, float *,       \
                                                  hipStream_t);

}  // namespace filt_detail
