// common.h -- shared declarations of the filter library (internal).
//
// Method: Yu & Fazekas, arXiv 2511.14390.  Forward = Sec. 2 Eq. 1 as a
// difference equation (per-sample coefficients, initial conditions).
// Backward = Sec. 3.1 Eqs. 6-9 / Appendix A in scalar form: the adjoint is the
// transposed (scatter) filter run in reverse time (the "backward of DF is TDF"
// remark after Eq. 9), fused with the coefficient and initial-condition
// gradient products.
//
// Time parallelism follows the associative-scan idea of Sec. 3.2: the signal
// is cut into chunks of L samples and every chunk is summarised by the affine
// map (Phi_c, s_c) that takes the filter state entering the chunk to the state
// leaving it (Phi_c = the product of the chunk's companion matrices, Eq. 4;
// s_c = the zero-state end state).  Chunks combine with the operator
// (Phi, s) + (Phi', s') = (Phi' Phi, Phi' s + s') of Sec. 3.2.  Three phases:
//   1. summary  -- every (channel, chunk) solves its chunk from zero state
//                  (s_c) and, for per-sample coefficients, from each unit
//                  state (the columns of Phi_c); time-invariant filters share
//                  one Phi per channel.
//   2. carry    -- a blocked scan over the chunk summaries (FP64) yields the
//                  exact state entering every chunk.
//   3. apply    -- every (channel, chunk) reruns its chunk from that state and
//                  writes the outputs (forward: y; backward: gx and the
//                  coefficient / initial-condition gradients).
//
// Register state: histories live in W = 2^ceil(log2(max(N, M+1))) registers
// addressed modulo W; the time loop is unrolled by W so every register index
// is a compile-time constant (no scratch, no shifting).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>
#include <utility>

#include "filt.h"

namespace filt_detail {

filt_status fail(filt_status s, const char *fmt, ...);
filt_status check_launch(const char *what);

// Optional per-kernel timing (filt_profile_*): a HIP event pair recorded on
// the launch stream around every kernel while enabled; free otherwise.
int prof_begin(const char *name, hipStream_t st);
void prof_end(int slot, hipStream_t st);

#define FILT_LAUNCH(NAME, ...)                                                                     \
    do {                                                                                           \
        const int filt_prof_slot_ = prof_begin(NAME, FILT_LAUNCH_STREAM_(__VA_ARGS__));            \
        hipLaunchKernelGGL(__VA_ARGS__);                                                           \
        prof_end(filt_prof_slot_, FILT_LAUNCH_STREAM_(__VA_ARGS__));                               \
    } while (0)
#define FILT_LAUNCH_STREAM_(K, G, B, S, ST, ...) ST

constexpr int kThreads = 256;
constexpr int kMaxOrder = 16;

// Frame-held coefficients: with a hop h >= 2 the coefficient row of time t
// is that of frame t / h (rows at frame rate, F = ceil(T / h) per channel).
// The division is a multiply-high and a shift, exact for t < 2^31 (checked on
// the host): with l = ceil(log2 h) and m = ceil(2^(31+l) / h), the excess
// m h - 2^(31+l) is below h <= 2^l, so floor(t m / 2^(31+l)) = floor(t / h).
// m = 0 marks per-sample rows.
struct FrameDiv {
    uint32_t m;
    int sh;  // l - 1
};

inline FrameDiv frame_div(int64_t hop)
{
    FrameDiv f{0u, 0};
    if (hop <= 1)
        return f;
    int l = 0;
    while ((int64_t(1) << l) < hop)
        ++l;
    const uint64_t num = uint64_t(1) << (31 + l);
    f.m = (uint32_t)((num + (uint64_t)hop - 1) / (uint64_t)hop);
    f.sh = l - 1;
    return f;
}

__device__ __forceinline__ uint32_t frame_of(const FrameDiv &f, uint32_t t)
{
    return __umulhi(t, f.m) >> f.sh;
}

// Device-side description of one problem.
struct Dims {
    int64_t B, T;
    int M, N;
    int tv, layout;
    int64_t F;      // coefficient rows per channel in time: T per sample, or frames
    int64_t hop;    // samples per coefficient row (1 per sample)
    FrameDiv fd;    // frame-held rows when fd.m != 0 (hop >= 2)
    int has_b;
    int64_t L, C;   // chunk length (multiple of 32) and number of chunks
    int64_t G, NB;  // carry: steps per block and number of blocks
    int a_vec;      // a rows are exactly W wide and vector-aligned (full-row loads)
    int ga_vec;     // same for the per-sample ga rows written by the backward
    int tz;         // time-invariant [B, T] problem on the matrix-core path (toeplitz.hip)
};

__device__ __forceinline__ int64_t sig_at(const Dims &d, int64_t b, int64_t t)
{
    return d.layout == FILT_LAYOUT_TB ? t * d.B + b : b * d.T + t;
}

// Start of the coefficient row (K taps) that applies at (channel b, time t).
__device__ __forceinline__ int64_t row_at(const Dims &d, int64_t b, int64_t t, int K)
{
    if (!d.tv)
        return b * K;
    const int64_t r = d.fd.m != 0 ? (int64_t)frame_of(d.fd, (uint32_t)t) : t;
    return (d.layout == FILT_LAYOUT_TB ? r * d.B + b : b * d.F + r) * (int64_t)K;
}

// x[t] for any t: negative times from xi (x[-j] = xi[j-1]), past T -> 0.
template <typename io_t, typename acc_t>
__device__ __forceinline__ acc_t ld_x(const Dims &d, const io_t *x, const io_t *xi, int64_t b,
                                      int64_t t)
{
    if (t >= 0)
        return t < d.T ? (acc_t)x[sig_at(d, b, t)] : acc_t(0);
    const int64_t j = -t;
    return (xi != nullptr && j <= d.M) ? (acc_t)xi[b * d.M + (j - 1)] : acc_t(0);
}

template <typename io_t, typename acc_t>
__device__ __forceinline__ acc_t ld_y(const Dims &d, const io_t *y, const io_t *yi, int64_t b,
                                      int64_t t)
{
    if (t >= 0)
        return t < d.T ? (acc_t)y[sig_at(d, b, t)] : acc_t(0);
    const int64_t j = -t;
    return (yi != nullptr && j <= d.N) ? (acc_t)yi[b * d.N + (j - 1)] : acc_t(0);
}

// Walks one per-(channel) sequence -- a signal or a coefficient row -- in
// time from chunk start t0: at(t) is the element (row start) of time t, with
// t - t0 clamped into [lo, hi] so every address stays inside [0, T-1].  Steps
// fetched past the end of a signal are only ever used with zero input and
// zero state, or not at all.  One multiply-add per access, no layout branch.
// Frame-held rows (fd.m != 0): p0 is the row of t0's frame, stride the
// elements per frame, and the row of time t sits frame(t) - frame(t0) rows on.
template <typename T>
struct Cursor {
    const T *p0;     // element of time t0
    int stride;      // elements per time step (the host checks it fits)
    int lo, hi;      // clamp of t - t0
    FrameDiv fd;
    uint32_t t0, f0; // frame-held rows: the chunk start and its frame

    __device__ __forceinline__ const T *at(int64_t t0_, int64_t t) const
    {
        const int r = min(max((int)(t - t0_), lo), hi);
        if (fd.m == 0)
            return p0 + (int64_t)r * stride;
        const int df = (int)frame_of(fd, t0 + (uint32_t)r) - (int)f0;
        return p0 + (int64_t)df * stride;
    }
};

// Cursor over a signal [layout] (K = 1) or over per-sample rows of K taps;
// it may reach `back` steps before t0 (never before time 0).
template <typename T>
__device__ __forceinline__ Cursor<T> cursor(const Dims &d, const T *base, int64_t b, int64_t t0,
                                            int K, int back = 4)
{
    Cursor<T> c;
    c.p0 = base + (d.layout == FILT_LAYOUT_TB ? t0 * d.B + b : b * d.T + t0) * (int64_t)K;
    c.stride = (int)((d.layout == FILT_LAYOUT_TB ? d.B : 1) * (int64_t)K);
    const int64_t lo = -t0 < -back ? -(int64_t)back : -t0;
    const int64_t hi = d.T - 1 - t0 > d.L + 4 ? d.L + 4 : d.T - 1 - t0;
    c.lo = (int)lo;
    c.hi = (int)hi;
    c.fd = FrameDiv{0u, 0};
    c.t0 = 0;
    c.f0 = 0;
    return c;
}

// Coefficient rows of channel b seen from chunk start t0: at(r) is the row
// (K taps) that applies at time t0 + r, r >= -t0 (per-sample rows r steps
// on; frame-held rows frame(t0 + r) - frame(t0) frames on).
template <typename T>
struct RowWalk {
    const T *p;      // row of time t0
    int64_t stride;  // elements per step (per frame when frame-held)
    FrameDiv fd;
    uint32_t t0, f0;

    __device__ __forceinline__ const T *at(int r) const
    {
        if (fd.m == 0)
            return p + (int64_t)r * stride;
        return p + (int64_t)((int)frame_of(fd, t0 + (uint32_t)r) - (int)f0) * stride;
    }
};

template <typename T>
__device__ __forceinline__ RowWalk<T> row_walk(const Dims &d, const T *base, int64_t b,
                                               int64_t t0, int K)
{
    RowWalk<T> w;
    w.p = base + row_at(d, b, t0, K);
    w.stride = (d.layout == FILT_LAYOUT_TB ? d.B : 1) * (int64_t)K;
    w.fd = d.tv ? d.fd : FrameDiv{0u, 0};
    w.t0 = (uint32_t)t0;
    w.f0 = w.fd.m != 0 ? frame_of(w.fd, (uint32_t)t0) : 0u;
    return w;
}

// Cursor over the coefficient rows (K taps) of channel b from chunk start
// t0: per-sample rows as cursor(), frame-held rows one row per frame.
template <typename T>
__device__ __forceinline__ Cursor<T> row_cursor(const Dims &d, const T *base, int64_t b,
                                                int64_t t0, int K, int back = 4)
{
    Cursor<T> c = cursor(d, base, b, t0, K, back);
    if (d.tv && d.fd.m != 0) {
        c.fd = d.fd;
        c.t0 = (uint32_t)t0;
        c.f0 = frame_of(d.fd, (uint32_t)t0);
        c.p0 = base + row_at(d, b, t0, K);
    }
    return c;
}

// Raw (unconverted) coefficient row: ra[k-1] = a_k (k = 1..W, 0 beyond N),
// rb[k] = b_k (k = 0.., 0 beyond M; b = [1] when no b is given).  FIR: the
// filter has feed-forward taps beyond b_0 (M > 0).  AV: the a rows are
// exactly W wide and aligned, read as whole vectors with no per-tap checks.
// br must be a valid address even without b (then only b_0 = 1 is used).
template <int W, bool FIR>
constexpr int kRawB = FIR ? W : 1;

template <int W, bool FIR, bool AV, typename io_t>
__device__ __forceinline__ void ld_raw(const Dims &d, const io_t *ar, const io_t *br,
                                       io_t (&ra)[W], io_t (&rb)[kRawB<W, FIR>])
{
    if constexpr (AV) {
        if constexpr (sizeof(io_t) == 4 && W % 4 == 0) {
#pragma unroll
            for (int q = 0; q < W / 4; ++q) {
                const float4 v = *reinterpret_cast<const float4 *>(ar + 4 * q);
                ra[4 * q + 0] = v.x;
                ra[4 * q + 1] = v.y;
                ra[4 * q + 2] = v.z;
                ra[4 * q + 3] = v.w;
            }
        } else if constexpr (sizeof(io_t) == 4 && W == 2) {
            const float2 v = *reinterpret_cast<const float2 *>(ar);
            ra[0] = v.x;
            ra[1] = v.y;
        } else {
#pragma unroll
            for (int k = 0; k < W; ++k)
                ra[k] = ar[k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < W; ++k)
            ra[k] = (k < d.N) ? ar[k] : io_t(0);
    }
    if constexpr (FIR) {
#pragma unroll
        for (int k = 0; k < W; ++k)
            rb[k] = (k <= d.M) ? br[k] : io_t(0);
    } else {
        const io_t b0 = br[0];
        rb[0] = d.has_b ? b0 : io_t(1);
    }
}

// ca[k] = a_k (k = 1..W, ca[0] = 0), cb[k] = b_k (k = 0..W-1) in acc_t.
template <int W, bool FIR, typename io_t, typename acc_t>
__device__ __forceinline__ void cvt_row(const io_t (&ra)[W], const io_t (&rb)[kRawB<W, FIR>],
                                        acc_t (&ca)[W + 1], acc_t (&cb)[W])
{
    ca[0] = acc_t(0);
#pragma unroll
    for (int k = 0; k < W; ++k)
        ca[k + 1] = (acc_t)ra[k];
#pragma unroll
    for (int k = 0; k < W; ++k)
        cb[k] = (k < kRawB<W, FIR>) ? (acc_t)rb[k < kRawB<W, FIR> ? k : 0] : acc_t(0);
}

// Converted time-invariant row of channel b (ac/bc are [B][K]; bc must be a
// valid address even without b).
template <int W, bool FIR, typename io_t, typename acc_t>
__device__ __forceinline__ void ld_row_lti(const Dims &d, const io_t *bc, const io_t *ac,
                                           int64_t b, acc_t (&ca)[W + 1], acc_t (&cb)[W])
{
    io_t ra[W], rb[kRawB<W, FIR>];
    ld_raw<W, FIR, false>(d, ac + (d.N > 0 ? b * d.N : 0), bc + (d.has_b ? b * (d.M + 1) : 0),
                          ra, rb);
    cvt_row<W, FIR>(ra, rb, ca, cb);
}

// Time-invariant problems with an FIR part in the order-8 bucket (FP32 I/O,
// FP64 state) run their tap loops up to the highest tap max(N, M) instead of
// the bucket width, a compile-time bound: an M = N = 4 filter then issues
// about half the FMAs of the width-8 loops (its other taps are zero).  Calls
// f(std::integral_constant<int, KT>) with that bound, or with W.
template <int W, bool FIR, typename io_t, typename acc_t, typename F>
void lti_tap_bound(const Dims &d, F &&f)
{
    if constexpr (W == 8 && FIR && sizeof(io_t) == 4 && sizeof(acc_t) == 8) {
        if (!d.tv) {
            switch (d.N > d.M ? d.N : d.M) {
            case 4:
                f(std::integral_constant<int, 4>{});
                return;
            case 5:
                f(std::integral_constant<int, 5>{});
                return;
            case 6:
                f(std::integral_constant<int, 6>{});
                return;
            case 7:
                f(std::integral_constant<int, 7>{});
                return;
            default:
                break;
            }
        }
    }
    f(std::integral_constant<int, W>{});
}

// f(std::integral_constant<int, i>) for i = 0..n-1, in order.
template <typename F, int... I>
__device__ __forceinline__ void static_for_seq(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int n, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_seq(f, std::make_integer_sequence<int, n>{});
}

// FP64 value moved within lane quads (two 32-bit DPP moves, quad_perm
// control); used by the recursions that split one chain's taps over a quad.
template <int CTRL>
__device__ __forceinline__ double quad_dpp(double v)
{
    // every source lane of a quad_perm is live, so bound_ctrl only spares the
    // move that would preload an "old" value
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, true);
}
constexpr int kQuadXor1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kQuadFromPrev = 0x90;  // quad_perm [0,0,1,2]: lane q reads lane q - 1
constexpr int kQuadFromNext = 0xF9;  // quad_perm [1,2,3,3]: lane q reads lane q + 1
constexpr int kQuadLane0 = 0x00;     // quad_perm [0,0,0,0]

// One step's loads of a quad lane: its four taps of the coefficient row and
// a signal sample with its gain.
template <typename io_t>
struct QuadRaw {
    io_t a[4];  // taps 4q .. 4q + 3 of the coefficient row (a_{4q+1} .. a_{4q+4})
    io_t s, g;  // signal sample and its gain (b_0, or 1 without b)
    io_t y;     // adjoint with gradients: the y sample entering the window
};

// Taps 4q .. 4q + 3 of one coefficient row (N == 16 and 16-byte aligned rows
// with AV; else element loads, clamped into the row and zeroed on use).
template <bool AV, typename io_t>
__device__ __forceinline__ void quad_taps(const io_t *row, int q, int N, io_t (&v)[4])
{
    if constexpr (AV && sizeof(io_t) == 4) {
        const float4 f = *reinterpret_cast<const float4 *>(row + 4 * q);
        v[0] = f.x;
        v[1] = f.y;
        v[2] = f.z;
        v[3] = f.w;
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            v[i] = row[min(4 * q + i, N - 1)];
    }
}

// -a_{4q+1+i} as a double (zero for taps past N).
template <bool AV, typename io_t>
__device__ __forceinline__ double quad_coef(const io_t (&v)[4], int i, int q, int N)
{
    if constexpr (AV && sizeof(io_t) == 4)
        return -(double)v[i];
    else
        return 4 * q + i < N ? -(double)v[i] : 0.0;
}

// Prefetch depth (time steps) of the summary and apply loops.  The apply
// kernels run one long sequential chain per (channel, chunk) and are
// latency-bound, so they keep more steps in flight.
constexpr int kSummaryPrefetch = 4;
constexpr int kApplyPrefetch = 8;

// Everything one time step reads from memory, fetched ahead of its use so the
// loads of step t + 2 overlap the arithmetic of step t.  TV: the coefficient
// row; s0..s2: signal samples whose meaning the caller sets.
template <int W, bool TV, bool FIR, typename io_t>
struct Prefetch {
    io_t ra[TV ? W : 1];
    io_t rb[TV ? kRawB<W, FIR> : 1];
    io_t s0, s1, s2;
};

// Decode a flat item index into (lane-in-chunk r, channel, chunk) with the
// nl lanes of a chunk adjacent, then channels (TB) or chunks (BT) fastest.
__device__ __forceinline__ void decode_lanes(const Dims &d, int64_t idx, int64_t ncs, int nl,
                                             int64_t &b, int64_t &c, int &r)
{
    r = (int)(idx % nl);
    const int64_t q = idx / nl;
    if (d.layout == FILT_LAYOUT_TB) {
        b = q % d.B;
        c = q / d.B;
    } else {
        c = q % ncs;
        b = q / ncs;
    }
}

// Decode a flat item index into (channel, chunk, column).  Channels vary
// fastest in the [T][B] layout (coalesced rows), chunks in [B][T].
__device__ __forceinline__ void decode(const Dims &d, int64_t idx, int64_t ncs, int64_t &b,
                                       int64_t &c, int64_t &j)
{
    if (d.layout == FILT_LAYOUT_TB) {
        b = idx % d.B;
        const int64_t r = idx / d.B;
        c = r % ncs;
        j = r / ncs;
    } else {
        c = idx % ncs;
        const int64_t r = idx / ncs;
        b = r % d.B;
        j = r / d.B;
    }
}


// Affine scan over chunk summaries (state S_{i+1} = Phi_i S_i + s_i).
//
// Steps i = 0 .. C-2 map state S_i to S_{i+1} = Phi S_i + s.  Forward: step i
// uses chunk i's summary and S_i is the state entering chunk i.  Backward:
// step i uses chunk C-1-i and S_i is the state entering chunk C-1-i from the
// future.  Blocked in three passes (blocks of G steps): block aggregates,
// a sequential pass over blocks, then the states inside each block.

struct CarryArgs {
    const double *summ;   // per-chunk summaries
    const double *phi;    // per-channel time-invariant Phi (and R), or null
    int64_t SS;           // stride of one chunk summary (doubles)
    int64_t soff;         // offset of the vector s within a chunk summary
    int D;                // state size N
    int R;                // extra outputs (M for backward, 0 for forward)
    int bwd;
    double *agg;          // [B][NB][D*D + D]
    double *bstart;       // [B][NB][D] state at each block start
    double *states;       // [B][C][D+R] state entering each chunk
};


inline unsigned grid_for(int64_t n)
{
    return (unsigned)((n + kThreads - 1) / kThreads);
}

// Workgroup size for a launch of n independent items: full 256-thread groups
// only when that still gives every CU several groups; otherwise one
// wavefront per group so the few items spread over all CUs instead of piling
// onto a quarter of them.
constexpr int64_t kCUs = 256;
inline unsigned block_for(int64_t n)
{
    return n >= kCUs * 4 * kThreads ? (unsigned)kThreads : 64u;
}
inline unsigned blocks_for(int64_t n)
{
    const unsigned bs = block_for(n);
    return (unsigned)((n + bs - 1) / bs);
}

// Time-invariant [B, T] problems on the matrix cores (toeplitz.hip): chunks
// of kTzL samples, 64 chunks per workgroup tile.
constexpr int kTzL = 64;

__host__ __device__ inline int round4(int v) { return (v + 3) & ~3; }

struct TzGeom {
    int KH, KS, KPF;   // forward GEMM depth: input-history rows, state rows, total
    int KW, KWp, KPB;  // backward: adjoint window max(N, M), padded, total depth
};

__host__ __device__ inline TzGeom tz_geom(int N, int M)
{
    TzGeom g;
    g.KH = round4(M);
    g.KS = round4(N);
    g.KPF = g.KH + kTzL + g.KS;
    g.KW = N > M ? N : M;
    g.KWp = round4(g.KW);
    g.KPB = kTzL + g.KWp;
    return g;
}

// Workspace carve-up, 256-byte aligned regions (FP64 unless noted).
struct WsPlan {
    size_t summ, phi, agg, bstart, states, part, yb, total;
    size_t tz_af, tz_ayb, tz_agx, tz_phib;  // matrix-core path (FP32 matrices)
};

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

inline WsPlan ws_plan(const Dims &d)
{
    const int64_t N = d.N, M = d.M;
    if (d.tz) {
        const TzGeom g = tz_geom(d.N, d.M);
        const int64_t KW = g.KW;
        const int64_t nwg = (d.C + 63) / 64;
        WsPlan w{};
        size_t off = 0;
        auto take = [&](size_t bytes) {
            size_t o = off;
            off = align256(off + bytes);
            return o;
        };
        w.tz_af = take((size_t)(d.B * g.KPF * kTzL) * sizeof(float));
        w.tz_ayb = take((size_t)(d.B * g.KPB * kTzL) * sizeof(float));
        w.tz_agx = take((size_t)(d.B * g.KPB * kTzL) * sizeof(float));
        w.phi = take((size_t)(d.B * N * N) * sizeof(double));
        w.tz_phib = take((size_t)(d.B * KW * KW) * sizeof(double));
        w.summ = take((size_t)(d.B * d.C * KW) * sizeof(double));
        w.states = take((size_t)(d.B * d.C * KW) * sizeof(double));
        // block (or 256-step tile) sums and start states of the carry
        const int64_t nb = std::max<int64_t>(d.NB, (d.C + 254) / 256);
        w.agg = take((size_t)(d.B * nb * (KW * KW + KW)) * sizeof(double));
        w.bstart = take((size_t)(d.B * nb * KW) * sizeof(double));
        w.part = take((size_t)(d.B * nwg * (N + M + 1)) * sizeof(double));
        w.total = off + 256;
        return w;
    }
    const int64_t SSf = N * N + N;
    const int64_t SSb = (N + 1) * (N + M);
    WsPlan w{};
    size_t off = 0;
    auto take = [&](size_t doubles) {
        size_t o = off;
        off = align256(off + doubles * sizeof(double));
        return o;
    };
    w.summ = take((size_t)(d.B * d.C * std::max(SSf, SSb)));
    w.phi = take((size_t)(d.B * (N * N + M * N)));
    // block (or 256-step tile) sums and start states of the carry
    const int64_t nb = std::max<int64_t>(d.NB, (d.C + 254) / 256);
    w.agg = take((size_t)(d.B * nb * (N * N + N)));
    w.bstart = take((size_t)(d.B * nb * std::max<int64_t>(N, 1)));
    w.states = take((size_t)(d.B * d.C * (N + M)));
    w.part = take((size_t)(d.B * d.C * (N + M + 1)));
    // per-sample problems: the adjoint for the coefficient-gradient pass
    w.yb = take(d.tv ? (size_t)(d.B * d.T) : 0);
    w.total = off + 256;
    return w;
}

// carry.hip
filt_status carry_run(const Dims &d, const CarryArgs &a, const void *init, bool init_f64,
                      hipStream_t st);
filt_status fir_states_run(const Dims &d, const double *summ, double *states, hipStream_t st);
filt_status reduce_lti_run(const Dims &d, const double *part, void *ga, void *gb, bool f64,
                           hipStream_t st);

// Frame-held coefficients, per-frame gradient products of one contiguous
// signal of T samples (a channel of a [B, T] problem, or a batched segment):
//   out[f K + j] = sign * sum_{t in frame f} ybar[t] s(t - k0 - j),  j < K,
// with s(u) = hist[-u - 1] for u < 0 (nh values, zero past them).
//
// One wavefront takes 64 consecutive frames f0 .. f0 + 63 (lane i frame
// f0 + i, lanes past nf idle) of hop samples.  Each lane keeps its K sums and
// a shift register of the K signal values its taps read, so a step needs
// only ybar[t] and s(t + 1 - k0).  The wavefront stages both for every lane
// through LDS in slices of kFrameSlice samples, loaded as runs of contiguous
// samples (each half wavefront one frame's slice), so the global loads are
// coalesced although every lane walks its own frame.  FP64 sums.
constexpr int kFrameSlice = 32;
constexpr int kFrameLds = 2 * 64 * (kFrameSlice + 1);  // elements per wavefront

template <typename io_t>
__device__ __forceinline__ void frame_sums_wave(const io_t *ybar, const io_t *s,
                                                const io_t *hist, int nh, int k0, int K,
                                                double sign, int64_t T, int64_t hop, int64_t f0,
                                                int nf, io_t *out, io_t *lds, int lane)
{
    constexpr int SL = kFrameSlice, SP = kFrameSlice + 1;
    static_assert(SL == 32, "the staging loop covers two frames' slices per load");
    constexpr int KM = kMaxOrder + 1;
    io_t *ly = lds, *ls = lds + 64 * SP;
    auto sval = [&](int64_t u) -> double {
        if (u >= 0)
            return u < T ? (double)s[u] : 0.0;
        return (hist != nullptr && -u <= nh) ? (double)hist[-u - 1] : 0.0;
    };
    const int64_t f = f0 + lane;
    const bool act = lane < nf;
    const int64_t t0 = f * hop;
    const int64_t len = act ? min(hop, T - t0) : 0;  // samples of this lane's frame
    double acc[KM], w[KM];  // w[j] = s(t - k0 - j) for the step t about to run
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        acc[j] = 0.0;
        w[j] = (act && j < K) ? sval(t0 - k0 - j) : 0.0;
    }
    for (int64_t r0 = 0; r0 < hop; r0 += SL) {
        // stage: for frame i of the wavefront, samples t = t0_i + r0 + e
        // (e < SL) of ybar and the values s(t + 1 - k0) >= 0 entering the
        // register after step t; every load issued before the LDS stores
        io_t vy[32], vs[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            const int i = 2 * k + (lane >> 5), e = lane & 31;
            const int64_t t = (f0 + i) * hop + r0 + e;
            const bool ok = i < nf && r0 + e < hop && t < T;
            const int64_t u = t + 1 - k0;
            vy[k] = ok ? ybar[t] : io_t(0);
            vs[k] = (ok && r0 + e + 1 < hop && u < T) ? s[u] : io_t(0);
        }
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            const int i = 2 * k + (lane >> 5), e = lane & 31;
            ly[i * SP + e] = vy[k];
            ls[i * SP + e] = vs[k];
        }
        __builtin_amdgcn_s_waitcnt(0xC07F);
        __builtin_amdgcn_wave_barrier();
        const int n = (int)min<int64_t>(SL, len - r0);
        for (int e = 0; e < n; ++e) {
            const double yb = (double)ly[lane * SP + e];
            const double nx = (double)ls[lane * SP + e];
#pragma unroll
            for (int j = 0; j < KM; ++j)
                acc[j] = __builtin_fma(yb, w[j], acc[j]);
#pragma unroll
            for (int j = KM - 1; j > 0; --j)
                w[j] = w[j - 1];
            w[0] = nx;
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (act) {
#pragma unroll
        for (int j = 0; j < KM; ++j)
            if (j < K)
                out[f * K + j] = (io_t)(sign * acc[j]);
    }
}

// Frame rows of a problem: time_varying = 0 (per channel), 1 (per sample)
// or h >= 2 (per frame of h samples).
inline void set_rows(Dims &d, int64_t time_varying)
{
    d.tv = time_varying != 0;
    d.hop = time_varying > 1 ? time_varying : 1;
    d.F = d.tv ? (d.T + d.hop - 1) / d.hop : 0;
    d.fd = frame_div(d.hop);
}

// Frame-held rows: ga / gb of every frame from a stored adjoint,
// ga_k[f] = -sum_{t in f} ybar[t] y[t-k], gb_k[f] = sum_{t in f} ybar[t] x[t-k].
template <typename io_t>
filt_status frame_coef_grads_run(const Dims &d, const io_t *ybar, const io_t *x,
                                 const io_t *xi, const io_t *y, const io_t *yi, io_t *ga,
                                 io_t *gb, hipStream_t st);

// grads.hip: per-sample coefficient gradients from a stored adjoint,
// ga_k[n] = -ybar[n] y[n-k] and gb_k[n] = ybar[n] x[n-k] (Eq. 8-9 per sample).
filt_status tv_coef_grads_run(const Dims &d, const float *ybar, const float *x, const float *xi,
                              const float *y, const float *yi, float *ga, float *gb,
                              hipStream_t st);
bool tv_coef_grads_fits(const Dims &d);  // 32-bit thread indexing
// grads.hip: time-invariant all-pole [B, T] ga from the adjoint ybar, summed
// over time (per-block FP64 partials in part, then the time-invariant
// reduction); part holds at least one record of N + 1 doubles per chunk.
filt_status lti_allpole_ga_run(const Dims &d, const float *ybar, const float *y,
                               const float *yi, float *ga, double *part, hipStream_t st);

// Time-invariant all-pole [B, T] problems with many chunks run their
// applies on the staged (stream) kernels as frame-held problems of one frame
// of T samples: the channel's coefficient row is the frame's row
// ([B][1][N] = [B][N]).  With few chunk chains (short or few signals) the
// per-lane applies are faster (a staged wavefront then walks its runs with
// little to overlap), hence the 32768-chain floor.
inline bool lti_stream_eligible(const Dims &d)
{
    return !d.tv && !d.tz && d.layout == FILT_LAYOUT_BT && !d.has_b && d.M == 0 && d.N > 0 &&
           d.N <= 8 && d.T >= 2 && d.T < ((int64_t)1 << 31) && d.B * d.C >= 32768;
}

// toeplitz.hip
struct TzPlan {
    int KW, KPF, KPB;
    int64_t nwg;  // workgroup tiles per channel
};
TzPlan tz_plan(const Dims &d);
filt_status tz_forward(const Dims &d, const float *x, const float *bc, const float *ac,
                       const float *xi, const float *yi, float *y, const WsPlan &w, char *ws,
                       hipStream_t st);
filt_status tz_backward(const Dims &d, const float *gy, const float *x, const float *y,
                        const float *bc, const float *ac, const float *xi, const float *yi,
                        float *gx, float *gb, float *ga, float *gxi, float *gyi, const WsPlan &w,
                        char *ws, hipStream_t st);

// Solves per lane in the per-sample chunk summaries: the lanes of one chunk
// share every coefficient row among their solves.
template <int W>
struct SummarySlots {
    static constexpr int value = W == 1 ? 2 : 3;
};

// summary.h: chunk summaries, one translation unit per (bucket, I/O type,
// direction).  They write summ/phi (see the kernels).
template <int W, typename io_t>
filt_status fwd_summary_w(const Dims &d, const io_t *x, const io_t *xi, const io_t *bc,
                          const io_t *ac, double *summ, double *phi, hipStream_t st);
template <int W, typename io_t>
filt_status bwd_summary_w(const Dims &d, const io_t *gy, const io_t *bc, const io_t *ac,
                          double *summ, double *phi, hipStream_t st);

// apply.h: whole forward / backward for one bucket and type pair.
template <int W, typename io_t, typename acc_t>
filt_status forward_w(const Dims &d, const io_t *x, const io_t *bc, const io_t *ac,
                      const io_t *xi, const io_t *yi, io_t *y, char *ws, hipStream_t st);
template <int W, typename io_t, typename acc_t>
filt_status backward_w(const Dims &d, const io_t *gy, const io_t *x, const io_t *y,
                       const io_t *bc, const io_t *ac, const io_t *xi, const io_t *yi, io_t *gx,
                       io_t *gb, io_t *ga, io_t *gxi, io_t *gyi, char *ws, hipStream_t st);

#define FILT_DECLARE_SUMMARY(W, IO, EXT)                                                           \
    EXT template filt_status fwd_summary_w<W, IO>(const Dims &, const IO *, const IO *,            \
                                                  const IO *, const IO *, double *, double *,      \
                                                  hipStream_t);                                    \
    EXT template filt_status bwd_summary_w<W, IO>(const Dims &, const IO *, const IO *,            \
                                                  const IO *, double *, double *, hipStream_t);
#define FILT_DECLARE_FWD(W, IO, ACC, EXT)                                                          \
    EXT template filt_status forward_w<W, IO, ACC>(const Dims &, const IO *, const IO *,           \
                                                   const IO *, const IO *, const IO *, IO *,       \
                                                   char *, hipStream_t);
#define FILT_DECLARE_BWD(W, IO, ACC, EXT)                                                          \
    EXT template filt_status backward_w<W, IO, ACC>(                                               \
        const Dims &, const IO *, const IO *, const IO *, const IO *, const IO *, const IO *,      \
        const IO *, IO *, IO *, IO *, IO *, IO *, char *, hipStream_t);
#define FILT_DECLARE_BUCKET(W, EXT)                                                                \
    FILT_DECLARE_SUMMARY(W, float, EXT)                                                            \
    FILT_DECLARE_SUMMARY(W, double, EXT)                                                           \
    FILT_DECLARE_FWD(W, float, float, EXT)                                                         \
    FILT_DECLARE_BWD(W, float, float, EXT)                                                         \
    FILT_DECLARE_FWD(W, float, double, EXT)                                                        \
    FILT_DECLARE_BWD(W, float, double, EXT)                                                        \
    FILT_DECLARE_FWD(W, double, double, EXT)                                                       \
    FILT_DECLARE_BWD(W, double, double, EXT)

// The explicit instantiations live in generated translation units (see
// build.py); every other unit sees them as extern.
#ifndef FILT_INSTANTIATING
FILT_DECLARE_BUCKET(1, extern)
FILT_DECLARE_BUCKET(2, extern)
FILT_DECLARE_BUCKET(4, extern)
FILT_DECLARE_BUCKET(8, extern)
FILT_DECLARE_BUCKET(16, extern)
FILT_DECLARE_BUCKET(32, extern)
#endif

}  // namespace filt_detail
