// stream.h -- the apply phase for per-sample all-pole filters (b = [1],
// M = 0) whose chunks are contiguous in memory: [B, T] signals and the
// segments of a batched plan.
//
// Each lane runs one chunk's recursion (Sec. 2 Eq. 1 forward; the transposed
// adjoint of Sec. 3.1 Eq. 7 backward) from its exact entering state, as in
// apply.h.  What differs is how the data reaches the lane.  A lane's next
// few coefficient rows and signal samples are one contiguous block,
// but the blocks of the 64 lanes of a wavefront lie chunk-lengths apart, so
// a direct per-lane load touches 64 cache lines per instruction.  Here the
// wavefront loads the 64 blocks together, neighbouring lanes reading
// neighbouring words (one or two lines per instruction), parks them in LDS,
// and every lane then reads its own rows from LDS.  The loads of the next
// run are issued before the current run is computed and held in registers
// meanwhile.  Outputs go the same way in reverse: each lane writes its run
// to LDS and the wavefront stores the 64 runs with contiguous stores.
//
// One wavefront per workgroup; lane i of workgroup w serves lane slot
// w*64 + i of the caller's lane list.
#pragma once

#include "common.h"

namespace filt_detail {

// Steps per staged run: the next run waits in registers while the current
// one is computed, so order-16 rows take shorter runs.
template <int W>
struct StreamSteps {
    static constexpr int value = W >= 16 ? 4 : 8;
};

template <int W>
struct StreamLds {
    static constexpr int S = StreamSteps<W>::value;
    static constexpr int CS = S * W + 4;  // coefficient floats per lane (padded)
    static constexpr int SS = S + 1;      // signal / output floats per lane (padded)
    float coef[64 * CS];
    float sig[64 * SS];
    float out[64 * SS];
    // per lane: element offsets from the kernel's base pointers (kept as
    // offsets so the accesses stay global-memory ones) and valid samples
    int64_t osig[64], ocoef[64], oout[64];
    int64_t ln[64];
    int lN[64];  // row width (the order) of each lane's filter
    // frame-held rows (lfm != 0): ocoef is the row of the chunk start's
    // frame; local step s takes the row frame(lt0 + s) - lf0 frames on
    uint32_t lt0[64], lf0[64], lfm[64];
    int lfsh[64];
};

// Row offset (in rows) of local step tc of lane i.
template <int W>
__device__ __forceinline__ int64_t stream_row_of(const StreamLds<W> &L, int i, int64_t tc)
{
    if (L.lfm[i] == 0)
        return tc;
    const FrameDiv f{L.lfm[i], L.lfsh[i]};
    return (int64_t)((int)frame_of(f, L.lt0[i] + (uint32_t)tc) - (int)L.lf0[i]);
}

// Lane i's row bookkeeping for chunk start t0 (fd.m == 0: per-sample rows).
template <int W>
__device__ __forceinline__ void stream_set_rows(StreamLds<W> &L, int i, int64_t t0,
                                                const FrameDiv &fd)
{
    L.lt0[i] = (uint32_t)t0;
    L.lfm[i] = fd.m;
    L.lfsh[i] = fd.sh;
    L.lf0[i] = fd.m != 0 ? frame_of(fd, (uint32_t)t0) : 0u;
}

// The arrays the lane offsets refer to.
struct StreamPtrs {
    const float *sig;
    const float *coef;
    float *out;
};

// Workgroups are one wavefront, so finishing the wave's own LDS traffic
// (lgkmcnt 0) makes every lane's LDS writes visible to all lanes; unlike a
// workgroup barrier this does not wait for the global loads of the runs
// still in flight.  (s_waitcnt operand: vmcnt 63, expcnt 7, lgkmcnt 0.)
__device__ __forceinline__ void stream_sync()
{
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
}

// Registers holding one run of the wavefront while the previous run is
// computed: coefficient words (float4 pieces when rows are whole vectors)
// and signal samples.
template <int W, bool VEC>
struct StreamRegs {
    static constexpr int S = StreamSteps<W>::value;
    static constexpr int NC = VEC ? S * W / 4 : S * W;  // coefficient loads per lane
    using cword = std::conditional_t<VEC, float4, float>;
    cword c[NC];
    float s[S];
    // which loads were real (the rest read a clamped address and are zeroed
    // when committed, so no load result is touched before it is needed)
    uint32_t okc[(NC + 31) / 32];
    uint32_t oks;
};

// Local step t clamped into [0, n - 1] (0 when the lane has no samples):
// runs past either end of a chunk read its first or last row instead.
__device__ __forceinline__ int64_t stream_clamp(int64_t t, int64_t n)
{
    return t < 0 ? 0 : (t < n ? t : (n > 0 ? n - 1 : 0));
}

// Load run `lo` (local steps [lo, lo + S)) of every lane: coefficient element
// (lane i, step s, tap k) for k < N, else 0; signal (lane i, step s).  Every
// load is issued (invalid ones read the lane's first row, which always exists,
// and are then replaced by 0), so the code is straight-line and the compiler
// can wait for exactly the loads a commit needs.
template <int W, bool VEC>
__device__ __forceinline__ void stream_load(const StreamLds<W> &L, const StreamPtrs &P, int64_t lo,
                                            StreamRegs<W, VEC> &r)
{
    constexpr int S = StreamSteps<W>::value;
    const int l = threadIdx.x;
    if constexpr (VEC) {
        constexpr int PER = S * W / 4;  // float4 pieces per lane run
#pragma unroll
        for (int j = 0; j < r.NC; ++j) {
            const int g = l + 64 * j;
            const int i = g / PER, q = g % PER;
            const int s = (4 * q) / W;
            const int64_t n = L.ln[i];
            const int64_t t = lo + s;
            // clamp into the lane's chunk (its first row when it has none)
            const int64_t tc = stream_clamp(t, n);
            r.c[j] = *reinterpret_cast<const float4 *>(P.coef + L.ocoef[i] +
                                                        stream_row_of(L, i, tc) * W + (4 * q) % W);
            if (j % 32 == 0)
                r.okc[j / 32] = 0;
            r.okc[j / 32] |= ((t >= 0 && t < n) ? 1u : 0u) << (j % 32);
        }
    } else {
#pragma unroll
        for (int j = 0; j < r.NC; ++j) {
            const int g = l + 64 * j;
            const int i = g / (S * W), e = g % (S * W);
            const int s = e / W, k = e % W;
            const int64_t n = L.ln[i];
            const int Ni = L.lN[i];
            const int64_t t = lo + s;
            const int64_t tc = stream_clamp(t, n);
            const int kc = k < Ni ? k : 0;
            r.c[j] = P.coef[L.ocoef[i] + stream_row_of(L, i, tc) * Ni + kc];
            if (j % 32 == 0)
                r.okc[j / 32] = 0;
            r.okc[j / 32] |= ((k < Ni && t >= 0 && t < n) ? 1u : 0u) << (j % 32);
        }
    }
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int g = l + 64 * j;
        const int i = g / S, s = g % S;
        const int64_t n = L.ln[i];
        const int64_t t = lo + s;
        const int64_t tc = stream_clamp(t, n);
        r.s[j] = P.sig[L.osig[i] + tc];
        if (j == 0)
            r.oks = 0;
        r.oks |= ((t >= 0 && t < n) ? 1u : 0u) << j;
    }
}

template <int W, bool VEC>
__device__ __forceinline__ void stream_commit(StreamLds<W> &L, const StreamRegs<W, VEC> &r)
{
    constexpr int S = StreamSteps<W>::value;
    const int l = threadIdx.x;
    if constexpr (VEC) {
        constexpr int PER = S * W / 4;
#pragma unroll
        for (int j = 0; j < r.NC; ++j) {
            const int g = l + 64 * j;
            const int i = g / PER, q = g % PER;
            const bool ok = (r.okc[j / 32] >> (j % 32)) & 1u;
            *reinterpret_cast<float4 *>(&L.coef[i * StreamLds<W>::CS + 4 * q]) =
                ok ? r.c[j] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    } else {
#pragma unroll
        for (int j = 0; j < r.NC; ++j) {
            const int g = l + 64 * j;
            const int i = g / (S * W), e = g % (S * W);
            const bool ok = (r.okc[j / 32] >> (j % 32)) & 1u;
            L.coef[i * StreamLds<W>::CS + e] = ok ? r.c[j] : 0.f;
        }
    }
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int g = l + 64 * j;
        L.sig[(g / S) * StreamLds<W>::SS + g % S] = ((r.oks >> j) & 1u) ? r.s[j] : 0.f;
    }
}

// Store run `lo` of every lane's output from LDS.
template <int W>
__device__ __forceinline__ void stream_flush(const StreamLds<W> &L, const StreamPtrs &P, int64_t lo)
{
    constexpr int S = StreamSteps<W>::value;
    const int l = threadIdx.x;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int g = l + 64 * j;
        const int i = g / S, s = g % S;
        if (lo + s < L.ln[i])
            P.out[L.oout[i] + lo + s] = L.out[i * StreamLds<W>::SS + s];
    }
}

// Coefficient row of step s of the run in LDS, as doubles a[1..W] (a[0]
// unused).
template <int W>
__device__ __forceinline__ void stream_row(const StreamLds<W> &L, int s, double (&a)[W + 1])
{
    const float *p = &L.coef[threadIdx.x * StreamLds<W>::CS + s * W];
    if constexpr (W % 4 == 0) {
#pragma unroll
        for (int q = 0; q < W / 4; ++q) {
            const float4 v = *reinterpret_cast<const float4 *>(p + 4 * q);
            a[4 * q + 1] = v.x;
            a[4 * q + 2] = v.y;
            a[4 * q + 3] = v.z;
            a[4 * q + 4] = v.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < W; ++k)
            a[k + 1] = p[k];
    }
}

// Forward: y[t] = x[t] - sum_k a_k[t] y[t-k] over the lane's chunk, from the
// entering state h0[i] = y[t0-1-i].  L is the chunk length (a multiple of 32).
template <int W, bool VEC>
__device__ __forceinline__ void stream_forward(StreamLds<W> &L, const StreamPtrs &P, int64_t Lc,
                                               const double (&h0)[W])
{
    constexpr int S = StreamSteps<W>::value;
    constexpr int m = W - 1;
    constexpr int SU = W > S ? W / S : 1;  // runs per unrolled group (static slots)
    const int i = threadIdx.x;
    double h[W];
#pragma unroll
    for (int q = 0; q < W; ++q)
        h[(-(q + 1)) & m] = h0[q];
    // run k is in LDS while runs k + 1 and k + 2 are in flight in registers
    // (ring slot (k + 1) & 1 holds run k + 1)
    constexpr int UG = SU > 2 ? SU : 2;  // runs per unrolled group
    StreamRegs<W, VEC> r[2];
    stream_load<W, VEC>(L, P, 0, r[0]);
    stream_commit<W, VEC>(L, r[0]);
    stream_sync();
    stream_load<W, VEC>(L, P, S, r[1]);
    stream_load<W, VEC>(L, P, 2 * S, r[0]);
    for (int64_t g0 = 0; g0 < Lc; g0 += UG * S) {
#pragma unroll
        for (int u = 0; u < UG; ++u) {
            const int64_t lo = g0 + u * S;  // Lc is a multiple of UG * S
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int st = (u % SU) * S + s;  // slots repeat every SU runs
                double a[W + 1];
                stream_row<W>(L, s, a);
                double p0 = L.sig[i * StreamLds<W>::SS + s], p1 = 0.0;
#pragma unroll
                for (int k = W; k >= 2; --k) {
                    if (k & 1)
                        p1 -= a[k] * h[(st - k) & m];
                    else
                        p0 -= a[k] * h[(st - k) & m];
                }
                const double y = (p0 + p1) - a[1] * h[(st - 1) & m];
                h[st & m] = y;
                L.out[i * StreamLds<W>::SS + s] = (float)y;
            }
            stream_sync();
            stream_flush<W>(L, P, lo);
            stream_commit<W, VEC>(L, r[(u + 1) & 1]);
            stream_sync();
            stream_load<W, VEC>(L, P, lo + 3 * S, r[(u + 1) & 1]);
        }
    }
}

// Backward (transposed adjoint, decreasing time) over the lane's chunk from
// the adjoint state entering from the next chunk, s0[i] = s_{i+1}; returns
// the state left before the chunk's first sample in s0 (gyi for chunk 0).
// Writes ybar (and gx = ybar).
template <int W, bool VEC>
__device__ __forceinline__ void stream_backward(StreamLds<W> &L, const StreamPtrs &P, int64_t Lc,
                                                double (&s0)[W])
{
    constexpr int S = StreamSteps<W>::value;
    constexpr int m = W - 1;
    constexpr int SU = W > S ? W / S : 1;
    const int i = threadIdx.x;
    // s_k sits in slot (k - t) mod W before time t is processed; the chunk
    // length is a multiple of W, so before its last sample s_k is in (k+1)
    double ss[W];
#pragma unroll
    for (int q = 0; q < W; ++q)
        ss[(q + 2) & m] = s0[q];
    constexpr int UG = SU > 2 ? SU : 2;
    StreamRegs<W, VEC> r[2];
    stream_load<W, VEC>(L, P, Lc - S, r[0]);
    stream_commit<W, VEC>(L, r[0]);
    stream_sync();
    stream_load<W, VEC>(L, P, Lc - 2 * S, r[1]);
    stream_load<W, VEC>(L, P, Lc - 3 * S, r[0]);
    for (int64_t g0 = 0; g0 < Lc; g0 += UG * S) {
#pragma unroll
        for (int u = 0; u < UG; ++u) {
            // run [lo, lo + S), walked downwards; Lc is a multiple of UG * S
            const int64_t lo = Lc - g0 - (u + 1) * S;
#pragma unroll
            for (int s = S - 1; s >= 0; --s) {
                // local time t = lo + s; t mod W = s - ((u % SU) + 1) S mod W
                const int tm = s - ((u % SU) + 1) * S;
                double a[W + 1];
                stream_row<W>(L, s, a);
                const double yb = (double)L.sig[i * StreamLds<W>::SS + s] + ss[(1 - tm) & m];
                ss[(1 - tm) & m] = -a[W] * yb;
#pragma unroll
                for (int k = 1; k < W; ++k)
                    ss[(k + 1 - tm) & m] -= a[k] * yb;
                L.out[i * StreamLds<W>::SS + s] = (float)yb;
            }
            stream_sync();
            stream_flush<W>(L, P, lo);
            stream_commit<W, VEC>(L, r[(u + 1) & 1]);
            stream_sync();
            stream_load<W, VEC>(L, P, lo - 3 * S, r[(u + 1) & 1]);
        }
    }
#pragma unroll
    for (int q = 0; q < W; ++q)
        s0[q] = ss[(q + 2) & m];
}

}  // namespace filt_detail

namespace filt_detail {

// Dense [B, T] problems: lane idx = (b, c) with c fastest.
template <int W, bool VEC>
__global__ void __launch_bounds__(64)
k_stream_fwd(Dims d, const float *__restrict__ x, const float *__restrict__ a,
             const float *__restrict__ yi, const double *__restrict__ states,
             float *__restrict__ y)
{
    __shared__ StreamLds<W> L;
    const int i = threadIdx.x;
    const int64_t idx = (int64_t)blockIdx.x * 64 + i;
    const bool act = idx < d.B * d.C;
    const int64_t c = act ? idx % d.C : 0, b = act ? idx / d.C : 0;
    const int64_t t0 = c * d.L;
    L.osig[i] = b * d.T + t0;
    L.ocoef[i] = row_at(d, b, t0, d.N);
    stream_set_rows(L, i, t0, d.fd);
    L.oout[i] = b * d.T + t0;
    L.ln[i] = act ? min(d.L, d.T - t0) : 0;
    L.lN[i] = d.N;
    double h0[W];
#pragma unroll
    for (int q = 0; q < W; ++q) {
        double v = 0.0;
        if (act && q < d.N)
            v = c == 0 ? (yi != nullptr ? (double)yi[b * d.N + q] : 0.0)
                       : states[(b * d.C + c) * d.N + q];
        h0[q] = v;
    }
    __syncthreads();
    stream_forward<W, VEC>(L, StreamPtrs{x, a, y}, d.L, h0);
}

// Writes ybar to yb (gx itself when gx is wanted: for b = [1] they are equal)
// and, from chunk 0, gyi.
template <int W, bool VEC>
__global__ void __launch_bounds__(64)
k_stream_bwd(Dims d, const float *__restrict__ gy, const float *__restrict__ a,
             const double *__restrict__ states, float *__restrict__ yb, float *__restrict__ gyi)
{
    __shared__ StreamLds<W> L;
    const int i = threadIdx.x;
    const int64_t idx = (int64_t)blockIdx.x * 64 + i;
    const bool act = idx < d.B * d.C;
    const int64_t c = act ? idx % d.C : 0, b = act ? idx / d.C : 0;
    const int64_t t0 = c * d.L;
    L.osig[i] = b * d.T + t0;
    L.ocoef[i] = row_at(d, b, t0, d.N);
    stream_set_rows(L, i, t0, d.fd);
    L.oout[i] = b * d.T + t0;
    L.ln[i] = act ? min(d.L, d.T - t0) : 0;
    L.lN[i] = d.N;
    double s0[W];
#pragma unroll
    for (int q = 0; q < W; ++q)
        s0[q] = (act && q < d.N && c + 1 < d.C) ? states[(b * d.C + c) * d.N + q] : 0.0;
    __syncthreads();
    stream_backward<W, VEC>(L, StreamPtrs{gy, a, yb}, d.L, s0);
    if (act && c == 0 && gyi != nullptr)
#pragma unroll
        for (int q = 0; q < W; ++q)
            if (q < d.N)
                gyi[b * d.N + q] = (float)s0[q];
}

// The staged path serves per-sample all-pole [B, T] problems with FP32 data
// and rows of up to 8 taps (order-16 rows already fill most of a cache line
// per lane and step, and the direct path keeps more of them in flight).
inline bool stream_eligible(const Dims &d)
{
    return d.tv && d.layout == FILT_LAYOUT_BT && !d.has_b && d.M == 0 && d.N > 0 && d.N <= 8;
}

template <int W>
filt_status stream_forward_run(const Dims &d, const float *x, const float *a, const float *yi,
                               const double *states, float *y, hipStream_t st)
{
    const unsigned grid = (unsigned)((d.B * d.C + 63) / 64);
    if (d.a_vec && W % 4 == 0)
        FILT_LAUNCH("stream_fwd_apply", (k_stream_fwd<W, (W % 4 == 0)>), dim3(grid), dim3(64), 0,
                    st, d, x, a, yi, states, y);
    else
        FILT_LAUNCH("stream_fwd_apply", (k_stream_fwd<W, false>), dim3(grid), dim3(64), 0, st, d,
                    x, a, yi, states, y);
    return check_launch("forward apply");
}

template <int W>
filt_status stream_backward_run(const Dims &d, const float *gy, const float *a,
                                const double *states, float *yb, float *gyi, hipStream_t st)
{
    const unsigned grid = (unsigned)((d.B * d.C + 63) / 64);
    if (d.a_vec && W % 4 == 0)
        FILT_LAUNCH("stream_bwd_apply", (k_stream_bwd<W, (W % 4 == 0)>), dim3(grid), dim3(64), 0,
                    st, d, gy, a, states, yb, gyi);
    else
        FILT_LAUNCH("stream_bwd_apply", (k_stream_bwd<W, false>), dim3(grid), dim3(64), 0, st, d,
                    gy, a, states, yb, gyi);
    return check_launch("backward apply");
}

}  // namespace filt_detail
