// quadstage.h -- staged quad applies for the batched order-16 bucket.
//
// The quad applies (apply.h) run each (segment, chunk) chain on a lane quad,
// lane q owning taps 4q+1 .. 4q+4.  In the batched plan a segment's rows are
// contiguous in time, so the 16 chains of a wavefront read 16 rows that lie
// a chunk length apart at every step: each load instruction touches 16
// separate 64-byte pieces, and the same quad apply on channel-interleaved
// data (where a wavefront's rows of one step are one 1 KB block) moves twice
// the bytes per microsecond.  Here the wavefront loads the next run of
// kQuadRun steps of all 16 chains together -- a wavefront reads one chain's
// run of rows, 1 KB contiguous -- parks it in LDS, and each
// quad then reads its taps from LDS; outputs are gathered in LDS and stored
// as contiguous runs.  The run after the one being computed is in flight in
// registers meanwhile.  Same arithmetic as fwd_apply_quad / bwd_apply_quad
// (FP64 state, quad butterfly), full-width rows only (every filter of the
// bucket of order 16 with 16-byte aligned rows); per-sample or frame-held.
//
// One wavefront per workgroup; wavefront w serves items 16w .. 16w + 15.
#pragma once

#include "common.h"

namespace filt_detail {

constexpr int kQuadRun = 16;       // steps per staged run
constexpr int kQuadChains = 16;    // chains (quads) per wavefront
constexpr int kQuadYFirst = kQuadRun + 16;  // y samples staged before the first (last in time) run
constexpr int kQuadYRing = 32;     // y ring per chain (a power of two >= run + 16)
static_assert(kQuadRun % 4 == 0 && kQuadRun <= 16 && kQuadRun + 16 <= kQuadYRing,
              "run length: whole float4 signal pieces, one ring");
constexpr int kQuadCPieces = kQuadRun * kQuadChains * 4 / 64;  // row float4 pieces per lane
constexpr int kQuadSPieces = kQuadRun * kQuadChains / 64;      // signal samples per lane

struct QuadStageLds {
    float coef[kQuadChains][kQuadRun * 16 + 4];  // the run's rows (padded)
    float sig[kQuadChains][kQuadRun + 1];
    float out[kQuadChains][kQuadRun + 1];
    // adjoint with ga: y of chunk-relative time tt in slot tt mod 32; while
    // run lo is computed it holds [lo - 17, lo + kQuadRun - 1) (the run's
    // window, the first sample of which enters at its last step), and the
    // samples [lo - kQuadRun - 17, lo - 17) of the next run's window wait in
    // registers
    float yw[kQuadChains][kQuadYRing + 1];
    // per chain: element offsets of the chunk's first row / sample, valid
    // steps, and the frame bookkeeping (lfm == 0: per-sample rows)
    int64_t ocoef[kQuadChains], osig[kQuadChains], ln[kQuadChains];
    int64_t lyT[kQuadChains];  // T - 1 - t0: y past it is clamped (no output uses it)
    int64_t lic[kQuadChains];  // initial-condition offset, -1 without yi
    uint32_t lt0[kQuadChains], lf0[kQuadChains], lfm[kQuadChains];
    int lfsh[kQuadChains];
};

struct QuadStageRegs {
    float4 c[kQuadCPieces];
    float s[kQuadSPieces];
    float y[kQuadYFirst * kQuadChains / 64];    // ga only
    uint32_t okc, oks;
};

__device__ __forceinline__ int64_t qs_row_of(const QuadStageLds &L, int i, int64_t tc)
{
    if (L.lfm[i] == 0)
        return tc;
    const FrameDiv f{L.lfm[i], L.lfsh[i]};
    return (int64_t)((int)frame_of(f, L.lt0[i] + (uint32_t)tc) - (int)L.lf0[i]);
}

// Chain i's bookkeeping for chunk c of segment sd (ln = 0: no chain).
__device__ __forceinline__ void qs_set_chain(QuadStageLds &L, int i, const SegDesc &sd,
                                             int64_t c, bool valid, bool has_yi = false)
{
    const int64_t t0 = c * sd.L;
    const int64_t n = valid ? (sd.T - t0 < sd.L ? sd.T - t0 : sd.L) : 0;
    L.ln[i] = n;
    L.lyT[i] = valid ? sd.T - 1 - t0 : 0;
    L.lic[i] = (valid && has_yi) ? sd.ic_off : -1;
    L.osig[i] = valid ? sd.x_off + t0 : 0;
    L.lt0[i] = (uint32_t)t0;
    L.lfm[i] = valid ? sd.fd.m : 0u;
    L.lfsh[i] = sd.fd.sh;
    const uint32_t f0 = (valid && sd.fd.m != 0) ? frame_of(sd.fd, (uint32_t)t0) : 0u;
    L.lf0[i] = f0;
    L.ocoef[i] = valid ? sd.a_off + (sd.fd.m != 0 ? (int64_t)f0 : t0) * 16 : 0;
}

// Load run `lo` (chunk-local steps [lo, lo + kQuadRun)) of all chains:
// g = lane + 64 j; coefficient piece g -> chain g / (4 kQuadRun), step
// (g / 4) % kQuadRun, quarter g % 4 (contiguous per-sample rows); sample
// g -> chain g / kQuadRun, step g % kQuadRun.  Steps outside [0, n) read the
// chain's first or last row and are zeroed at commit.
__device__ __forceinline__ void qs_load(const QuadStageLds &L, const float *__restrict__ coef,
                                        const float *__restrict__ sig, int64_t lo,
                                        QuadStageRegs &r)
{
    const int l = threadIdx.x;
    r.okc = 0;
#pragma unroll
    for (int j = 0; j < kQuadCPieces; ++j) {
        const int g = l + 64 * j;
        const int i = g / (4 * kQuadRun), s = (g / 4) % kQuadRun, qq = g & 3;
        const int64_t n = L.ln[i];
        const int64_t t = lo + s;
        const int64_t tc = t < 0 ? 0 : (t < n ? t : (n > 0 ? n - 1 : 0));
        r.c[j] = *reinterpret_cast<const float4 *>(coef + L.ocoef[i] + qs_row_of(L, i, tc) * 16 +
                                                   4 * qq);
        r.okc |= ((t >= 0 && t < n) ? 1u : 0u) << j;
    }
    r.oks = 0;
#pragma unroll
    for (int j = 0; j < kQuadSPieces; ++j) {
        const int g = l + 64 * j;
        const int i = g / kQuadRun, s = g % kQuadRun;
        const int64_t n = L.ln[i];
        const int64_t t = lo + s;
        const int64_t tc = t < 0 ? 0 : (t < n ? t : (n > 0 ? n - 1 : 0));
        r.s[j] = sig[L.osig[i] + tc];
        r.oks |= ((t >= 0 && t < n) ? 1u : 0u) << j;
    }
}

__device__ __forceinline__ void qs_commit(QuadStageLds &L, const QuadStageRegs &r)
{
    const int l = threadIdx.x;
#pragma unroll
    for (int j = 0; j < kQuadCPieces; ++j) {
        const int g = l + 64 * j;
        const int i = g / (4 * kQuadRun), s = (g / 4) % kQuadRun, qq = g & 3;
        *reinterpret_cast<float4 *>(&L.coef[i][s * 16 + 4 * qq]) =
            ((r.okc >> j) & 1u) ? r.c[j] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int j = 0; j < kQuadSPieces; ++j) {
        const int g = l + 64 * j;
        L.sig[g / kQuadRun][g % kQuadRun] = ((r.oks >> j) & 1u) ? r.s[j] : 0.f;
    }
}

// ga only: y at chunk-relative times t0 + e, e < NY (NY * 16 / 64 samples a
// lane: sample g -> chain g / NY, e = g % NY), into the chains' rings:
// before time 0 from the initial conditions (zero past 16 or without them),
// clamped below T.
template <int NY>
__device__ __forceinline__ void qs_load_y(const QuadStageLds &L, const float *__restrict__ y,
                                          const float *__restrict__ yi, int64_t t0,
                                          QuadStageRegs &r)
{
    const int l = threadIdx.x;
#pragma unroll
    for (int j = 0; j < NY * kQuadChains / 64; ++j) {
        const int g = l + 64 * j;
        const int i = g / NY, e = g % NY;
        const int64_t tt = t0 + e;                  // chunk-relative
        const int64_t ta = (int64_t)L.lt0[i] + tt;  // absolute in the segment
        float v = 0.f;
        if (ta >= 0) {
            v = y[L.osig[i] + (tt < L.lyT[i] ? tt : L.lyT[i])];
        } else if (L.lic[i] >= 0 && -ta <= 16) {
            v = yi[L.lic[i] + (-ta - 1)];
        }
        r.y[j] = v;
    }
}

template <int NY>
__device__ __forceinline__ void qs_commit_y(QuadStageLds &L, const QuadStageRegs &r, int64_t t0)
{
    const int l = threadIdx.x;
#pragma unroll
    for (int j = 0; j < NY * kQuadChains / 64; ++j) {
        const int g = l + 64 * j;
        const int i = g / NY, e = g % NY;
        L.yw[i][(int)(t0 + e) & (kQuadYRing - 1)] = r.y[j];
    }
}

// ga only: store run `lo` of the per-sample gradient rows of every chain
// from LDS (written over the run's coefficient rows), per-sample chains only
// (frame-held rows take the per-frame pass), as non-temporal float4 runs.
__device__ __forceinline__ void qs_flush_ga(const QuadStageLds &L, float *__restrict__ ga,
                                            int64_t lo)
{
    const int l = threadIdx.x;
#pragma unroll
    for (int j = 0; j < kQuadCPieces; ++j) {
        const int g = l + 64 * j;
        const int i = g / (4 * kQuadRun), s = (g / 4) % kQuadRun, qq = g & 3;
        if (L.lfm[i] == 0 && lo + s < L.ln[i]) {
            using f4 = float __attribute__((ext_vector_type(4)));
            const float4 v = *reinterpret_cast<const float4 *>(&L.coef[i][s * 16 + 4 * qq]);
            const f4 v4 = {v.x, v.y, v.z, v.w};
            __builtin_nontemporal_store(
                v4, reinterpret_cast<f4 *>(ga + L.ocoef[i] + (lo + s) * 16 + 4 * qq));
        }
    }
}

// Store run `lo` of every chain's outputs from LDS.
__device__ __forceinline__ void qs_flush(const QuadStageLds &L, float *__restrict__ out,
                                         int64_t lo)
{
    const int l = threadIdx.x;
#pragma unroll
    for (int j = 0; j < kQuadSPieces; ++j) {
        const int g = l + 64 * j;
        const int i = g / kQuadRun, s = g % kQuadRun;
        if (lo + s < L.ln[i])
            out[L.osig[i] + lo + s] = L.out[i][s];
    }
}

// The wavefront's own LDS traffic finished (workgroups are one wavefront).
__device__ __forceinline__ void qs_sync()
{
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
}

// Forward: y[t] = x[t] - sum_k a_k[t] y[t-k] for each chain from its
// entering state (yi for chunk 0, else the carry's state).
static __global__ void __launch_bounds__(64)
kb_fwd_apply_quad_staged(const SegDesc *__restrict__ segs, const Item *__restrict__ items,
                         int64_t n, const float *__restrict__ x, const float *__restrict__ a,
                         const float *__restrict__ yi, const double *__restrict__ ws,
                         float *__restrict__ y)
{
    __shared__ QuadStageLds L;
    const int l = threadIdx.x;
    const int k = l >> 2, q = l & 3;  // this lane's chain and tap group
    const int64_t item = (int64_t)blockIdx.x * kQuadChains + k;
    const bool valid = item < n;
    const Item it = items[valid ? item : 0];
    const SegDesc sd = segs[it.seg];
    const int64_t Lc = sd.L;  // the bucket's chunk length (every segment)
    if (q == 0)
        qs_set_chain(L, k, sd, it.chunk, valid);
    double w[4];  // w[i] = y[t - 4q - 1 - i]
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int kk = 4 * q + i;
        double v = 0.0;
        if (valid) {
            if (it.chunk == 0)
                v = yi != nullptr ? (double)yi[sd.ic_off + kk] : 0.0;
            else
                v = ws[sd.states_off + (int64_t)it.chunk * 16 + kk];
        }
        w[i] = v;
    }
    qs_sync();
    QuadStageRegs r;
    qs_load(L, a, x, 0, r);
    qs_commit(L, r);
    qs_sync();
    for (int64_t lo = 0; lo < Lc; lo += kQuadRun) {
        if (lo + kQuadRun < Lc)
            qs_load(L, a, x, lo + kQuadRun, r);
#pragma unroll
        for (int s = 0; s < kQuadRun; ++s) {
            const float4 c4 = *reinterpret_cast<const float4 *>(&L.coef[k][s * 16 + 4 * q]);
            const double ca[4] = {-(double)c4.x, -(double)c4.y, -(double)c4.z, -(double)c4.w};
            double p = 0.0;
#pragma unroll
            for (int i = 3; i >= 0; --i)
                p = __builtin_fma(ca[i], w[i], p);
            double tot = p + quad_dpp<kQuadXor1>(p);
            tot = tot + quad_dpp<kQuadXor2>(tot);
            const double v = (double)L.sig[k][s] + tot;
            if (q == 0)
                L.out[k][s] = (float)v;
            const double prev = quad_dpp<kQuadFromPrev>(w[3]);
            w[3] = w[2];
            w[2] = w[1];
            w[1] = w[0];
            w[0] = q == 0 ? v : prev;
        }
        qs_sync();
        qs_flush(L, y, lo);
        if (lo + kQuadRun < Lc)
            qs_commit(L, r);
        qs_sync();
    }
}

// Backward (transposed adjoint, decreasing time) from the state entering
// from the next chunk; writes ybar (= gx without b) and gyi from chunk 0.
// GA: also the per-sample gradient rows ga_k[t] = -ybar[t] y[t-k] (Sec. 3.1
// Eq. 8 per sample) of per-sample chains, lane q its taps 4q+1 .. 4q+4 from
// a window wy[i] = y[t - 4q - 1 - i] sliding down one sample per step; the
// run's ga rows overwrite its coefficient rows in LDS (each lane its own
// slot, after reading it) and leave as contiguous runs.
template <bool GA>
__global__ void __launch_bounds__(64)
kb_bwd_apply_quad_staged(const SegDesc *__restrict__ segs, const Item *__restrict__ items,
                         int64_t n, const float *__restrict__ gy, const float *__restrict__ a,
                         const double *__restrict__ ws, float *__restrict__ gx,
                         float *__restrict__ gyi, const float *__restrict__ y,
                         const float *__restrict__ yi, float *__restrict__ ga)
{
    __shared__ QuadStageLds L;
    const int l = threadIdx.x;
    const int k = l >> 2, q = l & 3;
    const int64_t item = (int64_t)blockIdx.x * kQuadChains + k;
    const bool valid = item < n;
    const Item it = items[valid ? item : 0];
    const SegDesc sd = segs[it.seg];
    const int64_t Lc = sd.L;
    if (q == 0)
        qs_set_chain(L, k, sd, it.chunk, valid, yi != nullptr);
    double st[4];  // st[i] = s_{4q+1+i}
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int kk = 4 * q + i;
        st[i] = (valid && it.chunk + 1 < sd.C) ? ws[sd.states_off + (int64_t)it.chunk * 16 + kk]
                                                : 0.0;
    }
    qs_sync();
    QuadStageRegs r;
    constexpr int kRing = kQuadYRing - 1;
    qs_load(L, a, gy, Lc - kQuadRun, r);
    if constexpr (GA)
        qs_load_y<kQuadYFirst>(L, y, yi, Lc - kQuadRun - 17, r);
    qs_commit(L, r);
    if constexpr (GA)
        qs_commit_y<kQuadYFirst>(L, r, Lc - kQuadRun - 17);
    qs_sync();
    // wy[i] = y[t - 4q - 1 - i] for the chunk's last step t = Lc - 1
    float wy[4];
    if constexpr (GA) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            wy[i] = L.yw[k][(int)(Lc - 2 - 4 * q - i) & kRing];
    }
    for (int64_t lo = Lc - kQuadRun; lo >= 0; lo -= kQuadRun) {
        // the next run's rows and gy, and the y it adds to the ring
        // ([lo - 25, lo - 17): the rest of its window is already there)
        if (lo > 0) {
            qs_load(L, a, gy, lo - kQuadRun, r);
            if constexpr (GA)
                qs_load_y<kQuadRun>(L, y, yi, lo - kQuadRun - 17, r);
        }
#pragma unroll
        for (int s = kQuadRun - 1; s >= 0; --s) {
            const float4 c4 = *reinterpret_cast<const float4 *>(&L.coef[k][s * 16 + 4 * q]);
            const double yb = (double)L.sig[k][s] + quad_dpp<kQuadLane0>(st[0]);
            if (q == 0)
                L.out[k][s] = (float)yb;
            if constexpr (GA) {
                const float nyb = -(float)yb;
                *reinterpret_cast<float4 *>(&L.coef[k][s * 16 + 4 * q]) =
                    make_float4(nyb * wy[0], nyb * wy[1], nyb * wy[2], nyb * wy[3]);
                wy[0] = wy[1];
                wy[1] = wy[2];
                wy[2] = wy[3];
                // y[t - 4q - 5] enters
                wy[3] = L.yw[k][(int)(lo + s - 4 * q - 5) & kRing];
            }
            const double nx = quad_dpp<kQuadFromNext>(st[0]);
            st[0] = __builtin_fma(-(double)c4.x, yb, st[1]);
            st[1] = __builtin_fma(-(double)c4.y, yb, st[2]);
            st[2] = __builtin_fma(-(double)c4.z, yb, st[3]);
            st[3] = __builtin_fma(-(double)c4.w, yb, q == 3 ? 0.0 : nx);
        }
        qs_sync();
        qs_flush(L, gx, lo);
        if constexpr (GA)
            qs_flush_ga(L, ga, lo);
        if (lo > 0) {
            qs_commit(L, r);
            if constexpr (GA)
                qs_commit_y<kQuadRun>(L, r, lo - kQuadRun - 17);
        }
        qs_sync();
    }
    if (valid && it.chunk == 0 && gyi != nullptr) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            gyi[sd.ic_off + 4 * q + i] = (float)st[i];
    }
}

}  // namespace filt_detail
