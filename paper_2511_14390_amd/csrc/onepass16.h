// onepass16.h -- single-pass chunked scan for the batched plan's orders 5..16.
//
// Same structure as onepass.h (one launch per direction over tiles taken by
// ticket, decoupled look-back across tiles), for orders up to 16: a tile is
// P = 16 sub-chunks of L samples, handled by one workgroup of 16 DPP rows
// (256 threads), and the sub-chunk maps live in LDS instead of registers.
//
// Summaries without a driven solve.  A sub-chunk's forward map is
// state_out = Phi state_in + G x.  By duality (the adjoint of Sec. 3.1 Eq. 7
// run over the sub-chunk alone), the adjoint solve seeded with the unit
// state s_{i+1} = 1 at the sub-chunk's end -- which is the cotangent of
// state_out[i] -- leaves the adjoint state row i of Phi at its start, and
// its ybar sequence is row i of G, so s[i] = sum_t ybar_i[t] x[t] comes from
// one extra FMA per step.  Row lane i runs that solve (the coefficient
// broadcast of summary.h's row solves), 16 lanes give all of Phi and s, and
// no lane runs a separate driven solve.  The backward mirrors it: the
// adjoint map of a sub-chunk is Phi^T, and forward solve j from the unit
// state e_j gives its row j (the final state) and the driven part
// sum_t gy[t] y_j[t].
//
// Per tile: stage rows and signal in LDS; 16 row summaries; the tile map as
// a chain of 16 x 16 products over the sub-chunks (one entry per thread);
// publish, look back (wavefront 0), publish the inclusive state; entering
// states of the sub-chunks by a chain of matrix-vector products; the
// sub-chunk recursions from LDS on lane quads (four taps a lane, quad
// butterfly sums, as apply.h), outputs through LDS.
#pragma once

#include "onepass.h"
#include "summary.h"

namespace filt_detail {

constexpr int kTicketRun16 = 1;  // tickets per atomic (tickets held ahead delay the tiles waiting on them)

struct OnePass16 {
    static constexpr int P = 16;            // sub-chunks (DPP rows) per tile
    static constexpr int L = 32;            // samples per sub-chunk
    static constexpr int S = P * L;         // samples per tile
    static constexpr int CS = L * 16 + 16;  // LDS floats per sub-chunk, rows (padding spreads banks)
    static constexpr int XS = L + 1;        // LDS floats per sub-chunk, signal
    static constexpr int YS = 16 + L + 1;   // LDS floats per sub-chunk, y with 16 of history
    static constexpr int MS = 17;           // LDS doubles per map row: Phi[i][0..15], s[i]
    static constexpr int REC = 16 * 16 + 16;
    static constexpr int kThreads = 256;
};

// Stage rows [n][N] (N <= 16) as [P][L][16] with the padded sub-chunk
// stride; every load of the tile is issued before the first LDS store.
__device__ __forceinline__ void stage_rows16(float *cs, const float *__restrict__ a,
                                             int64_t a_off, int64_t t0, const FrameDiv &fd, int n,
                                             int N, int t)
{
    using G = OnePass16;
    if (N == 16 && (a_off % 4) == 0) {
        constexpr int K = G::S * 4 / G::kThreads;
        const int nv = n * 4;  // float4 pieces of the valid rows
        float4 val[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int v = t + G::kThreads * i;
            val[i] = v < nv ? *reinterpret_cast<const float4 *>(
                                  a + tile_row(a_off, t0, fd, v >> 2, 16) + 4 * (v & 3))
                            : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int v = t + G::kThreads * i;
            const int r = v >> 2, part = v & 3;
            *reinterpret_cast<float4 *>(cs + (r / G::L) * G::CS + (r % G::L) * 16 + 4 * part) =
                val[i];
        }
    } else {
        constexpr int K = G::S * 16 / G::kThreads;
        float val[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int e = t + G::kThreads * i;
            const int r = e >> 4, tap = e & 15;
            val[i] = (r < n && tap < N) ? a[tile_row(a_off, t0, fd, r, N) + tap] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int e = t + G::kThreads * i;
            const int r = e >> 4, tap = e & 15;
            cs[(r / G::L) * G::CS + (r % G::L) * 16 + tap] = val[i];
        }
    }
}

// A signal's n samples (zero past n) as [P][L] with row stride XS.
__device__ __forceinline__ void stage_signal16(float *xs, const float *__restrict__ src, int n,
                                               int t)
{
    using G = OnePass16;
    constexpr int K = G::S / G::kThreads;
    float v[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int e = t + G::kThreads * i;
        v[i] = e < n ? src[e] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int e = t + G::kThreads * i;
        xs[(e / G::L) * G::XS + (e % G::L)] = v[i];
    }
}

// The tile map as a chain over the sub-chunk maps in LDS (maps[p][i][0..16]),
// applied in order p = first, first + dir, ...: A <- map_p after A.  Thread
// (i, j) forms entry (i, j); threads with j == 0 also the offset column.
// Result in buf (one of the two buffers; returned).
__device__ __forceinline__ double *chain_maps(const double *maps, double *buf0, double *buf1,
                                              int first, int dir, int t)
{
    using G = OnePass16;
    const int i = t >> 4, j = t & 15;
    double *A = buf0, *B = buf1;
    {
        const double *m = maps + first * 16 * G::MS;
        A[i * G::MS + j] = m[i * G::MS + j];
        if (j == 0)
            A[i * G::MS + 16] = m[i * G::MS + 16];
    }
    __syncthreads();
    for (int step = 1; step < G::P; ++step) {
        const double *m = maps + (first + dir * step) * 16 * G::MS + i * G::MS;
        double v = 0.0, q = m[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const double mc = m[c];
            v = __builtin_fma(mc, A[c * G::MS + j], v);
            q = __builtin_fma(mc, A[c * G::MS + 16], q);
        }
        B[i * G::MS + j] = v;
        if (j == 0)
            B[i * G::MS + 16] = q;
        __syncthreads();
        double *tmp = A;
        A = B;
        B = tmp;
    }
    return A;
}

// Look-back of a 16-wide tile by wavefront 0 (lanes 0..63), one aggregate
// staged at a time in `stage` (REC doubles).  Result state in st (16 doubles
// of LDS), written by lanes 0..15.
template <bool REV>
__device__ __forceinline__ void look_back16(const OnePassArgs &A, int64_t tile_base, int64_t k,
                                            int64_t ntile, const double *init, int lane,
                                            double *stage, double *st)
{
    using G = OnePass16;
    const int64_t step = REV ? 1 : -1;
    int64_t base = k + step;
    int64_t found = -2;
    int spins = 0;
    for (;;) {
        const int64_t j = base + step * lane;
        const bool out = REV ? j >= ntile : j < 0;
        const int f = out ? 2 : flag_load(&A.flag[tile_base + j]);
        const uint64_t inc = __ballot(f == 2);
        const uint64_t none = __ballot(f == 0);
        const int first = inc ? __ffsll((unsigned long long)inc) - 1 : 64;
        const uint64_t before = first >= 64 ? ~0ull : ((1ull << first) - 1);
        if (none & before) {
            if (++spins > kSpinLimit) {
                if (lane == 0)
                    atomicAdd(A.timeouts, 1);
                found = -3;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        if (first < 64) {
            const int64_t jf = base + step * first;
            found = (REV ? jf >= ntile : jf < 0) ? -1 : jf;
            break;
        }
        base += 64 * step;
    }
    double s = 0.0;  // lane i < 16: component i
    if (lane < 16) {
        if (found >= 0)
            s = rec_load(&A.inc[(tile_base + found) * 16 + lane]);
        else if (found == -1)
            s = init[lane];
    }
    if (found >= -1) {
        int64_t next = found >= 0 ? found - step : (REV ? ntile - 1 : 0);
        int64_t left = REV ? next - k : k - next;
        while (left > 0) {
            const double *g = A.agg + (tile_base + next) * G::REC;
            for (int e = lane; e < G::REC; e += 64)
                stage[e] = rec_load(&g[e]);
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            // broadcast the current state through LDS, then one row per lane
            if (lane < 16)
                stage[G::REC + lane] = s;
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
            __builtin_amdgcn_wave_barrier();
            if (lane < 16) {
                double acc = stage[16 * 16 + lane];
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    acc = __builtin_fma(stage[lane * 16 + c], stage[G::REC + c], acc);
                s = acc;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
            __builtin_amdgcn_wave_barrier();
            next -= step;
            --left;
        }
    }
    if (lane < 16)
        st[lane] = s;
}

// Publish the tile map (MS-strided rows in LDS) as a REC record, flag 1.
__device__ __forceinline__ void publish_aggregate16(const OnePassArgs &A, int64_t rec,
                                                    const double *map, int t)
{
    using G = OnePass16;
    double *g = A.agg + rec * G::REC;
    rec_store(&g[t], map[(t >> 4) * G::MS + (t & 15)]);
    if (t < 16)
        rec_store(&g[256 + t], map[t * G::MS + 16]);
    wait_stores();  // every wavefront's share, before the barrier
    __syncthreads();
    if (t == 0)
        flag_store(&A.flag[rec], 1);
}

// ------------------------------------------------------------------ forward

__global__ void __launch_bounds__(256)
kb_onepass16_fwd(OnePassArgs A, const float *__restrict__ x, const float *__restrict__ a,
                 const float *__restrict__ yi, float *__restrict__ y)
{
    using G = OnePass16;
    constexpr int L = G::L;
    __shared__ __align__(16) float cs[G::P * G::CS];
    __shared__ float xs[G::P * G::XS];
    __shared__ double maps[G::P * 16 * G::MS];
    __shared__ double buf[2][16 * G::MS + 16];
    __shared__ double st[16];
    __shared__ int tk;
    const int t = threadIdx.x;
    const int row = t >> 4, j = t & 15;
    const int q = (int)(blockIdx.x % (unsigned)A.nlists);
    int *const counter = A.ticket + q * kTicketStride;
    const int64_t lo = A.list_off[q], ln = A.list_off[q + 1] - lo;
    int64_t tkt = 0, run_end = 0;
    for (;;) {
        if (tkt == run_end) {
            if (t == 0)
                tk = atomicAdd(counter, kTicketRun16);
            __syncthreads();
            tkt = tk;
            run_end = tkt + kTicketRun16;
            __syncthreads();
        }
        if (tkt >= ln)
            return;
        const int2 it = A.tiles[lo + tkt++];
        const SegDesc sd = A.segs[it.x];
        const int64_t k = it.y;
        const int64_t t0 = k * G::S;
        const int n = (int)min<int64_t>(G::S, sd.T - t0);
        const int N = sd.N;
        const int64_t rec = sd.tile_base + k;

        // 1. stage
        stage_signal16(xs, x + sd.x_off + t0, n, t);
        stage_rows16(cs, a, sd.a_off, t0, sd.fd, n, N, t);
        __syncthreads();

        // 2. row summaries: adjoint solve j of sub-chunk `row`, seeded with
        // s_{j+1} = 1 at its end; s_k before relative step s sits in
        // ss[(k - s) & 15]; the first step is s = L - 1 = 15 (mod 16)
        {
            const float *crow = cs + row * G::CS + j;
            const float *xr = xs + row * G::XS;
            double ss[16];
#pragma unroll
            for (int e = 0; e < 16; ++e)
                ss[e] = e == ((j + 2) & 15) ? 1.0 : 0.0;
            double acc = 0.0;
            for (int rel = L - 16; rel >= 0; rel -= 16) {
                static_for<16>([&](auto I) {
                    constexpr int s = 15 - decltype(I)::value;
                    const double cf = -(double)crow[(rel + s) * 16];
                    const double yb = ss[(1 - s) & 15];
                    acc = __builtin_fma(yb, (double)xr[rel + s], acc);
                    row_bwd_step<s>(cf, ss);
                    __builtin_amdgcn_sched_barrier(0);
                });
            }
            // after the sub-chunk's first step s_k sits in ss[(k + 1) & 15]
            double *mrow = maps + (row * 16 + j) * G::MS;
#pragma unroll
            for (int i = 0; i < 16; ++i)
                mrow[i] = ss[(i + 2) & 15];
            mrow[16] = acc;
        }
        __syncthreads();

        // 3. tile map: sub-chunk 0 first
        const double *tile = chain_maps(maps, buf[0], buf[1], 0, 1, t);

        // 4. look-back (the state entering the segment is yi)
        double *other = buf[tile == buf[0]];
        if (k > 0) {
            publish_aggregate16(A, rec, tile, t);
            if (t < 64) {
                double init[16];
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    init[i] = (yi != nullptr && i < N) ? (double)yi[sd.ic_off + i] : 0.0;
                look_back16<false>(A, sd.tile_base, k, sd.ntile, init, t, other, st);
            }
        } else if (t < 16) {
            st[t] = (yi != nullptr && t < N) ? (double)yi[sd.ic_off + t] : 0.0;
        }
        __syncthreads();
        // inclusive state, then the entering states of the sub-chunks (in
        // the buffer the look-back staged through)
        double *sv = other;
        if (t < 16) {
            if (k + 1 < sd.ntile) {
                double acc = tile[t * G::MS + 16];
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    acc = __builtin_fma(tile[t * G::MS + c], st[c], acc);
                rec_store(&A.inc[rec * 16 + t], acc);
                wait_stores();
                if (t == 0)
                    flag_store(&A.flag[rec], 2);
            }
            sv[t] = st[t];
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
            __builtin_amdgcn_wave_barrier();
            for (int p = 0; p + 1 < G::P; ++p) {
                const double *m = maps + (p * 16 + t) * G::MS;
                double acc = m[16];
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    acc = __builtin_fma(m[c], sv[p * 16 + c], acc);
                sv[(p + 1) * 16 + t] = acc;
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();

        // 5. apply on quads: wavefront w runs sub-chunks 4w .. 4w + 3 on its
        // lanes 0..15 (quad q of sub-chunk p owns taps 4q + 1 .. 4q + 4)
        if ((t & 63) < 16) {
            const int p = 4 * (t >> 6) + ((t & 15) >> 2), q = t & 3;
            double w[4];  // w[i] = y[t - 4q - 1 - i]
#pragma unroll
            for (int i = 0; i < 4; ++i)
                w[i] = sv[p * 16 + 4 * q + i];
            const float *cp = cs + p * G::CS + 4 * q;
            float *xp = xs + p * G::XS;
#pragma unroll 4
            for (int s = 0; s < L; ++s) {
                const float4 a4 = *reinterpret_cast<const float4 *>(cp + s * 16);
                double pr = -(double)a4.w * w[3];
                pr = __builtin_fma(-(double)a4.z, w[2], pr);
                pr = __builtin_fma(-(double)a4.y, w[1], pr);
                pr = __builtin_fma(-(double)a4.x, w[0], pr);
                double tot = pr + quad_dpp<kQuadXor1>(pr);
                tot = tot + quad_dpp<kQuadXor2>(tot);
                const double v = (double)xp[s] + tot;
                const double prev = quad_dpp<kQuadFromPrev>(w[3]);
                w[3] = w[2];
                w[2] = w[1];
                w[1] = w[0];
                w[0] = q == 0 ? v : prev;
                if (q == 0)
                    xp[s] = (float)v;
            }
        }
        __syncthreads();
        for (int e = t; e < n; e += G::kThreads)
            y[sd.x_off + t0 + e] = xs[(e / L) * G::XS + (e % L)];
        __syncthreads();
    }
}

// ----------------------------------------------------------------- backward

__global__ void __launch_bounds__(256)
kb_onepass16_bwd(OnePassArgs A, const float *__restrict__ gy, const float *__restrict__ a,
                 const float *__restrict__ y, const float *__restrict__ yi,
                 float *__restrict__ gx, float *__restrict__ ga, float *__restrict__ gyi)
{
    using G = OnePass16;
    constexpr int L = G::L;
    __shared__ __align__(16) float cs[G::P * G::CS];
    __shared__ float gs[G::P * G::XS];
    __shared__ float ys[G::P * G::YS];
    __shared__ double maps[G::P * 16 * G::MS];
    __shared__ double buf[2][16 * G::MS + 16];
    __shared__ double st[16];
    __shared__ int tk;
    const int t = threadIdx.x;
    const int row = t >> 4, j = t & 15;
    const int q = (int)(blockIdx.x % (unsigned)A.nlists);
    int *const counter = A.ticket + q * kTicketStride;
    const int64_t lo = A.list_off[q], ln = A.list_off[q + 1] - lo;
    int64_t tkt = 0, run_end = 0;
    for (;;) {
        if (tkt == run_end) {
            if (t == 0)
                tk = atomicAdd(counter, kTicketRun16);
            __syncthreads();
            tkt = tk;
            run_end = tkt + kTicketRun16;
            __syncthreads();
        }
        if (tkt >= ln)
            return;
        const int2 it = A.tiles[lo + tkt++];
        const SegDesc sd = A.segs[it.x];
        const int64_t k = it.y;
        const int64_t t0 = k * G::S;
        const int n = (int)min<int64_t>(G::S, sd.T - t0);
        const int N = sd.N;
        const int64_t rec = sd.tile_base + k;
        // per-sample ga rows are formed here; frame-held rows get theirs
        // from the stored adjoint in a separate pass
        const bool want_ga = ga != nullptr && sd.fd.m == 0;

        // 1. stage gy, rows, and y with 16 samples of history per sub-chunk
        stage_signal16(gs, gy + sd.x_off + t0, n, t);
        stage_rows16(cs, a, sd.a_off, t0, sd.fd, n, N, t);
        if (want_ga) {
            // positions -16 .. S-1 of the tile: K per thread, one more for
            // threads below 16
            constexpr int K = G::S / G::kThreads;
            float v[K + 1];
#pragma unroll
            for (int i = 0; i <= K; ++i) {
                const int e = t - 16 + G::kThreads * i;
                const int64_t tt = t0 + e;
                v[i] = 0.f;
                if (e < n && (i < K || t < 16)) {
                    if (tt >= 0)
                        v[i] = y[sd.x_off + tt];
                    else if (yi != nullptr && -tt <= N)
                        v[i] = yi[sd.ic_off + (-tt - 1)];
                }
            }
#pragma unroll
            for (int i = 0; i <= K; ++i) {
                const int e = t - 16 + G::kThreads * i;
                if (i < K || t < 16) {
                    const int p = e >= 0 ? e / L : -1, r = e - p * L;
                    if (p >= 0)
                        ys[p * G::YS + 16 + r] = v[i];
                    if (r >= L - 16 && p + 1 < G::P)
                        ys[(p + 1) * G::YS + (r - (L - 16))] = v[i];
                }
            }
        }
        __syncthreads();

        // 2. row summaries: forward solve j of sub-chunk `row` from the unit
        // state y(start - 1 - j) = 1; h[t & 15] = y_j[t]; the driven part of
        // the adjoint map is sum_t gy[t] y_j[t]
        {
            const float *crow = cs + row * G::CS + j;
            const float *gr = gs + row * G::XS;
            double h[16];
#pragma unroll
            for (int e = 0; e < 16; ++e)
                h[e] = e == ((-1 - j) & 15) ? 1.0 : 0.0;
            double acc = 0.0;
            for (int rel = 0; rel < L; rel += 16) {
                static_for<16>([&](auto I) {
                    constexpr int s = decltype(I)::value;
                    const double cf = -(double)crow[(rel + s) * 16];
                    h[s] = row_fwd_step<s>(cf, h);
                    acc = __builtin_fma(h[s], (double)gr[rel + s], acc);
                    __builtin_amdgcn_sched_barrier(0);
                });
            }
            // y_j(end - 1 - i) = h[15 - i] = Phi[i][j] = adjoint map [j][i]
            double *mrow = maps + (row * 16 + j) * G::MS;
#pragma unroll
            for (int i = 0; i < 16; ++i)
                mrow[i] = h[15 - i];
            mrow[16] = acc;
        }
        __syncthreads();

        // 3. tile map: the last sub-chunk first
        const double *tile = chain_maps(maps, buf[0], buf[1], G::P - 1, -1, t);

        // 4. look-back over the later tiles; nothing enters the last one
        double *other = buf[tile == buf[0]];
        if (k + 1 < sd.ntile) {
            publish_aggregate16(A, rec, tile, t);
            if (t < 64) {
                double zero[16];
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    zero[i] = 0.0;
                look_back16<true>(A, sd.tile_base, k, sd.ntile, zero, t, other, st);
            }
        } else if (t < 16) {
            st[t] = 0.0;
        }
        __syncthreads();
        double *sv = other;  // adjoint state entering each sub-chunk at its end
        if (t < 16) {
            if (k > 0) {
                double acc = tile[t * G::MS + 16];
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    acc = __builtin_fma(tile[t * G::MS + c], st[c], acc);
                rec_store(&A.inc[rec * 16 + t], acc);
                wait_stores();
                if (t == 0)
                    flag_store(&A.flag[rec], 2);
            }
            sv[(G::P - 1) * 16 + t] = st[t];
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
            __builtin_amdgcn_wave_barrier();
            for (int p = G::P - 1; p > 0; --p) {
                const double *m = maps + (p * 16 + t) * G::MS;
                double acc = m[16];
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    acc = __builtin_fma(m[c], sv[p * 16 + c], acc);
                sv[(p - 1) * 16 + t] = acc;
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();

        // 5. adjoint on quads from the sub-chunk's top state: lane q keeps
        // s_{4q+1..4q+4}; ybar = gy + s_1 (lane 0 of the quad); s_k <- s_{k+1}
        // - a_k ybar, s_{4q+5} from lane q + 1.  gx = ybar into gs, the ga row
        // over the coefficient row it was read from.
        if ((t & 63) < 16) {
            const int p = 4 * (t >> 6) + ((t & 15) >> 2), q = t & 3;
            double s4[4];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                s4[i] = sv[p * 16 + 4 * q + i];
            float *cp = cs + p * G::CS + 4 * q;
            float *gp = gs + p * G::XS;
            const float *yp = ys + p * G::YS + 16 - 4 * q;  // y(t - 4q - i - 1) = yp[s - 1 - i]
#pragma unroll 4
            for (int s = L - 1; s >= 0; --s) {
                const float4 a4 = *reinterpret_cast<const float4 *>(cp + s * 16);
                const double s1 = quad_dpp<kQuadLane0>(s4[0]);
                const double yb = (double)gp[s] + s1;
                // the DPP move runs on every lane of the quad (lane 2 reads
                // lane 3); only then is lane 3's value replaced by zero
                const double nx = quad_dpp<kQuadFromNext>(s4[0]);
                const double nxt = q == 3 ? 0.0 : nx;
                s4[0] = __builtin_fma(-(double)a4.x, yb, s4[1]);
                s4[1] = __builtin_fma(-(double)a4.y, yb, s4[2]);
                s4[2] = __builtin_fma(-(double)a4.z, yb, s4[3]);
                s4[3] = __builtin_fma(-(double)a4.w, yb, nxt);
                if (want_ga) {
                    float4 g4;
                    g4.x = (float)(-yb * (double)yp[s - 1]);
                    g4.y = (float)(-yb * (double)yp[s - 2]);
                    g4.z = (float)(-yb * (double)yp[s - 3]);
                    g4.w = (float)(-yb * (double)yp[s - 4]);
                    *reinterpret_cast<float4 *>(cp + s * 16) = g4;
                }
                if (q == 0)
                    gp[s] = (float)yb;
            }
            if (k == 0 && p == 0 && gyi != nullptr) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (4 * q + i < N)
                        gyi[sd.ic_off + 4 * q + i] = (float)s4[i];
            }
        }
        __syncthreads();
        if (gx != nullptr)
            for (int e = t; e < n; e += G::kThreads)
                gx[sd.x_off + t0 + e] = gs[(e / L) * G::XS + (e % L)];
        if (want_ga) {
            const int64_t a0 = sd.a_off + t0 * N;
            if (N == 16 && (a0 % 4) == 0) {
                for (int v = t; v < n * 4; v += G::kThreads) {
                    const int r = v >> 2, part = v & 3;
                    *reinterpret_cast<float4 *>(ga + a0 + 4 * (int64_t)v) =
                        *reinterpret_cast<const float4 *>(cs + (r / L) * G::CS + (r % L) * 16 +
                                                          4 * part);
                }
            } else {
                for (int e = t; e < n * N; e += G::kThreads) {
                    const int r = e / N, tap = e - r * N;
                    ga[a0 + e] = cs[(r / L) * G::CS + (r % L) * 16 + tap];
                }
            }
        }
        __syncthreads();
    }
}

}  // namespace filt_detail
