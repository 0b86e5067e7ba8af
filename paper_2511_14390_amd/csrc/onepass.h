// onepass.h -- single-pass chunked scan for the batched plan's low orders.
//
// The three-phase scan (summaries, carry, apply; common.h) reads every input
// twice and walks the chunk states in separate launches.  For per-sample
// all-pole filters of order W <= 4 the whole forward (or backward) of a
// segment instead runs as one launch over tiles, each tile handled by one
// wavefront from start to end:
//
//   1. stage the tile's signal and coefficient rows in LDS (coalesced);
//   2. every lane summarises its sub-chunk of L samples as the affine map
//      state_out = Phi state_in + s (Sec. 2 Eq. 4 companion steps; W unit
//      solves and one driven solve, all in FP64 registers);
//   3. an inclusive scan of the 64 maps across the wavefront (Sec. 3.2
//      operator: later map after earlier) gives every lane its prefix and
//      the tile its aggregate map;
//   4. decoupled look-back across tiles: the tile publishes its aggregate,
//      then walks back over its predecessors' flags until it finds one that
//      published its inclusive state, applies the aggregates in between and
//      publishes its own inclusive state;
//   5. every lane reruns its sub-chunk from its exact entering state out of
//      LDS and the tile's outputs leave through LDS with coalesced stores.
//
// Tiles take their order from atomic ticket counters, each over a list in
// which every tile comes after the tiles it waits for, so a wavefront only
// ever waits for wavefronts that hold a smaller ticket of the same list and
// are therefore running or done.  The bucket's segments are split over
// kOnePassLists such lists (whole segments, balanced by tile count; a
// tile's predecessors are in its own list), workgroup g serving list
// g mod kOnePassLists: one counter per list instead of one for the launch,
// since every ticket is an atomic at the device's coherence point and a
// single counter serialises them all.  Every wait is bounded: past
// kSpinLimit polls it counts a timeout and goes on with a zero state, so the
// kernel always ends (the result is then wrong and the counter says so).
//
// The backward is the same structure in reverse time on the adjoint
// (transposed form, Sec. 3.1 Eq. 7), tiles waiting for their successors,
// and the apply also forms gx = ybar (b = [1]), the per-sample
// ga_k[t] = -ybar[t] y[t-k] (Eq. 9 per sample) and, on the first tile, gyi.
#pragma once

#include "batched.h"

namespace filt_detail {

template <int W>
struct OnePass {
    static constexpr int L = W <= 2 ? 32 : 16; // samples per lane (sub-chunk)
    static constexpr int S = 64 * L;           // samples per tile
    static constexpr int XS = L + 1;           // LDS floats per lane, signal
    static constexpr int YS = W + L + 1;       // LDS floats per lane, y with W of history
    static constexpr int CS = L * W + 4;       // LDS floats per lane, rows (16-byte aligned)
    static constexpr int REC = W * W + W;      // doubles of one affine map
    static constexpr int kLook = 32;           // aggregates staged per look-back round
};

constexpr int kOnePassMaxW = 4;
constexpr int kSpinLimit = 1 << 22;
constexpr int kOnePassLists = 8;   // ticket lists of a launch (orders up to 4)
constexpr int kTicketStride = 32;  // ints between two lists' counters (128 bytes)

struct OnePassArgs {
    const SegDesc *segs;
    const int2 *tiles;  // (segment, tile): the lists one after another, each in ticket order
    int64_t ntiles;
    double *agg;        // per tile: aggregate map (REC doubles)
    double *inc;        // per tile: inclusive state (W doubles)
    int *flag;          // per tile: 0 none, 1 aggregate, 2 inclusive
    int *ticket;        // list q's counter at ticket[q * kTicketStride] (zero at launch)
    int *timeouts;      // bounded waits that ran out
    int nlists;         // lists in use (1 .. kOnePassLists)
    int64_t list_off[kOnePassLists + 1];  // list q: tiles[list_off[q] .. list_off[q + 1])
};

// Records shared between workgroups (flags, aggregates, inclusive states)
// move through device-coherent accesses: relaxed atomic loads and stores at
// agent scope carry the sc1 bit, so they go to and come from the coherence
// point shared by all XCDs without touching the rest of the caches.  (An
// acquire or release at agent scope would instead invalidate or write back
// the whole L2 of the XCD on every poll and publish.)  A publisher waits for
// its record stores to complete (vmcnt 0) before it stores the flag; a
// reader issues its record loads only after the flag it polled has arrived.
__device__ __forceinline__ int flag_load(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void flag_store(int *p, int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double rec_load(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void rec_store(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until this wavefront's stores have completed (are visible at device
// scope for sc1 stores); also a compiler barrier for memory.
__device__ __forceinline__ void wait_stores()
{
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// An affine map of the state: out = P in + v.
template <int W>
struct Affine {
    double P[W][W];
    double v[W];
};

template <int W>
__device__ __forceinline__ Affine<W> affine_identity()
{
    Affine<W> r;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        r.v[i] = 0.0;
#pragma unroll
        for (int j = 0; j < W; ++j)
            r.P[i][j] = i == j ? 1.0 : 0.0;
    }
    return r;
}

// later after earlier: (P_l P_e, P_l v_e + v_l)
template <int W>
__device__ __forceinline__ Affine<W> affine_then(const Affine<W> &earlier, const Affine<W> &later)
{
    Affine<W> r;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        double acc = later.v[i];
#pragma unroll
        for (int k = 0; k < W; ++k)
            acc = __builtin_fma(later.P[i][k], earlier.v[k], acc);
        r.v[i] = acc;
#pragma unroll
        for (int j = 0; j < W; ++j) {
            double p = 0.0;
#pragma unroll
            for (int k = 0; k < W; ++k)
                p = __builtin_fma(later.P[i][k], earlier.P[k][j], p);
            r.P[i][j] = p;
        }
    }
    return r;
}

template <int W>
__device__ __forceinline__ void affine_apply(const Affine<W> &f, const double (&s)[W],
                                             double (&out)[W])
{
#pragma unroll
    for (int i = 0; i < W; ++i) {
        double acc = f.v[i];
#pragma unroll
        for (int k = 0; k < W; ++k)
            acc = __builtin_fma(f.P[i][k], s[k], acc);
        out[i] = acc;
    }
}

// The map of lane `src` (shuffled; width 64).  DOWN: from lane + d, else
// lane - d.
template <int W, bool DOWN>
__device__ __forceinline__ Affine<W> affine_shfl(const Affine<W> &f, int d)
{
    Affine<W> r;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        r.v[i] = DOWN ? __shfl_down(f.v[i], d, 64) : __shfl_up(f.v[i], d, 64);
#pragma unroll
        for (int j = 0; j < W; ++j)
            r.P[i][j] = DOWN ? __shfl_down(f.P[i][j], d, 64) : __shfl_up(f.P[i][j], d, 64);
    }
    return r;
}

template <int W>
__device__ __forceinline__ Affine<W> affine_bcast(const Affine<W> &f, int lane)
{
    Affine<W> r;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        r.v[i] = __shfl(f.v[i], lane, 64);
#pragma unroll
        for (int j = 0; j < W; ++j)
            r.P[i][j] = __shfl(f.P[i][j], lane, 64);
    }
    return r;
}

// Inclusive scan of the lanes' maps in time order: ascending lanes
// (forward) or descending lanes (backward, DOWN).
template <int W, bool DOWN>
__device__ __forceinline__ Affine<W> wave_scan(Affine<W> f, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const Affine<W> o = affine_shfl<W, DOWN>(f, d);
        const bool has = DOWN ? lane + d < 64 : lane >= d;
        if (has)
            f = affine_then<W>(o, f);
    }
    return f;
}

// Stage n samples of a signal (zero past n) into LDS as [64 lanes][L] with
// row stride XS.  Every load of the tile is issued before the first LDS
// store, so the tile costs one memory latency, not one per load.
template <int S, int L, int XS>
__device__ __forceinline__ void stage_signal(float *xs, const float *__restrict__ src, int n,
                                             int lane)
{
    constexpr int K = S / 64;
    float v[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int e = lane + 64 * i;
        v[i] = e < n ? src[e] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int e = lane + 64 * i;
        xs[(e / L) * XS + (e % L)] = v[i];
    }
}

// Start of the coefficient row of tile sample r (tile start t0): per-sample
// rows follow the samples, frame-held rows (fd.m != 0) their frames.
__device__ __forceinline__ int64_t tile_row(int64_t a_off, int64_t t0, const FrameDiv &fd, int r,
                                            int N)
{
    const int64_t t = t0 + r;
    return a_off + (fd.m != 0 ? (int64_t)frame_of(fd, (uint32_t)t) : t) * N;
}

// Stage the tile's coefficient rows [n][N] into LDS as [64 lanes][L][W]
// (zero taps past N and rows past n); loads first, then the LDS stores.
// Per-sample rows of order W (>= 4 or whole float4 pieces of several rows)
// load as vectors; frame-held rows as vectors only when a row is one float4.
template <int W>
__device__ __forceinline__ void stage_rows(float *cs, const float *__restrict__ a, int64_t a_off,
                                           int64_t t0, const FrameDiv &fd, int n, int N,
                                           int lane)
{
    using G = OnePass<W>;
    constexpr int L = G::L;
    const int64_t a0 = a_off + t0 * N;
    if (fd.m != 0 && N == 4 && W == 4 && (a_off % 4) == 0) {
        constexpr int K = G::S / 64;  // one float4 (a row) per sample
        float4 val[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int r = lane + 64 * i;
            val[i] = r < n ? *reinterpret_cast<const float4 *>(a + tile_row(a_off, t0, fd, r, 4))
                           : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int r = lane + 64 * i;
            *reinterpret_cast<float4 *>(cs + (r / L) * G::CS + (r % L) * W) = val[i];
        }
    } else if (fd.m == 0 && N == W && (a0 % 4) == 0 && (W * L) % 4 == 0) {
        // whole float4 pieces of rows below n; the rest one float at a time
        constexpr int K = G::S * W / 4 / 64;
        const int nv = (n * W) / 4;
        float4 val[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int v = lane + 64 * i;
            const int e = 4 * v;
            val[i] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (v < nv) {
                val[i] = *reinterpret_cast<const float4 *>(a + a0 + e);
            } else if (e < n * W) {
                float t4[4] = {0.f, 0.f, 0.f, 0.f};
                for (int q = 0; q < 4 && e + q < n * W; ++q)
                    t4[q] = a[a0 + e + q];
                val[i] = make_float4(t4[0], t4[1], t4[2], t4[3]);
            }
        }
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int e = 4 * (lane + 64 * i);
            const int r = e / W, p = r / L, rr = r % L;
            *reinterpret_cast<float4 *>(cs + p * G::CS + rr * W + (e % W)) = val[i];
        }
    } else {
        constexpr int K = G::S * W / 64;
        float val[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int e = lane + 64 * i;
            const int r = e / W, tap = e % W;
            val[i] = (r < n && tap < N) ? a[tile_row(a_off, t0, fd, r, N) + tap] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const int e = lane + 64 * i;
            const int r = e / W, tap = e % W;
            cs[(r / L) * G::CS + (r % L) * W + tap] = val[i];
        }
    }
}

// Coefficient row s of this lane, converted: c[k] = a_k (k = 1..W).
template <int W>
__device__ __forceinline__ void lds_row(const float *cl, int s, double (&c)[W + 1])
{
    c[0] = 0.0;
    if constexpr (W == 4) {
        const float4 v = *reinterpret_cast<const float4 *>(cl + s * 4);
        c[1] = v.x;
        c[2] = v.y;
        c[3] = v.z;
        c[4] = v.w;
    } else if constexpr (W == 2) {
        const float2 v = *reinterpret_cast<const float2 *>(cl + s * 2);
        c[1] = v.x;
        c[2] = v.y;
    } else {
#pragma unroll
        for (int k = 0; k < W; ++k)
            c[k + 1] = cl[s * W + k];
    }
}

// Look-back.  Tile k of a segment (tile_base + k its record) finds its
// entering state: walks over the tiles that come before it in time -- k - 1,
// k - 2, ... (forward) or k + 1, k + 2, ... (backward, REV) -- until one has
// published its inclusive state, stages the aggregates in between through
// LDS and applies them in time order.  Past the segment's first (last) tile
// the state is `init`.  Every lane returns the same state.
template <int W, bool REV>
__device__ __forceinline__ void look_back(const OnePassArgs &A, int64_t tile_base, int64_t k,
                                          int64_t ntile, const double (&init)[W], int lane,
                                          double *stage, double (&S)[W])
{
    using G = OnePass<W>;
    const int64_t step = REV ? 1 : -1;
    int64_t base = k + step;  // nearest predecessor in time
    int64_t found = -2;       // tile whose inclusive state starts the walk (-1: init)
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
    if (found == -3) {
#pragma unroll
        for (int i = 0; i < W; ++i)
            S[i] = 0.0;
        return;
    }
    // start: the inclusive state of `found` (or init)
    if (found >= 0) {
#pragma unroll
        for (int i = 0; i < W; ++i)
            S[i] = rec_load(&A.inc[(tile_base + found) * W + i]);
    } else {
#pragma unroll
        for (int i = 0; i < W; ++i)
            S[i] = init[i];
    }
    // aggregates of the tiles strictly between `found` and k, in time order
    int64_t next = found >= 0 ? found - step : (REV ? ntile - 1 : 0);
    int64_t left = REV ? next - k : k - next;  // number of aggregates still to apply
    while (left > 0) {
        const int cnt = (int)min<int64_t>(left, G::kLook);
        for (int e = lane; e < cnt * G::REC; e += 64) {
            const int q = e / G::REC, r = e % G::REC;
            stage[e] = rec_load(&A.agg[(tile_base + next - step * q) * G::REC + r]);
        }
        __syncthreads();
        for (int q = 0; q < cnt; ++q) {
            const double *g = stage + q * G::REC;
            double Sn[W];
#pragma unroll
            for (int i = 0; i < W; ++i) {
                double acc = g[W * W + i];
#pragma unroll
                for (int c = 0; c < W; ++c)
                    acc = __builtin_fma(g[i * W + c], S[c], acc);
                Sn[i] = acc;
            }
#pragma unroll
            for (int i = 0; i < W; ++i)
                S[i] = Sn[i];
        }
        __syncthreads();
        next -= step * cnt;
        left -= cnt;
    }
}

// Publish: aggregate (flag 1) from lane `from`.
template <int W>
__device__ __forceinline__ void publish_aggregate(const OnePassArgs &A, int64_t rec,
                                                  const Affine<W> &f, int lane, int from)
{
    using G = OnePass<W>;
    if (lane == from) {
        double *g = A.agg + rec * G::REC;
#pragma unroll
        for (int i = 0; i < W; ++i) {
#pragma unroll
            for (int j = 0; j < W; ++j)
                rec_store(&g[i * W + j], f.P[i][j]);
            rec_store(&g[W * W + i], f.v[i]);
        }
        wait_stores();
        flag_store(&A.flag[rec], 1);
    }
}

template <int W>
__device__ __forceinline__ void publish_inclusive(const OnePassArgs &A, int64_t rec,
                                                  const double (&s)[W], int lane)
{
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < W; ++i)
            rec_store(&A.inc[rec * W + i], s[i]);
        wait_stores();
        flag_store(&A.flag[rec], 2);
    }
}

// One ticket per atomic, taken when the wavefront is free to start the
// tile (holding tickets ahead would make the tiles that wait for them wait
// longer: every delay before a tile publishes its aggregate holds up the
// tiles after it in the same segment).
__device__ __forceinline__ int64_t take_ticket(int *ticket, int lane)
{
    int t = 0;
    if (lane == 0)
        t = atomicAdd(ticket, 1);
    return __builtin_amdgcn_readfirstlane(__shfl(t, 0, 64));
}

// ------------------------------------------------------------------ forward

template <int W>
__global__ void __launch_bounds__(64)
kb_onepass_fwd(OnePassArgs A, const float *__restrict__ x, const float *__restrict__ a,
               const float *__restrict__ yi, float *__restrict__ y)
{
    using G = OnePass<W>;
    constexpr int L = G::L, m = W - 1;
    __shared__ float xs[64 * G::XS];
    __shared__ __align__(16) float cs[64 * G::CS];
    __shared__ double stage[G::kLook * G::REC];
    const int lane = threadIdx.x;
    const int q = (int)(blockIdx.x % (unsigned)A.nlists);
    int *const counter = A.ticket + q * kTicketStride;
    const int64_t lo = A.list_off[q], ln = A.list_off[q + 1] - lo;
    for (;;) {
        const int64_t tk = take_ticket(counter, lane);
        if (tk >= ln)
            return;
        const int2 it = A.tiles[lo + tk];
        const SegDesc sd = A.segs[it.x];
        const int64_t k = it.y;
        const int64_t t0 = k * G::S;
        const int n = (int)min<int64_t>(G::S, sd.T - t0);
        const int N = sd.N;
        const int64_t rec = sd.tile_base + k;

        // 1. stage
        stage_signal<G::S, L, G::XS>(xs, x + sd.x_off + t0, n, lane);
        stage_rows<W>(cs, a, sd.a_off, t0, sd.fd, n, N, lane);
        __syncthreads();
        const float *xl = xs + lane * G::XS;
        const float *cl = cs + lane * G::CS;

        // 2. summary: h[q][t & m] = y_q[t] of solve q (q < W: unit state
        // y(-1-q) = 1, no input; q = W: zero state, input x)
        double h[W + 1][W];
#pragma unroll
        for (int q = 0; q <= W; ++q)
#pragma unroll
            for (int e = 0; e < W; ++e)
                h[q][e] = (q < W && e == ((-1 - q) & m)) ? 1.0 : 0.0;
#pragma unroll
        for (int s = 0; s < L; ++s) {
            double c[W + 1];
            lds_row<W>(cl, s, c);
            const double u = xl[s];
#pragma unroll
            for (int q = 0; q <= W; ++q) {
                double acc = q == W ? u : 0.0;
#pragma unroll
                for (int kk = W; kk >= 1; --kk)
                    acc = __builtin_fma(-c[kk], h[q][(s - kk) & m], acc);
                h[q][s & m] = acc;
            }
        }
        // state index i = y(t_end - 1 - i) = h[.][m - i]
        Affine<W> f;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            f.v[i] = h[W][m - i];
#pragma unroll
            for (int j = 0; j < W; ++j)
                f.P[i][j] = h[j][m - i];
        }

        // 3. scan across the wavefront
        const Affine<W> incl = wave_scan<W, false>(f, lane);
        Affine<W> excl = affine_shfl<W, false>(incl, 1);
        if (lane == 0)
            excl = affine_identity<W>();
        const Affine<W> tile = affine_bcast<W>(incl, 63);

        // 4. look-back
        double init[W];
#pragma unroll
        for (int i = 0; i < W; ++i)
            init[i] = (yi != nullptr && i < N) ? (double)yi[sd.ic_off + i] : 0.0;
        double Sin[W];
        if (k == 0) {
#pragma unroll
            for (int i = 0; i < W; ++i)
                Sin[i] = init[i];
        } else {
            publish_aggregate<W>(A, rec, tile, lane, 63);
            look_back<W, false>(A, sd.tile_base, k, sd.ntile, init, lane, stage, Sin);
        }
        if (k + 1 < sd.ntile) {
            double So[W];
            affine_apply<W>(tile, Sin, So);
            publish_inclusive<W>(A, rec, So, lane);
        }

        // 5. apply from the lane's entering state
        double Se[W];
        affine_apply<W>(excl, Sin, Se);
        double hy[W];
#pragma unroll
        for (int i = 0; i < W; ++i)
            hy[(-1 - i) & m] = Se[i];
        float *xw = xs + lane * G::XS;
#pragma unroll
        for (int s = 0; s < L; ++s) {
            double c[W + 1];
            lds_row<W>(cl, s, c);
            double acc = xl[s];
#pragma unroll
            for (int kk = W; kk >= 1; --kk)
                acc = __builtin_fma(-c[kk], hy[(s - kk) & m], acc);
            hy[s & m] = acc;
            xw[s] = (float)acc;
        }
        __syncthreads();
        for (int e = lane; e < n; e += 64)
            y[sd.x_off + t0 + e] = xs[(e / L) * G::XS + (e % L)];
        __syncthreads();
    }
}

// ----------------------------------------------------------------- backward

template <int W>
__global__ void __launch_bounds__(64)
kb_onepass_bwd(OnePassArgs A, const float *__restrict__ gy, const float *__restrict__ a,
               const float *__restrict__ y, const float *__restrict__ yi,
               float *__restrict__ gx, float *__restrict__ ga, float *__restrict__ gyi)
{
    using G = OnePass<W>;
    constexpr int L = G::L;
    __shared__ float gs[64 * G::XS];
    __shared__ float ys[64 * G::YS];
    __shared__ __align__(16) float cs[64 * G::CS];
    __shared__ double stage[G::kLook * G::REC];
    const int lane = threadIdx.x;
    const int q = (int)(blockIdx.x % (unsigned)A.nlists);
    int *const counter = A.ticket + q * kTicketStride;
    const int64_t lo = A.list_off[q], ln = A.list_off[q + 1] - lo;
    for (;;) {
        const int64_t tk = take_ticket(counter, lane);
        if (tk >= ln)
            return;
        const int2 it = A.tiles[lo + tk];
        const SegDesc sd = A.segs[it.x];
        const int64_t k = it.y;
        const int64_t t0 = k * G::S;
        const int n = (int)min<int64_t>(G::S, sd.T - t0);
        const int N = sd.N;
        const int64_t rec = sd.tile_base + k;
        // per-sample ga rows are formed here; frame-held rows get theirs
        // from the stored adjoint in a separate pass
        const bool want_ga = ga != nullptr && sd.fd.m == 0;

        // 1. stage gy, the rows and y with W samples of history per lane
        stage_signal<G::S, L, G::XS>(gs, gy + sd.x_off + t0, n, lane);
        stage_rows<W>(cs, a, sd.a_off, t0, sd.fd, n, N, lane);
        if (want_ga) {
            // positions -W .. S-1 of the tile, K + 1 per lane (the last
            // round only for lanes below W)
            constexpr int K = G::S / 64;
            float v[K + 1];
#pragma unroll
            for (int i = 0; i <= K; ++i) {
                const int e = lane - W + 64 * i;
                const int64_t t = t0 + e;
                v[i] = 0.f;
                if (e < n && (i < K || lane < W)) {
                    if (t >= 0)
                        v[i] = y[sd.x_off + t];
                    else if (yi != nullptr && -t <= N)
                        v[i] = yi[sd.ic_off + (-t - 1)];
                }
            }
#pragma unroll
            for (int i = 0; i <= K; ++i) {
                const int e = lane - W + 64 * i;
                if (i < K || lane < W) {
                    // own lane's slot, and the history slot of the next lane
                    const int p = e >= 0 ? e / L : -1, r = e - p * L;
                    if (p >= 0)
                        ys[p * G::YS + W + r] = v[i];
                    if (r >= L - W && p + 1 < 64)
                        ys[(p + 1) * G::YS + (r - (L - W))] = v[i];
                }
            }
        }
        __syncthreads();
        const float *gl = gs + lane * G::XS;
        float *cl = cs + lane * G::CS;

        // 2. adjoint summary in reverse time: st[q][i] = s_{i+1}; q < W unit
        // state s_{q+1} = 1 at the top, no input; q = W zero state, input gy
        double st[W + 1][W];
#pragma unroll
        for (int q = 0; q <= W; ++q)
#pragma unroll
            for (int i = 0; i < W; ++i)
                st[q][i] = (q < W && i == q) ? 1.0 : 0.0;
#pragma unroll
        for (int s = L - 1; s >= 0; --s) {
            double c[W + 1];
            lds_row<W>(cl, s, c);
            const double g = gl[s];
#pragma unroll
            for (int q = 0; q <= W; ++q) {
                const double yb = (q == W ? g : 0.0) + st[q][0];
#pragma unroll
                for (int i = 0; i < W; ++i)
                    st[q][i] = __builtin_fma(-c[i + 1], yb, i + 1 < W ? st[q][i + 1] : 0.0);
            }
        }
        Affine<W> f;
#pragma unroll
        for (int i = 0; i < W; ++i) {
            f.v[i] = st[W][i];
#pragma unroll
            for (int j = 0; j < W; ++j)
                f.P[i][j] = st[j][i];
        }

        // 3. suffix scan (time runs down the lanes)
        const Affine<W> incl = wave_scan<W, true>(f, lane);
        Affine<W> excl = affine_shfl<W, true>(incl, 1);
        if (lane == 63)
            excl = affine_identity<W>();
        const Affine<W> tile = affine_bcast<W>(incl, 0);

        // 4. look-back over the later tiles; nothing enters the last one
        double zero[W];
#pragma unroll
        for (int i = 0; i < W; ++i)
            zero[i] = 0.0;
        double Stop[W];
        if (k + 1 == sd.ntile) {
#pragma unroll
            for (int i = 0; i < W; ++i)
                Stop[i] = 0.0;
        } else {
            publish_aggregate<W>(A, rec, tile, lane, 0);
            look_back<W, true>(A, sd.tile_base, k, sd.ntile, zero, lane, stage, Stop);
        }
        if (k > 0) {
            double So[W];
            affine_apply<W>(tile, Stop, So);
            publish_inclusive<W>(A, rec, So, lane);
        }

        // 5. adjoint apply from the lane's top state: gx = ybar, ga rows
        double sv[W];
        affine_apply<W>(excl, Stop, sv);
        const float *yl = ys + lane * G::YS;
        float *gw = gs + lane * G::XS;
#pragma unroll
        for (int s = L - 1; s >= 0; --s) {
            double c[W + 1];
            lds_row<W>(cl, s, c);
            const double yb = (double)gl[s] + sv[0];
#pragma unroll
            for (int i = 0; i < W; ++i)
                sv[i] = __builtin_fma(-c[i + 1], yb, i + 1 < W ? sv[i + 1] : 0.0);
            gw[s] = (float)yb;
            if (want_ga) {
#pragma unroll
                for (int kk = 1; kk <= W; ++kk)
                    cl[s * W + kk - 1] = (float)(-yb * (double)yl[W + s - kk]);
            }
        }
        if (k == 0 && lane == 0 && gyi != nullptr) {
#pragma unroll
            for (int i = 0; i < W; ++i)
                if (i < N)
                    gyi[sd.ic_off + i] = (float)sv[i];
        }
        __syncthreads();
        if (gx != nullptr)
            for (int e = lane; e < n; e += 64)
                gx[sd.x_off + t0 + e] = gs[(e / L) * G::XS + (e % L)];
        if (want_ga) {
            const int64_t a0 = sd.a_off + t0 * N;
            if (N == W && (a0 % 4) == 0) {
                const int nv = (n * W) / 4;
                for (int v = lane; v < nv; v += 64) {
                    const int e = 4 * v, r = e / W;
                    const float4 val = *reinterpret_cast<const float4 *>(
                        cs + (r / L) * G::CS + (r % L) * W + (e % W));
                    *reinterpret_cast<float4 *>(ga + a0 + e) = val;
                }
                for (int e = 4 * nv + lane; e < n * W; e += 64) {
                    const int r = e / W;
                    ga[a0 + e] = cs[(r / L) * G::CS + (r % L) * W + (e % W)];
                }
            } else {
                for (int e = lane; e < n * N; e += 64) {
                    const int r = e / N, tap = e % N;
                    ga[a0 + e] = cs[(r / L) * G::CS + (r % L) * W + tap];
                }
            }
        }
        __syncthreads();
    }
}

// Clears a bucket's flags and its lists' ticket counters (a kernel, not a
// memset, so captured graphs replay it faithfully).
__global__ void __launch_bounds__(256) kb_onepass_reset(int *flag, int64_t n, int *ticket)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        flag[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x < kOnePassLists)
        ticket[threadIdx.x * kTicketStride] = 0;
}

}  // namespace filt_detail
