// batched.hip -- plans for batched ragged filtering (see batched.h): device
// item tables, the workspace, the launch sequence of one forward / backward,
// hipGraph capture of forward + backward, and the chunk-length autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

#include "onepass16.h"

namespace filt_detail {

FILT_DECLARE_BATCHED(1, extern)
FILT_DECLARE_BATCHED(2, extern)
FILT_DECLARE_BATCHED(4, extern)
FILT_DECLARE_BATCHED(8, extern)
FILT_DECLARE_BATCHED(16, extern)

namespace {

constexpr int kBuckets = 5;  // W = 1, 2, 4, 8, 16
constexpr int kBucketW[kBuckets] = {1, 2, 4, 8, 16};
// Untuned plans: the single-pass kernel for orders up to 4 and the
// three-phase scan above (measured faster there); the tuner times both at
// several chunk lengths per bucket and keeps the faster
constexpr bool kDefaultOnePass[kBuckets] = {true, true, true, false, false};

int bucket_of(int N)
{
    int w = 1, i = 0;
    while (w < N) {
        w <<= 1;
        ++i;
    }
    return i;
}

// Carry kernels over the segment table: one workgroup per (segment, block)
// item, or per segment for the pass over blocks.
__global__ void __launch_bounds__(64)
kb_carry_agg(const SegDesc *__restrict__ segs, const Item *__restrict__ items, double *ws, int bwd)
{
    const Item it = items[blockIdx.x];
    const SegDesc sd = segs[it.seg];
    carry_agg_body(seg_dims(sd), seg_carry(sd, ws, bwd), 0, it.chunk);
}

__global__ void __launch_bounds__(256)
kb_carry_blocks(const SegDesc *__restrict__ segs, const Item *__restrict__ items, double *ws,
                int bwd, const float *__restrict__ yi)
{
    const Item it = items[blockIdx.x];
    const SegDesc sd = segs[it.seg];
    const float *init = (!bwd && yi != nullptr) ? yi + sd.ic_off : nullptr;
    const Dims d = seg_dims(sd);
    const CarryArgs a = seg_carry(sd, ws, bwd);
    extern __shared__ double carry_stage[];
#define CALL(DB) carry_blocks_body<DB>(d, a, init, 0, 0, carry_stage)
    FILT_CARRY_DB(a.D, CALL);
#undef CALL
}

__global__ void __launch_bounds__(256)
kb_carry_fill(const SegDesc *__restrict__ segs, const Item *__restrict__ items, double *ws, int bwd)
{
    const Item it = items[blockIdx.x];
    const SegDesc sd = segs[it.seg];
    const Dims d = seg_dims(sd);
    const CarryArgs a = seg_carry(sd, ws, bwd);
    extern __shared__ double carry_stage[];
#define CALL(DB) carry_fill_body<DB>(d, a, 0, it.chunk, carry_stage)
    FILT_CARRY_DB(a.D, CALL);
#undef CALL
}

template <typename T>
filt_status to_device(T *&dst, const std::vector<T> &src)
{
    if (dst != nullptr) {
        hipFree(dst);
        dst = nullptr;
    }
    if (src.empty())
        return FILT_OK;
    if (hipMalloc((void **)&dst, src.size() * sizeof(T)) != hipSuccess)
        return fail(FILT_EHIP, "hipMalloc of a plan table failed");
    if (hipMemcpy(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return fail(FILT_EHIP, "hipMemcpy of a plan table failed");
    return FILT_OK;
}

}  // namespace

}  // namespace filt_detail

using namespace filt_detail;

struct filt_plan {
    std::vector<filt_segment> segs;
    int64_t chunk[kBuckets];
    bool bucket_av[kBuckets];
    // device tables
    SegDesc *d_segs = nullptr;
    Item *d_items = nullptr;
    double *d_ws = nullptr;
    size_t ws_doubles = 0;
    int64_t sum_off[kBuckets], sum_n[kBuckets], app_off[kBuckets], app_n[kBuckets];
    // carry items per bucket: (segment, block) and (segment) lists
    int64_t cblk_off[kBuckets], cblk_n[kBuckets], cseg_off[kBuckets], cseg_n[kBuckets];
    // dynamic LDS (doubles) of a bucket's carry launches: its largest staged run
    int64_t blk_lds[kBuckets], fill_lds[kBuckets];
    int max_order[kBuckets];
    // the buckets touch disjoint segments, so each bucket's launch chain runs
    // on a stream of its own, forked from and joined back into the caller's
    // stream by events (also inside a captured graph)
    hipStream_t side[kBuckets] = {};
    hipEvent_t fork = nullptr, join[kBuckets] = {};
    // single-pass buckets (orders up to kOnePassMaxW): tile lists in ticket
    // order for each direction, per-tile records in d_ws, flags and ticket
    // counters in d_flags
    bool onepass[kBuckets] = {};
    int2 *d_tiles = nullptr;
    int *d_flags = nullptr;
    size_t flags_n = 0;
    int64_t tiles_fwd_off[kBuckets] = {}, tiles_bwd_off[kBuckets] = {}, ntiles[kBuckets] = {};
    int64_t agg_off[kBuckets] = {}, inc_off[kBuckets] = {}, flag_off[kBuckets] = {};
    int64_t ticket_off[kBuckets] = {};
    int nlists[kBuckets] = {};
    int64_t list_off[kBuckets][kOnePassLists + 1] = {};
    // frame-held segments per bucket: items (segment, first frame, frames)
    // of the per-frame gradient pass; and an adjoint buffer for backward
    // calls that want ga but no gx
    int64_t fr_off[kBuckets] = {}, fr_n[kBuckets] = {};
    float *d_ybar = nullptr;
    // captured forward + backward
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int64_t default_chunk(int W)
{
    // per-sample filters: the N x N transition stored per chunk must stay
    // small next to the coefficients read; short filters favour short chunks
    const int64_t L = std::max<int64_t>(128, 12 * (int64_t)W);
    return ((L + 31) / 32) * 32;
}

void drop_graph(filt_plan *p)
{
    if (p->exec != nullptr)
        hipGraphExecDestroy(p->exec);
    if (p->graph != nullptr)
        hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

// Lay out segments, item lists and workspace for the current chunk lengths.
filt_status plan_layout(filt_plan *p)
{
    drop_graph(p);
    const int nseg = (int)p->segs.size();
    std::vector<SegDesc> sd(nseg);
    size_t off = 0;
    for (int i = 0; i < nseg; ++i) {
        const filt_segment &s = p->segs[i];
        SegDesc &d = sd[i];
        const int bk = bucket_of(std::max(s.N, 1));
        d.x_off = s.x_off;
        d.T = s.T;
        d.a_off = s.a_off;
        d.ic_off = s.ic_off;
        d.N = s.N;
        d.hop = s.hop > 1 ? s.hop : 1;
        d.fd = frame_div(d.hop);
        d.L = p->chunk[bk];
        d.C = (s.T + d.L - 1) / d.L;
        const int64_t steps = std::max<int64_t>(d.C - 1, 1);
        int64_t G = 1;
        while (G * G < steps)
            ++G;
        d.G = G;
        d.NB = (steps + G - 1) / G;
        const int W = kBucketW[bk];
        const int vec = W >= 4 ? 4 : W;
        d.a_vec = (s.N == W) && (s.a_off % vec == 0);
        d.tile_base = d.ntile = 0;
        if (p->onepass[bk])
            continue;  // its records come with the tiles below
        const int64_t SS = (int64_t)s.N * s.N + s.N;
        d.summ_off = (int64_t)off;
        off += (size_t)(d.C * SS);
        d.states_off = (int64_t)off;
        off += (size_t)(d.C * s.N);
        d.agg_off = (int64_t)off;
        off += (size_t)(d.NB * SS);
        d.bstart_off = (int64_t)off;
        off += (size_t)(d.NB * std::max(s.N, 1));
        off = (off + 1) & ~size_t(1);  // keep every region 16-byte aligned
    }
    for (int b = 0; b < kBuckets; ++b)
        p->bucket_av[b] = true;
    // single-pass buckets: tiles per segment, records, ticket lists (whole
    // segments per list, balanced by tiles; in each list every tile after
    // the tiles it waits for, longest segments first in each rank so the
    // longest chains start early)
    std::vector<int2> tiles;
    size_t nflags = 0;
    {
        std::vector<int> order(nseg);
        for (int i = 0; i < nseg; ++i)
            order[i] = i;
        std::stable_sort(order.begin(), order.end(),
                         [&](int u, int v) { return p->segs[u].T > p->segs[v].T; });
        for (int b = 0; b < kBuckets; ++b) {
            if (!p->onepass[b])
                continue;
            // orders up to 4: one wavefront per tile of 64 lanes x 32 (orders 1, 2)
            // or 16 (order 4) samples, maps of
            // W x W; orders 5..16: one workgroup per tile of 16 x 32 samples,
            // maps of 16 x 16
            const int W = kBucketW[b] <= kOnePassMaxW ? kBucketW[b] : 16;
            const int64_t S = kBucketW[b] == 1   ? OnePass<1>::S
                              : kBucketW[b] == 2 ? OnePass<2>::S
                              : kBucketW[b] == 4 ? OnePass<4>::S
                                                 : OnePass16::S;
            int64_t nt = 0, maxt = 0;
            for (int i = 0; i < nseg; ++i) {
                if (bucket_of(std::max(p->segs[i].N, 1)) != b)
                    continue;
                sd[i].ntile = (p->segs[i].T + S - 1) / S;
                sd[i].tile_base = nt;
                nt += sd[i].ntile;
                maxt = std::max(maxt, sd[i].ntile);
            }
            p->ntiles[b] = nt;
            p->agg_off[b] = (int64_t)off;
            off += (size_t)(nt * (W * W + W));
            p->inc_off[b] = (int64_t)off;
            off += (size_t)(nt * W);
            off = (off + 1) & ~size_t(1);
            // flags, then the lists' ticket counters on lines of their own,
            // then the timeout counter
            p->flag_off[b] = (int64_t)nflags;
            const size_t toff = ((size_t)nflags + (size_t)nt + kTicketStride - 1) /
                                kTicketStride * kTicketStride;
            p->ticket_off[b] = (int64_t)toff;
            nflags = toff + (size_t)(kOnePassLists + 1) * kTicketStride;
            const int nl = kOnePassLists;
            p->nlists[b] = nl;
            std::vector<int> list_of(nseg, -1);
            std::vector<int64_t> load(nl, 0);
            for (int i : order) {  // longest first, each to the lightest list
                if (bucket_of(std::max(p->segs[i].N, 1)) != b)
                    continue;
                const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                list_of[i] = l;
                load[l] += sd[i].ntile;
            }
            p->list_off[b][0] = 0;
            for (int l = 0; l < nl; ++l)
                p->list_off[b][l + 1] = p->list_off[b][l] + load[l];
            for (int dir = 0; dir < 2; ++dir) {
                (dir == 0 ? p->tiles_fwd_off[b] : p->tiles_bwd_off[b]) = (int64_t)tiles.size();
                for (int l = 0; l < nl; ++l)
                    for (int64_t r = 0; r < maxt; ++r)
                        for (int i : order) {
                            if (list_of[i] != l || r >= sd[i].ntile)
                                continue;
                            const int64_t k = dir == 0 ? r : sd[i].ntile - 1 - r;
                            tiles.push_back(make_int2(i, (int)k));
                        }
            }
        }
    }
    std::vector<Item> items;
    for (int b = 0; b < kBuckets; ++b) {
        const int W = kBucketW[b];
        const int S = W == 1 ? 2 : 3;  // SummarySlots
        p->sum_off[b] = (int64_t)items.size();
        for (int i = 0; i < nseg; ++i) {
            if (p->onepass[b] || bucket_of(std::max(p->segs[i].N, 1)) != b)
                continue;
            // full-width rows only if every segment of the bucket has them
            // (an order-0 segment has none)
            p->bucket_av[b] = p->bucket_av[b] && sd[i].a_vec;
            if (p->segs[i].N == 0)
                continue;
            // order-16 bucket: one item per chunk (a DPP row and a quad);
            // else nl lanes of S solves each
            const int nl = W == 16 ? 1 : (sd[i].N + 1 + S - 1) / S;
            for (int64_t c = 0; c + 1 < sd[i].C; ++c)
                for (int r = 0; r < nl; ++r)
                    items.push_back(Item{i, (int32_t)c, r, 0});
        }
        p->sum_n[b] = (int64_t)items.size() - p->sum_off[b];
        p->app_off[b] = (int64_t)items.size();
        for (int i = 0; i < nseg; ++i) {
            if (p->onepass[b] || bucket_of(std::max(p->segs[i].N, 1)) != b)
                continue;
            for (int64_t c = 0; c < sd[i].C; ++c)
                items.push_back(Item{i, (int32_t)c, 0, 0});
        }
        p->app_n[b] = (int64_t)items.size() - p->app_off[b];
    }
    for (int b = 0; b < kBuckets; ++b) {
        auto in_bucket = [&](int i) {
            return !p->onepass[b] && sd[i].C > 1 && sd[i].N > 0 &&
                   bucket_of(std::max(p->segs[i].N, 1)) == b;
        };
        p->cblk_off[b] = (int64_t)items.size();
        p->blk_lds[b] = p->fill_lds[b] = 0;
        p->max_order[b] = 0;
        for (int i = 0; i < nseg; ++i)
            if (in_bucket(i)) {
                const int n = sd[i].N;
                const CarryRec cr = carry_rec(n, (int64_t)n * n + n);
                p->blk_lds[b] = std::max<int64_t>(
                    p->blk_lds[b], (int64_t)stage_steps(cr.blk_len, sd[i].NB) * cr.blk_len);
                p->fill_lds[b] = std::max<int64_t>(
                    p->fill_lds[b], (int64_t)stage_steps(cr.fill_len, sd[i].G) * cr.fill_len);
                p->max_order[b] = std::max(p->max_order[b], n);
                for (int64_t k = 0; k < sd[i].NB; ++k)
                    items.push_back(Item{i, (int32_t)k, 0, 0});
            }
        p->cblk_n[b] = (int64_t)items.size() - p->cblk_off[b];
        p->cseg_off[b] = (int64_t)items.size();
        for (int i = 0; i < nseg; ++i)
            if (in_bucket(i))
                items.push_back(Item{i, 0, 0, 0});
        p->cseg_n[b] = (int64_t)items.size() - p->cseg_off[b];
    }

    // per-frame gradient items of each bucket's frame-held segments
    for (int b = 0; b < kBuckets; ++b) {
        p->fr_off[b] = (int64_t)items.size();
        for (int i = 0; i < nseg; ++i) {
            if (bucket_of(std::max(p->segs[i].N, 1)) != b || sd[i].fd.m == 0 || sd[i].N == 0)
                continue;
            const int64_t F = (sd[i].T + sd[i].hop - 1) / sd[i].hop;
            for (int64_t f0 = 0; f0 < F; f0 += 64)
                items.push_back(Item{i, (int32_t)f0, (int32_t)std::min<int64_t>(64, F - f0), 0});
        }
        p->fr_n[b] = (int64_t)items.size() - p->fr_off[b];
    }

    filt_status s = to_device(p->d_segs, sd);
    if (s != FILT_OK)
        return s;
    s = to_device(p->d_items, items);
    if (s != FILT_OK)
        return s;
    s = to_device(p->d_tiles, tiles);
    if (s != FILT_OK)
        return s;
    if (nflags > p->flags_n) {
        if (p->d_flags != nullptr)
            hipFree(p->d_flags);
        p->d_flags = nullptr;
        if (hipMalloc((void **)&p->d_flags, nflags * sizeof(int)) != hipSuccess)
            return fail(FILT_EHIP, "hipMalloc of the plan's tile flags failed");
        if (hipMemset(p->d_flags, 0, nflags * sizeof(int)) != hipSuccess)
            return fail(FILT_EHIP, "hipMemset of the plan's tile flags failed");
        p->flags_n = nflags;
    }
    if (off > p->ws_doubles) {
        if (p->d_ws != nullptr)
            hipFree(p->d_ws);
        p->d_ws = nullptr;
        if (hipMalloc((void **)&p->d_ws, std::max<size_t>(off, 1) * sizeof(double)) != hipSuccess)
            return fail(FILT_EHIP, "hipMalloc of the plan workspace (%zu bytes) failed",
                        off * sizeof(double));
        p->ws_doubles = off;
    }
    return FILT_OK;
}

BucketArgs bucket_args(const filt_plan *p, int b, const float *a)
{
    BucketArgs ba{};
    ba.segs = p->d_segs;
    ba.sum_items = p->d_items + p->sum_off[b];
    ba.sum_n = p->sum_n[b];
    ba.app_items = p->d_items + p->app_off[b];
    ba.app_n = p->app_n[b];
    ba.av = p->bucket_av[b] && ((uintptr_t)a % 16 == 0);
    return ba;
}

filt_status carry_launch(const filt_plan *p, int b, int bwd, const float *yi, hipStream_t st)
{
    if (p->cseg_n[b] == 0)
        return FILT_OK;
    const Item *blk = p->d_items + p->cblk_off[b];
    const Item *seg = p->d_items + p->cseg_off[b];
    const int n = p->max_order[b];
    FILT_LAUNCH("batched_carry_agg", kb_carry_agg, dim3((unsigned)p->cblk_n[b]), dim3(64), 0, st,
                p->d_segs, blk, p->d_ws, bwd);
    FILT_LAUNCH("batched_carry_blocks", kb_carry_blocks, dim3((unsigned)p->cseg_n[b]),
                dim3(carry_threads(p->blk_lds[b], n)), p->blk_lds[b] * sizeof(double), st,
                p->d_segs, seg, p->d_ws, bwd, yi);
    FILT_LAUNCH("batched_carry_fill", kb_carry_fill, dim3((unsigned)p->cblk_n[b]),
                dim3(carry_threads(p->fill_lds[b], n)), p->fill_lds[b] * sizeof(double), st,
                p->d_segs, blk, p->d_ws, bwd);
    return check_launch("batched carry");
}

OnePassArgs onepass_args(const filt_plan *p, int b, bool bwd)
{
    OnePassArgs A{};
    A.segs = p->d_segs;
    A.tiles = p->d_tiles + (bwd ? p->tiles_bwd_off[b] : p->tiles_fwd_off[b]);
    A.ntiles = p->ntiles[b];
    A.agg = p->d_ws + p->agg_off[b];
    A.inc = p->d_ws + p->inc_off[b];
    A.flag = p->d_flags + p->flag_off[b];
    A.ticket = p->d_flags + p->ticket_off[b];
    A.timeouts = A.ticket + kOnePassLists * kTicketStride;
    A.nlists = std::max(p->nlists[b], 1);
    for (int l = 0; l <= kOnePassLists; ++l)
        A.list_off[l] = p->list_off[b][std::min(l, A.nlists)];
    return A;
}

// Workgroups of a single-pass launch: enough for every CU to hold several
// (the LDS of a tile bounds how many are resident), and at least one per
// ticket list; the rest find their list's counter past its end and leave.
unsigned onepass_grid(int64_t ntiles, int nlists)
{
    return (unsigned)std::max<int64_t>(nlists, std::min<int64_t>(ntiles, kCUs * 16));
}

unsigned onepass_grid16(int64_t ntiles, int nlists)
{
    return (unsigned)std::max<int64_t>(nlists, std::min<int64_t>(ntiles, kCUs * 2));
}

template <int W>
filt_status onepass_forward(const filt_plan *p, int b, const float *x, const float *a,
                            const float *yi, float *y, hipStream_t st)
{
    const OnePassArgs A = onepass_args(p, b, false);
    FILT_LAUNCH("batched_onepass_reset", kb_onepass_reset, dim3(64), dim3(256), 0, st, A.flag,
                A.ntiles, A.ticket);
    if constexpr (W <= kOnePassMaxW)
        FILT_LAUNCH(FILT_BNAME("batched_onepass_fwd", W), kb_onepass_fwd<W>,
                    dim3(onepass_grid(A.ntiles, A.nlists)), dim3(64), 0, st, A, x, a, yi, y);
    else
        FILT_LAUNCH(FILT_BNAME("batched_onepass_fwd", W), kb_onepass16_fwd,
                    dim3(onepass_grid16(A.ntiles, A.nlists)), dim3(OnePass16::kThreads), 0, st, A, x, a, yi,
                    y);
    return check_launch("batched single-pass forward");
}

template <int W>
filt_status onepass_backward(const filt_plan *p, int b, const float *gy, const float *y,
                             const float *a, const float *yi, float *gx, float *ga, float *gyi,
                             hipStream_t st)
{
    const OnePassArgs A = onepass_args(p, b, true);
    FILT_LAUNCH("batched_onepass_reset", kb_onepass_reset, dim3(64), dim3(256), 0, st, A.flag,
                A.ntiles, A.ticket);
    if constexpr (W <= kOnePassMaxW)
        FILT_LAUNCH(FILT_BNAME("batched_onepass_bwd", W), kb_onepass_bwd<W>,
                    dim3(onepass_grid(A.ntiles, A.nlists)), dim3(64), 0, st, A, gy, a, y, yi, gx, ga, gyi);
    else
        FILT_LAUNCH(FILT_BNAME("batched_onepass_bwd", W), kb_onepass16_bwd,
                    dim3(onepass_grid16(A.ntiles, A.nlists)), dim3(OnePass16::kThreads), 0, st, A, gy, a, y,
                    yi, gx, ga, gyi);
    return check_launch("batched single-pass backward");
}

// One bucket's forward: summaries, carry, apply.
template <int W, int B>
filt_status bucket_forward(const filt_plan *p, const float *x, const float *a, const float *yi,
                           float *y, hipStream_t st)
{
    if (p->onepass[B])
        return onepass_forward<W>(p, B, x, a, yi, y, st);
    filt_status s = batched_fwd_summary<W>(bucket_args(p, B, a), x, a, p->d_ws, st);
    if (s == FILT_OK)
        s = carry_launch(p, B, 0, yi, st);
    if (s != FILT_OK)
        return s;
    if constexpr (kStreamBucket<W>)
        return batched_stream_fwd<W>(bucket_args(p, B, a), p->chunk[B], x, a, yi, p->d_ws, y, st);
    return batched_fwd_apply<W>(bucket_args(p, B, a), x, a, yi, p->d_ws, y, st);
}

// One bucket's backward: summaries, carry, adjoint apply (+ coefficient
// gradients).
// ga of the bucket's frame-held segments from the adjoint ybar.
filt_status frame_grads_launch(const filt_plan *p, int b, const float *ybar, const float *y,
                               const float *yi, float *ga, hipStream_t st)
{
    if (ga == nullptr || p->fr_n[b] == 0)
        return FILT_OK;
    FILT_LAUNCH(FILT_BNAME("batched_frame_grads", kBucketW[b]), kb_frame_grads,
                dim3((unsigned)p->fr_n[b]), dim3(64), 0, st, p->d_segs,
                p->d_items + p->fr_off[b], ybar, y, yi, ga);
    return check_launch("batched frame gradients");
}

template <int W, int B>
filt_status bucket_backward(const filt_plan *p, const float *gy, const float *y, const float *a,
                            const float *yi, float *gx, float *ga, float *gyi, hipStream_t st)
{
    // frame-held rows take their gradients from the stored adjoint (gx is
    // ybar for b = [1]); without gx it goes to the plan's own buffer
    if (gx == nullptr && ga != nullptr && p->fr_n[B] > 0)
        gx = p->d_ybar;
    filt_status s = FILT_OK;
    if (p->onepass[B]) {
        s = onepass_backward<W>(p, B, gy, y, a, yi, gx, ga, gyi, st);
        if (s != FILT_OK)
            return s;
        return frame_grads_launch(p, B, gx, y, yi, ga, st);
    }
    s = batched_bwd_summary<W>(bucket_args(p, B, a), gy, a, p->d_ws, st);
    if (s == FILT_OK)
        s = carry_launch(p, B, 1, nullptr, st);
    if (s != FILT_OK)
        return s;
    if (gx == nullptr)
        return batched_bwd_apply<W>(bucket_args(p, B, a), gy, y, a, yi, p->d_ws, gx, ga, gyi, st);
    if constexpr (kStreamBucket<W>)
        s = batched_stream_bwd<W>(bucket_args(p, B, a), p->chunk[B], gy, y, a, yi, p->d_ws, gx,
                                  ga, gyi, st);
    else
        s = batched_bwd_split<W>(bucket_args(p, B, a), p->chunk[B], gy, y, a, yi, p->d_ws, gx,
                                 ga, gyi, st);
    if (s != FILT_OK)
        return s;
    return frame_grads_launch(p, B, gx, y, yi, ga, st);
}

// Does the plan have work in bucket b?
bool bucket_busy(const filt_plan *p, int b)
{
    return p->sum_n[b] > 0 || p->app_n[b] > 0 || (p->onepass[b] && p->ntiles[b] > 0);
}


// The stream each bucket's launches go to: the two smallest buckets share
// one, so the step uses four concurrent streams (the hardware queues a
// process gets by default).
constexpr int kStreamOf[kBuckets] = {1, 1, 2, 3, 4};

// Runs fn(b, stream) for every busy bucket in mask, each on its own stream
// forked from st, the longest-running (highest order) first; st waits for
// all of them.  With one busy bucket it runs on st directly.
template <typename F>
filt_status fork_buckets(const filt_plan *p, hipStream_t st, unsigned mask, F &&fn)
{
    int busy = 0;
    for (int b = 0; b < kBuckets; ++b)
        busy += ((mask >> b) & 1u) && bucket_busy(p, b);
    if (busy <= 1 || p->fork == nullptr) {
        filt_status s = FILT_OK;
        for (int b = kBuckets - 1; b >= 0 && s == FILT_OK; --b)
            if (((mask >> b) & 1u) && bucket_busy(p, b))
                s = fn(b, st);
        return s;
    }
    if (hipEventRecord(p->fork, st) != hipSuccess)
        return fail(FILT_EHIP, "hipEventRecord (fork) failed");
    filt_status s = FILT_OK;
    for (int b = kBuckets - 1; b >= 0; --b) {
        if (!(((mask >> b) & 1u) && bucket_busy(p, b)))
            continue;
        hipStream_t side = p->side[kStreamOf[b]];
        if (hipStreamWaitEvent(side, p->fork, 0) != hipSuccess)
            return fail(FILT_EHIP, "hipStreamWaitEvent (fork) failed");
        if (s == FILT_OK)
            s = fn(b, side);
        // join even after a failed launch so a capture stays well formed
        if (hipEventRecord(p->join[b], side) != hipSuccess ||
            hipStreamWaitEvent(st, p->join[b], 0) != hipSuccess)
            return fail(FILT_EHIP, "event join of a bucket stream failed");
    }
    return s;
}

// The launch sequence of one direction, restricted to the buckets in mask.
filt_status run_forward(const filt_plan *p, const float *x, const float *a, const float *yi,
                        float *y, hipStream_t st, unsigned mask = 0x1f)
{
    return fork_buckets(p, st, mask, [&](int b, hipStream_t s) -> filt_status {
        switch (b) {
        case 0: return bucket_forward<1, 0>(p, x, a, yi, y, s);
        case 1: return bucket_forward<2, 1>(p, x, a, yi, y, s);
        case 2: return bucket_forward<4, 2>(p, x, a, yi, y, s);
        case 3: return bucket_forward<8, 3>(p, x, a, yi, y, s);
        default: return bucket_forward<16, 4>(p, x, a, yi, y, s);
        }
    });
}

filt_status run_backward(const filt_plan *p, const float *gy, const float *y, const float *a,
                         const float *yi, float *gx, float *ga, float *gyi, hipStream_t st,
                         unsigned mask = 0x1f)
{
    return fork_buckets(p, st, mask, [&](int b, hipStream_t s) -> filt_status {
        switch (b) {
        case 0: return bucket_backward<1, 0>(p, gy, y, a, yi, gx, ga, gyi, s);
        case 1: return bucket_backward<2, 1>(p, gy, y, a, yi, gx, ga, gyi, s);
        case 2: return bucket_backward<4, 2>(p, gy, y, a, yi, gx, ga, gyi, s);
        case 3: return bucket_backward<8, 3>(p, gy, y, a, yi, gx, ga, gyi, s);
        default: return bucket_backward<16, 4>(p, gy, y, a, yi, gx, ga, gyi, s);
        }
    });
}

// Forward then backward of every bucket on the bucket's own stream, with one
// fork and one join: a bucket's adjoint needs only its own forward, so the
// low-order buckets' backward runs while the order-16 forward still does
// (the captured fwd + bwd step).
filt_status run_step(const filt_plan *p, const float *x, const float *a, const float *yi,
                     const float *gy, float *y, float *gx, float *ga, float *gyi, hipStream_t st)
{
    return fork_buckets(p, st, 0x1f, [&](int b, hipStream_t s) -> filt_status {
        switch (b) {
        case 0: {
            const filt_status r = bucket_forward<1, 0>(p, x, a, yi, y, s);
            return r != FILT_OK ? r : bucket_backward<1, 0>(p, gy, y, a, yi, gx, ga, gyi, s);
        }
        case 1: {
            const filt_status r = bucket_forward<2, 1>(p, x, a, yi, y, s);
            return r != FILT_OK ? r : bucket_backward<2, 1>(p, gy, y, a, yi, gx, ga, gyi, s);
        }
        case 2: {
            const filt_status r = bucket_forward<4, 2>(p, x, a, yi, y, s);
            return r != FILT_OK ? r : bucket_backward<4, 2>(p, gy, y, a, yi, gx, ga, gyi, s);
        }
        case 3: {
            const filt_status r = bucket_forward<8, 3>(p, x, a, yi, y, s);
            return r != FILT_OK ? r : bucket_backward<8, 3>(p, gy, y, a, yi, gx, ga, gyi, s);
        }
        default: {
            const filt_status r = bucket_forward<16, 4>(p, x, a, yi, y, s);
            return r != FILT_OK ? r : bucket_backward<16, 4>(p, gy, y, a, yi, gx, ga, gyi, s);
        }
        }
    });
}

filt_status check_plan(const filt_plan *p)
{
    if (p == nullptr)
        return fail(FILT_EINVAL, "plan is NULL");
    return FILT_OK;
}

}  // namespace

extern "C" {

filt_status filt_plan_create(const filt_segment *segs, int32_t nseg, const int32_t *chunks,
                             filt_plan **out)
{
    if (out == nullptr)
        return fail(FILT_EINVAL, "out is NULL");
    *out = nullptr;
    if (nseg < 0 || (nseg > 0 && segs == nullptr))
        return fail(FILT_EINVAL, "bad segment list");
    for (int i = 0; i < nseg; ++i) {
        const filt_segment &s = segs[i];
        if (s.T < 0 || s.x_off < 0 || s.a_off < 0 || s.ic_off < 0)
            return fail(FILT_EINVAL, "segment %d: negative size or offset", i);
        if (s.N < 0 || s.N > 16)
            return fail(s.N < 0 ? FILT_EINVAL : FILT_EUNSUPPORTED, "segment %d: order %d", i, s.N);
        if (s.hop < 0)
            return fail(FILT_EINVAL, "segment %d: hop %d (0 or 1: per-sample rows, h >= 2: "
                        "frame-held rows)", i, (int)s.hop);
        if (s.T > ((int64_t)1 << 31) - 64)
            return fail(FILT_EUNSUPPORTED, "segment %d: T too large for a plan", i);
    }
    filt_plan *p = new filt_plan();
    p->segs.assign(segs, segs + nseg);
    for (int b = 0; b < kBuckets; ++b) {
        const int32_t c = chunks != nullptr ? chunks[b] : 0;
        if (c < -1 || (c > 0 && c % 32 != 0)) {
            delete p;
            return fail(FILT_EINVAL,
                        "chunk %d for bucket %d: -1 (single pass), 0 (default) or a positive "
                        "multiple of 32",
                        (int)c, b);
        }
        p->chunk[b] = c > 0 ? c : default_chunk(kBucketW[b]);
        p->onepass[b] = c < 0 || (c == 0 && kDefaultOnePass[b]);
    }
    bool ev_ok = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) == hipSuccess;
    for (int b = 0; b < kBuckets && ev_ok; ++b)
        ev_ok = hipStreamCreateWithFlags(&p->side[b], hipStreamNonBlocking) == hipSuccess &&
                hipEventCreateWithFlags(&p->join[b], hipEventDisableTiming) == hipSuccess;
    if (!ev_ok) {
        filt_plan_destroy(p);
        return fail(FILT_EHIP, "creating the plan's bucket streams failed");
    }
    filt_status s = plan_layout(p);
    // backward calls that want ga without gx stage the adjoint of the
    // frame-held segments here
    bool frames = false;
    int64_t nybar = 0;
    for (int i = 0; i < nseg; ++i) {
        frames = frames || segs[i].hop > 1;
        nybar = std::max<int64_t>(nybar, segs[i].x_off + segs[i].T);
    }
    if (!frames)
        nybar = 0;
    if (s == FILT_OK && nybar > 0 &&
        hipMalloc((void **)&p->d_ybar, (size_t)nybar * sizeof(float)) != hipSuccess)
        s = fail(FILT_EHIP, "hipMalloc of the plan's adjoint buffer failed");
    if (s != FILT_OK) {
        filt_plan_destroy(p);
        return s;
    }
    *out = p;
    return FILT_OK;
}

void filt_plan_destroy(filt_plan *p)
{
    if (p == nullptr)
        return;
    drop_graph(p);
    for (int b = 0; b < kBuckets; ++b) {
        if (p->side[b] != nullptr)
            hipStreamDestroy(p->side[b]);
        if (p->join[b] != nullptr)
            hipEventDestroy(p->join[b]);
    }
    if (p->fork != nullptr)
        hipEventDestroy(p->fork);
    if (p->d_tiles != nullptr)
        hipFree(p->d_tiles);
    if (p->d_ybar != nullptr)
        hipFree(p->d_ybar);
    if (p->d_flags != nullptr)
        hipFree(p->d_flags);
    if (p->d_segs != nullptr)
        hipFree(p->d_segs);
    if (p->d_items != nullptr)
        hipFree(p->d_items);
    if (p->d_ws != nullptr)
        hipFree(p->d_ws);
    delete p;
}

filt_status filt_plan_get_chunks(const filt_plan *p, int32_t *chunks)
{
    filt_status s = check_plan(p);
    if (s != FILT_OK)
        return s;
    if (chunks == nullptr)
        return fail(FILT_EINVAL, "chunks is NULL");
    for (int b = 0; b < kBuckets; ++b)
        chunks[b] = p->onepass[b] ? -1 : (int32_t)p->chunk[b];
    return FILT_OK;
}

filt_status filt_plan_forward(filt_plan *p, const float *x, const float *a, const float *yi,
                              float *y, void *stream)
{
    filt_status s = check_plan(p);
    if (s != FILT_OK)
        return s;
    if (x == nullptr || y == nullptr || a == nullptr)
        return fail(FILT_EINVAL, "x, a and y are required");
    return run_forward(p, x, a, yi, y, (hipStream_t)stream);
}

filt_status filt_plan_backward(filt_plan *p, const float *gy, const float *y, const float *a,
                               const float *yi, float *gx, float *ga, float *gyi, void *stream)
{
    filt_status s = check_plan(p);
    if (s != FILT_OK)
        return s;
    if (gy == nullptr || a == nullptr)
        return fail(FILT_EINVAL, "gy and a are required");
    if (ga != nullptr && y == nullptr)
        return fail(FILT_EINVAL, "ga requested but y is NULL");
    return run_backward(p, gy, y, a, yi, gx, ga, gyi, (hipStream_t)stream);
}

filt_status filt_plan_tune(filt_plan *p, const float *x, const float *a, const float *yi,
                           const float *gy, float *y, float *gx, float *ga, float *gyi,
                           void *stream)
{
    filt_status s = check_plan(p);
    if (s != FILT_OK)
        return s;
    if (x == nullptr || a == nullptr || gy == nullptr || y == nullptr)
        return fail(FILT_EINVAL, "x, a, gy and y are required to tune");
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(FILT_EHIP, "hipEventCreate failed");
    static const int64_t cands[] = {64, 128, 192, 256, 384, 512, 1024, 2048};
    for (int b = 0; b < kBuckets; ++b) {
        bool any = false;
        for (const filt_segment &sg : p->segs)
            any = any || (bucket_of(std::max(sg.N, 1)) == b);
        if (!any)
            continue;
        const int W = kBucketW[b];
        int64_t best = p->chunk[b];
        bool best_one = p->onepass[b];
        float best_ms = 1e30f;
        // candidate 0: the single-pass kernel (its tiles have a fixed
        // length); then the three-phase scan at each chunk length
        for (int ci = -1; ci < (int)(sizeof cands / sizeof cands[0]); ++ci) {
            const int64_t L = ci < 0 ? p->chunk[b] : cands[ci];
            if (ci >= 0 && L < 4 * W)
                continue;
            p->onepass[b] = ci < 0;
            p->chunk[b] = L;
            s = plan_layout(p);
            if (s != FILT_OK)
                break;
            float med[3];
            for (int rep = 0; rep < 3 && s == FILT_OK; ++rep) {
                hipEventRecord(e0, st);
                s = run_forward(p, x, a, yi, y, st, 1u << b);
                if (s == FILT_OK)
                    s = run_backward(p, gy, y, a, yi, gx, ga, gyi, st, 1u << b);
                hipEventRecord(e1, st);
                hipEventSynchronize(e1);
                hipEventElapsedTime(&med[rep], e0, e1);
            }
            if (s != FILT_OK)
                break;
            std::sort(med, med + 3);
            if (med[1] < best_ms) {
                best_ms = med[1];
                best = L;
                best_one = ci < 0;
            }
        }
        p->chunk[b] = best;
        p->onepass[b] = best_one;
        if (s != FILT_OK)
            break;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (s != FILT_OK)
        return s;
    return plan_layout(p);
}

filt_status filt_plan_capture(filt_plan *p, const float *x, const float *a, const float *yi,
                              const float *gy, float *y, float *gx, float *ga, float *gyi,
                              void *stream)
{
    filt_status s = check_plan(p);
    if (s != FILT_OK)
        return s;
    if (x == nullptr || a == nullptr || gy == nullptr || y == nullptr)
        return fail(FILT_EINVAL, "x, a, gy and y are required");
    drop_graph(p);
    hipStream_t st = (hipStream_t)stream;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(FILT_EHIP, "hipStreamBeginCapture failed");
    s = run_step(p, x, a, yi, gy, y, gx, ga, gyi, st);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (s != FILT_OK) {
        if (g != nullptr)
            hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess || g == nullptr)
        return fail(FILT_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    p->graph = g;
    if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        drop_graph(p);
        return fail(FILT_EHIP, "hipGraphInstantiate failed");
    }
    return FILT_OK;
}

filt_status filt_plan_replay(filt_plan *p, void *stream)
{
    filt_status s = check_plan(p);
    if (s != FILT_OK)
        return s;
    if (p->exec == nullptr)
        return fail(FILT_EINVAL, "no captured graph: call filt_plan_capture first");
    if (hipGraphLaunch(p->exec, (hipStream_t)stream) != hipSuccess)
        return fail(FILT_EHIP, "hipGraphLaunch failed");
    return FILT_OK;
}

}  // extern "C"
