// batched.hip -- plans for batched ragged filtering (see batched.h): device
// item tables, the workspace, the launch sequence of one forward / backward,
// hipGraph capture of forward + backward, and the chunk-length autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

#include "batched.h"

namespace filt_detail {

FILT_DECLARE_BATCHED(1, extern)
FILT_DECLARE_BATCHED(2, extern)
FILT_DECLARE_BATCHED(4, extern)
FILT_DECLARE_BATCHED(8, extern)
FILT_DECLARE_BATCHED(16, extern)

namespace {

constexpr int kBuckets = 5;  // W = 1, 2, 4, 8, 16
constexpr int kBucketW[kBuckets] = {1, 2, 4, 8, 16};

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
    int64_t cblk_off = 0, cblk_n = 0, cseg_off = 0, cseg_n = 0;
    // dynamic LDS (doubles) of the carry launches: the largest staged run
    int64_t blk_lds = 0, fill_lds = 0;
    int max_order = 0;
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
    std::vector<Item> items;
    for (int b = 0; b < kBuckets; ++b) {
        const int W = kBucketW[b];
        const int S = W == 1 ? 2 : 3;  // SummarySlots
        p->sum_off[b] = (int64_t)items.size();
        for (int i = 0; i < nseg; ++i) {
            if (bucket_of(std::max(p->segs[i].N, 1)) != b)
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
            if (bucket_of(std::max(p->segs[i].N, 1)) != b)
                continue;
            for (int64_t c = 0; c < sd[i].C; ++c)
                items.push_back(Item{i, (int32_t)c, 0, 0});
        }
        p->app_n[b] = (int64_t)items.size() - p->app_off[b];
    }
    p->cblk_off = (int64_t)items.size();
    p->blk_lds = p->fill_lds = 0;
    p->max_order = 0;
    for (int i = 0; i < nseg; ++i)
        if (sd[i].C > 1 && sd[i].N > 0) {
            const int n = sd[i].N;
            const CarryRec cr = carry_rec(n, (int64_t)n * n + n);
            p->blk_lds = std::max<int64_t>(p->blk_lds, (int64_t)stage_steps(cr.blk_len, sd[i].NB) * cr.blk_len);
            p->fill_lds = std::max<int64_t>(p->fill_lds, (int64_t)stage_steps(cr.fill_len, sd[i].G) * cr.fill_len);
            p->max_order = std::max(p->max_order, n);
            for (int64_t k = 0; k < sd[i].NB; ++k)
                items.push_back(Item{i, (int32_t)k, 0, 0});
        }
    p->cblk_n = (int64_t)items.size() - p->cblk_off;
    p->cseg_off = (int64_t)items.size();
    for (int i = 0; i < nseg; ++i)
        if (sd[i].C > 1 && sd[i].N > 0)
            items.push_back(Item{i, 0, 0, 0});
    p->cseg_n = (int64_t)items.size() - p->cseg_off;

    filt_status s = to_device(p->d_segs, sd);
    if (s != FILT_OK)
        return s;
    s = to_device(p->d_items, items);
    if (s != FILT_OK)
        return s;
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

filt_status carry_launch(const filt_plan *p, int bwd, const float *yi, hipStream_t st)
{
    if (p->cseg_n == 0)
        return FILT_OK;
    const Item *blk = p->d_items + p->cblk_off;
    const Item *seg = p->d_items + p->cseg_off;
    const int n = p->max_order;
    FILT_LAUNCH("batched_carry_agg", kb_carry_agg, dim3((unsigned)p->cblk_n), dim3(64), 0, st,
                p->d_segs, blk, p->d_ws, bwd);
    FILT_LAUNCH("batched_carry_blocks", kb_carry_blocks, dim3((unsigned)p->cseg_n),
                dim3(carry_threads(p->blk_lds, n)), p->blk_lds * sizeof(double), st, p->d_segs,
                seg, p->d_ws, bwd, yi);
    FILT_LAUNCH("batched_carry_fill", kb_carry_fill, dim3((unsigned)p->cblk_n),
                dim3(carry_threads(p->fill_lds, n)), p->fill_lds * sizeof(double), st, p->d_segs,
                blk, p->d_ws, bwd);
    return check_launch("batched carry");
}

// The launch sequence of one direction, restricted to the buckets in mask.
filt_status run_forward(const filt_plan *p, const float *x, const float *a, const float *yi,
                        float *y, hipStream_t st, unsigned mask = 0x1f)
{
    filt_status s = FILT_OK;
#define FILT_BUCKETS(CALL)                                                                         \
    if ((mask & 1u) && s == FILT_OK) s = CALL(1, 0);                                               \
    if ((mask & 2u) && s == FILT_OK) s = CALL(2, 1);                                               \
    if ((mask & 4u) && s == FILT_OK) s = CALL(4, 2);                                               \
    if ((mask & 8u) && s == FILT_OK) s = CALL(8, 3);                                               \
    if ((mask & 16u) && s == FILT_OK) s = CALL(16, 4);
#define FWD_SUM(W, B) batched_fwd_summary<W>(bucket_args(p, B, a), x, a, p->d_ws, st)
#define FWD_APP(W, B)                                                                              \
    (kStreamBucket<W> ? batched_stream_fwd<W>(bucket_args(p, B, a), p->chunk[B], x, a, yi, p->d_ws, \
                                              y, st)                                               \
                      : batched_fwd_apply<W>(bucket_args(p, B, a), x, a, yi, p->d_ws, y, st))
    FILT_BUCKETS(FWD_SUM)
    if (s == FILT_OK)
        s = carry_launch(p, 0, yi, st);
    FILT_BUCKETS(FWD_APP)
#undef FWD_SUM
#undef FWD_APP
    return s;
}

filt_status run_backward(const filt_plan *p, const float *gy, const float *y, const float *a,
                         const float *yi, float *gx, float *ga, float *gyi, hipStream_t st,
                         unsigned mask = 0x1f)
{
    filt_status s = FILT_OK;
#define BWD_SUM(W, B) batched_bwd_summary<W>(bucket_args(p, B, a), gy, a, p->d_ws, st)
#define BWD_APP(W, B)                                                                              \
    (gx == nullptr                                                                                 \
         ? batched_bwd_apply<W>(bucket_args(p, B, a), gy, y, a, yi, p->d_ws, gx, ga, gyi, st)       \
     : kStreamBucket<W>                                                                            \
         ? batched_stream_bwd<W>(bucket_args(p, B, a), p->chunk[B], gy, y, a, yi, p->d_ws, gx, ga,  \
                                 gyi, st)                                                          \
         : batched_bwd_split<W>(bucket_args(p, B, a), p->chunk[B], gy, y, a, yi, p->d_ws, gx, ga,   \
                                gyi, st))
    FILT_BUCKETS(BWD_SUM)
    if (s == FILT_OK)
        s = carry_launch(p, 1, nullptr, st);
    FILT_BUCKETS(BWD_APP)
#undef BWD_SUM
#undef BWD_APP
#undef FILT_BUCKETS
    return s;
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
        if (s.T > ((int64_t)1 << 31) - 64)
            return fail(FILT_EUNSUPPORTED, "segment %d: T too large for a plan", i);
    }
    filt_plan *p = new filt_plan();
    p->segs.assign(segs, segs + nseg);
    for (int b = 0; b < kBuckets; ++b) {
        int64_t L = chunks != nullptr && chunks[b] > 0 ? chunks[b] : default_chunk(kBucketW[b]);
        if (L % 32 != 0) {
            delete p;
            return fail(FILT_EINVAL, "chunk %lld for bucket %d is not a multiple of 32",
                        (long long)L, b);
        }
        p->chunk[b] = L;
    }
    const filt_status s = plan_layout(p);
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
        chunks[b] = (int32_t)p->chunk[b];
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
        float best_ms = 1e30f;
        for (int64_t L : cands) {
            if (L < 4 * W)
                continue;
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
            }
        }
        p->chunk[b] = best;
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
    s = run_forward(p, x, a, yi, y, st);
    if (s == FILT_OK)
        s = run_backward(p, gy, y, a, yi, gx, ga, gyi, st);
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
