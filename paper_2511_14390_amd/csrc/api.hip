// api.hip -- C ABI entry points of libfilt.so: argument validation,
// workspace plan and dispatch to the per-bucket kernels.
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "common.h"

namespace filt_detail {

thread_local char g_err[512] = "";

filt_status fail(filt_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

// ------------------------------------------------------------ profiling
//
// While enabled, every launch is bracketed by two events from a pool created
// by filt_profile_enable (host side).  When the pool is exhausted further
// launches are not recorded.
struct ProfRec {
    const char *name;
    int ev;
};
constexpr int kProfEvents = 1 << 14;
bool g_prof_on = false;
hipEvent_t g_prof_ev[kProfEvents];
int g_prof_nev = 0;        // events created
int g_prof_used = 0;       // events handed out
ProfRec g_prof_rec[kProfEvents / 2];
int g_prof_nrec = 0;
char g_prof_only[64] = "";  // record only launches of this name (empty: all)

int prof_begin(const char *name, hipStream_t st)
{
    if (!g_prof_on || g_prof_used + 2 > g_prof_nev)
        return -1;
    if (g_prof_only[0] != 0 && strncmp(name, g_prof_only, sizeof g_prof_only) != 0)
        return -1;
    const int r = g_prof_nrec++;
    g_prof_rec[r].name = name;
    g_prof_rec[r].ev = g_prof_used;
    g_prof_used += 2;
    hipEventRecord(g_prof_ev[g_prof_rec[r].ev], st);
    return r;
}

void prof_end(int slot, hipStream_t st)
{
    if (slot < 0)
        return;
    hipEventRecord(g_prof_ev[g_prof_rec[slot].ev + 1], st);
}

filt_status check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(FILT_EHIP, "%s: %s", what, hipGetErrorString(e));
    return FILT_OK;
}


inline int pow2_at_least(int v)
{
    int w = 1;
    while (w < v)
        w <<= 1;
    return w;
}

int64_t auto_chunk(const filt_problem *p)
{
    const int64_t B = p->B, T = p->T;
    // Enough (channel, chunk) chains to keep every SIMD busy in the apply
    // phase.  Per-sample filters pay N + 1 solves per sample in the summary
    // whatever the chunk length, plus an N x N FP64 transition per chunk, so
    // they take fewer, longer chunks; time-invariant filters summarise with one
    // solve per sample and favour many short chunks.
    const int64_t target = p->time_varying ? 32768 : 262144;
    int64_t per = (target + B - 1) / std::max<int64_t>(B, 1);
    int64_t L = (T + per - 1) / std::max<int64_t>(per, 1);
    if (p->time_varying) {
        // keep the 8 (N^2 + N) / L transition bytes per sample well below
        // the 4 (N + M + 1) bytes of coefficients.  The order-16 bucket in
        // [T, B] takes longer chunks still (its applies run four lanes per
        // chain and the carry is the longer part); in [B, T] a wavefront's
        // chains sit L rows apart, and 16 N = 256 rows of 64 bytes is a
        // power-of-two stride that piles their loads onto the same memory
        // channels
        const bool longer = p->N > 8 && p->layout == FILT_LAYOUT_TB;
        L = std::max<int64_t>(L, (longer ? 16 : 12) * (int64_t)p->N);
    } else {
        L = std::max<int64_t>(L, 128);
    }
    L = ((L + 31) / 32) * 32;
    return std::max<int64_t>(32, std::min<int64_t>(L, 1 << 16));
}

filt_status validate(const filt_problem *p, const void *x_or_gy, const void *b, const void *a)
{
    if (p == nullptr)
        return fail(FILT_EINVAL, "problem is NULL");
    if (p->B < 0 || p->T < 0)
        return fail(FILT_EINVAL, "B and T must be >= 0 (B=%lld T=%lld)", (long long)p->B,
                    (long long)p->T);
    if (p->M < 0 || p->N < 0)
        return fail(FILT_EINVAL, "orders must be >= 0 (M=%d N=%d)", p->M, p->N);
    if (p->M > kMaxOrder || p->N > kMaxOrder)
        return fail(FILT_EUNSUPPORTED, "orders above %d are not supported (M=%d N=%d)",
                    kMaxOrder, p->M, p->N);
    if (p->layout != FILT_LAYOUT_TB && p->layout != FILT_LAYOUT_BT)
        return fail(FILT_EINVAL, "layout must be FILT_LAYOUT_TB or FILT_LAYOUT_BT");
    if (p->time_varying < 0)
        return fail(FILT_EINVAL, "time_varying must be 0, 1 or a hop >= 2 (got %d)",
                    p->time_varying);
    if (p->chunk < 0 || (p->chunk % 32) != 0)
        return fail(FILT_EINVAL, "chunk must be 0 or a positive multiple of 32 (got %d)",
                    p->chunk);
    if (p->flags & ~(FILT_F32_STATE | FILT_RECURRENCE | FILT_TOEPLITZ))
        return fail(FILT_EINVAL, "unknown flags 0x%x", p->flags);
    if (p->B == 0 || p->T == 0)
        return FILT_OK;
    if (p->time_varying > 1 && p->T >= ((int64_t)1 << 31))
        return fail(FILT_EUNSUPPORTED, "frame-held coefficients need T < 2^31 (T=%lld)",
                    (long long)p->T);
    if (p->layout == FILT_LAYOUT_TB &&
        p->B * (int64_t)(std::max(p->N, p->M + 1) + 1) >= ((int64_t)1 << 31))
        return fail(FILT_EUNSUPPORTED, "[T][B] layout with B * taps >= 2^31 (B=%lld)",
                    (long long)p->B);
    if (x_or_gy == nullptr)
        return fail(FILT_EINVAL, "input signal is NULL");
    if (b == nullptr && p->M != 0)
        return fail(FILT_EINVAL, "b is NULL but M=%d (NULL b means b=[1], M=0)", p->M);
    if (a == nullptr && p->N != 0)
        return fail(FILT_EINVAL, "a is NULL but N=%d", p->N);
    return FILT_OK;
}

// Time-invariant [B, T] problems with FP32 data take the matrix-core path
// unless the caller asks for the per-lane recurrence or another chunk length.
bool tz_eligible(const filt_problem *p, bool f32_io)
{
    return f32_io && (p->flags & FILT_TOEPLITZ) && !(p->flags & FILT_RECURRENCE) &&
           !p->time_varying && p->layout == FILT_LAYOUT_BT && p->N >= 1 &&
           (p->chunk == 0 || p->chunk == kTzL);
}

Dims make_dims(const filt_problem *p, int has_b, bool f32_io)
{
    Dims d{};
    d.tz = tz_eligible(p, f32_io);
    d.B = p->B;
    d.T = p->T;
    d.M = p->M;
    d.N = p->N;
    set_rows(d, p->time_varying);
    d.layout = p->layout;
    d.has_b = has_b;
    d.L = d.tz ? kTzL : (p->chunk > 0 ? p->chunk : auto_chunk(p));
    d.C = (d.T + d.L - 1) / d.L;
    const int64_t steps = std::max<int64_t>(d.C - 1, 1);
    int64_t G = 1;
    while (G * G < steps)
        ++G;
    d.G = G;
    d.NB = (steps + G - 1) / G;
    return d;
}

template <typename io_t, typename acc_t>
filt_status forward_dispatch(const Dims &d, int W, const io_t *x, const io_t *bc, const io_t *ac,
                             const io_t *xi, const io_t *yi, io_t *y, char *ws, hipStream_t st)
{
#define FWD(w)                                                                                     \
    case w:                                                                                        \
        return forward_w<w, io_t, acc_t>(d, x, bc, ac, xi, yi, y, ws, st);
    switch (W) {
        FWD(1) FWD(2) FWD(4) FWD(8) FWD(16) FWD(32)
    default:
        return fail(FILT_EUNSUPPORTED, "register bucket %d", W);
    }
#undef FWD
}

template <typename io_t, typename acc_t>
filt_status backward_dispatch(const Dims &d, int W, const io_t *gy, const io_t *x, const io_t *y,
                              const io_t *bc, const io_t *ac, const io_t *xi, const io_t *yi,
                              io_t *gx, io_t *gb, io_t *ga, io_t *gxi, io_t *gyi, char *ws,
                              hipStream_t st)
{
#define BWD(w)                                                                                     \
    case w:                                                                                        \
        return backward_w<w, io_t, acc_t>(d, gy, x, y, bc, ac, xi, yi, gx, gb, ga, gxi, gyi, ws, \
                                          st);
    switch (W) {
        BWD(1) BWD(2) BWD(4) BWD(8) BWD(16) BWD(32)
    default:
        return fail(FILT_EUNSUPPORTED, "register bucket %d", W);
    }
#undef BWD
}


template <typename T>
__global__ void __launch_bounds__(256) k_zero(T *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = T(0);
}

template <typename T>
filt_status zero_fill(T *p, int64_t n, hipStream_t st)
{
    if (p == nullptr || n <= 0)
        return FILT_OK;
    const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    FILT_LAUNCH("zero_fill", k_zero<T>, dim3(g), dim3(256), 0, st, p, n);
    return check_launch("zero fill");
}

template <typename io_t>
filt_status forward_entry(const filt_problem *p, const io_t *x, const io_t *bc, const io_t *ac,
                          const io_t *xi, const io_t *yi, io_t *y, void *ws, size_t ws_bytes,
                          void *stream)
{
    filt_status s = validate(p, x, bc, ac);
    if (s != FILT_OK)
        return s;
    if (p->B == 0 || p->T == 0)
        return FILT_OK;
    if (y == nullptr)
        return fail(FILT_EINVAL, "y is NULL");
    Dims d = make_dims(p, bc != nullptr, sizeof(io_t) == 4);
    {
        const int W = pow2_at_least(std::max(std::max(p->N, p->M + 1), 1));
        const size_t vec = W >= 4 ? 16 : (size_t)W * sizeof(*ac);
        d.a_vec = (p->N == W) && ((uintptr_t)ac % vec == 0);
        d.ga_vec = 0;
    }
    const WsPlan w = ws_plan(d);
    if (ws == nullptr || ws_bytes < w.total)
        return fail(FILT_EWORKSPACE, "workspace of %zu bytes needed, %zu given", w.total,
                    ws == nullptr ? (size_t)0 : ws_bytes);
    char *wsa = (char *)(((uintptr_t)ws + 255) & ~uintptr_t(255));
    const int W = pow2_at_least(std::max(std::max(p->N, p->M + 1), 1));
    hipStream_t st = (hipStream_t)stream;
    // without b the kernels read b_0 = 1 but still need a valid address
    const io_t *bvalid = bc != nullptr ? bc : (ac != nullptr ? ac : x);
    if constexpr (sizeof(io_t) == 4) {
        if (d.tz)
            return tz_forward(d, x, bvalid, ac, xi, yi, y, w, wsa, st);
    }
    const bool f64 = sizeof(io_t) == 8 || !(p->flags & FILT_F32_STATE);
    if (f64)
        return forward_dispatch<io_t, double>(d, W, x, bvalid, ac, xi, yi, y, wsa, st);
    return forward_dispatch<io_t, float>(d, W, x, bvalid, ac, xi, yi, y, wsa, st);
}

template <typename io_t>
filt_status backward_entry(const filt_problem *p, const io_t *gy, const io_t *x, const io_t *y,
                           const io_t *bc, const io_t *ac, const io_t *xi, const io_t *yi,
                           io_t *gx, io_t *gb, io_t *ga, io_t *gxi, io_t *gyi, void *ws,
                           size_t ws_bytes, void *stream)
{
    filt_status s = validate(p, gy, bc, ac);
    if (s != FILT_OK)
        return s;
    if (p->B == 0 || p->T == 0) {
        // no output depends on any input: the per-channel gradients (initial
        // conditions, time-invariant coefficients) are zero, the per-sample
        // ones are empty.  Cleared by a kernel, not a memset node, so the call
        // stays capturable.
        if (p->B == 0)
            return FILT_OK;
        hipStream_t st = (hipStream_t)stream;
        const int64_t nb = p->time_varying ? 0 : p->B * (int64_t)(p->M + 1);
        const int64_t na = p->time_varying ? 0 : p->B * (int64_t)p->N;
        s = zero_fill(gb, bc != nullptr ? nb : 0, st);
        if (s == FILT_OK)
            s = zero_fill(ga, na, st);
        if (s == FILT_OK)
            s = zero_fill(gxi, p->B * (int64_t)p->M, st);
        if (s == FILT_OK)
            s = zero_fill(gyi, p->B * (int64_t)p->N, st);
        return s;
    }
    if (gb != nullptr && bc == nullptr)
        return fail(FILT_EINVAL, "gb requested but b is NULL");
    if (gb != nullptr && x == nullptr)
        return fail(FILT_EINVAL, "gb requested but x is NULL");
    if (ga != nullptr && (y == nullptr || p->N == 0))
        return fail(FILT_EINVAL, "ga requested but y is NULL or N == 0");
    Dims d = make_dims(p, bc != nullptr, sizeof(io_t) == 4);
    {
        const int W = pow2_at_least(std::max(std::max(p->N, p->M + 1), 1));
        const size_t vec = W >= 4 ? 16 : (size_t)W * sizeof(*ac);
        d.a_vec = (p->N == W) && ((uintptr_t)ac % vec == 0);
        // full-row kernels also store ga rows as vectors
        d.a_vec = d.a_vec && (ga == nullptr || ((uintptr_t)ga % vec == 0));
        d.ga_vec = d.a_vec;
    }
    const WsPlan w = ws_plan(d);
    if (ws == nullptr || ws_bytes < w.total)
        return fail(FILT_EWORKSPACE, "workspace of %zu bytes needed, %zu given", w.total,
                    ws == nullptr ? (size_t)0 : ws_bytes);
    char *wsa = (char *)(((uintptr_t)ws + 255) & ~uintptr_t(255));
    const int W = pow2_at_least(std::max(std::max(p->N, p->M + 1), 1));
    hipStream_t st = (hipStream_t)stream;
    // without b the kernels read b_0 = 1 but still need a valid address
    const io_t *bvalid = bc != nullptr ? bc : (ac != nullptr ? ac : gy);
    if constexpr (sizeof(io_t) == 4) {
        if (d.tz)
            return tz_backward(d, gy, x, y, bvalid, ac, xi, yi, gx, gb, ga, gxi, gyi, w, wsa, st);
    }
    const bool f64 = sizeof(io_t) == 8 || !(p->flags & FILT_F32_STATE);
    if (f64)
        return backward_dispatch<io_t, double>(d, W, gy, x, y, bvalid, ac, xi, yi, gx, gb, ga, gxi,
                                               gyi, wsa, st);
    return backward_dispatch<io_t, float>(d, W, gy, x, y, bvalid, ac, xi, yi, gx, gb, ga, gxi, gyi,
                                          wsa, st);
}


// ------------------------------------------------------------ static scratch
//
// filt_forward_noalloc runs the forward with its workspace in this array
// instead of a caller buffer.  Every device the library runs on holds its
// own copy from module load until the process ends.  In host code `scratch`
// only names the symbol: its device address is looked up once per device
// (with that device current) and kept in g_scratch_ptr.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

filt_status scratch_of_current_device(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess)
        return fail(FILT_EHIP, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(FILT_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            return fail(FILT_EHIP, "hipGetSymbolAddress of the static scratch failed: %s",
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FILT_OK;
}

}  // namespace filt_detail

using namespace filt_detail;


extern "C" {

filt_status filt_forward_noalloc(const filt_problem *p, const float *x, const float *b,
                                 const float *a, const float *xi, const float *yi, float *y,
                                 void *stream)
{
    filt_status s = validate(p, x, b, a);
    if (s != FILT_OK)
        return s;
    if (p->B == 0 || p->T == 0)
        return FILT_OK;
    // the workspace this problem needs, with the 256-byte alignment margin
    const size_t need = ws_plan(make_dims(p, b != nullptr, true)).total;
    if (need > kScratchBytes)
        return fail(FILT_EWORKSPACE,
                    "problem needs %zu bytes of workspace, the static scratch holds %zu "
                    "(use filt_forward with a caller workspace)",
                    need, kScratchBytes);
    void *ws = nullptr;
    s = scratch_of_current_device(&ws);
    if (s != FILT_OK)
        return s;
    return forward_entry<float>(p, x, b, a, xi, yi, y, ws, kScratchBytes, stream);
}

filt_status filt_workspace_bytes(const filt_problem *p, size_t *bytes)
{
    filt_status s = validate(p, (const void *)1, (const void *)1, (const void *)1);
    if (s != FILT_OK)
        return s;
    if (bytes == nullptr)
        return fail(FILT_EINVAL, "bytes is NULL");
    if (p->B == 0 || p->T == 0) {
        *bytes = 0;
        return FILT_OK;
    }
    // either data type: the matrix-core path serves FP32 data only
    *bytes = std::max(ws_plan(make_dims(p, 1, true)).total, ws_plan(make_dims(p, 1, false)).total);
    return FILT_OK;
}

int64_t filt_auto_chunk(const filt_problem *p)
{
    if (p == nullptr || p->B <= 0 || p->T <= 0)
        return 0;
    if (tz_eligible(p, true))
        return kTzL;
    return p->chunk > 0 ? p->chunk : auto_chunk(p);
}

filt_status filt_forward(const filt_problem *p, const float *x, const float *b, const float *a,
                         const float *xi, const float *yi, float *y, void *ws, size_t ws_bytes,
                         void *stream)
{
    return forward_entry<float>(p, x, b, a, xi, yi, y, ws, ws_bytes, stream);
}

filt_status filt_backward(const filt_problem *p, const float *gy, const float *x, const float *y,
                          const float *b, const float *a, const float *xi, const float *yi,
                          float *gx, float *gb, float *ga, float *gxi, float *gyi, void *ws,
                          size_t ws_bytes, void *stream)
{
    return backward_entry<float>(p, gy, x, y, b, a, xi, yi, gx, gb, ga, gxi, gyi, ws, ws_bytes,
                                 stream);
}

filt_status filt_forward_f64(const filt_problem *p, const double *x, const double *b,
                             const double *a, const double *xi, const double *yi, double *y,
                             void *ws, size_t ws_bytes, void *stream)
{
    return forward_entry<double>(p, x, b, a, xi, yi, y, ws, ws_bytes, stream);
}

filt_status filt_backward_f64(const filt_problem *p, const double *gy, const double *x,
                              const double *y, const double *b, const double *a,
                              const double *xi, const double *yi, double *gx, double *gb,
                              double *ga, double *gxi, double *gyi, void *ws, size_t ws_bytes,
                              void *stream)
{
    return backward_entry<double>(p, gy, x, y, b, a, xi, yi, gx, gb, ga, gxi, gyi, ws, ws_bytes,
                                  stream);
}

const char *filt_strerror(filt_status s)
{
    switch (s) {
    case FILT_OK:
        return "ok";
    case FILT_EINVAL:
        return "invalid argument";
    case FILT_EUNSUPPORTED:
        return "unsupported problem";
    case FILT_EWORKSPACE:
        return "workspace too small";
    case FILT_EHIP:
        return "HIP error";
    }
    return "unknown status";
}

const char *filt_last_error(void) { return g_err; }

filt_status filt_profile_enable(int on)
{
    if (on) {
        while (g_prof_nev < kProfEvents) {
            if (hipEventCreate(&g_prof_ev[g_prof_nev]) != hipSuccess)
                return fail(FILT_EHIP, "hipEventCreate failed");
            ++g_prof_nev;
        }
        g_prof_used = 0;
        g_prof_nrec = 0;
    }
    g_prof_on = on != 0;
    return FILT_OK;
}

filt_status filt_profile_only(const char *name)
{
    if (name == nullptr) {
        g_prof_only[0] = 0;
        return FILT_OK;
    }
    if (strlen(name) >= sizeof g_prof_only)
        return fail(FILT_EINVAL, "kernel name longer than %zu characters", sizeof g_prof_only - 1);
    strcpy(g_prof_only, name);
    return FILT_OK;
}

int filt_profile_read(char *names, int32_t *counts, double *total_ms, int max_entries)
{
    int n = 0;
    for (int r = 0; r < g_prof_nrec; ++r) {
        float ms = 0.f;
        if (hipEventSynchronize(g_prof_ev[g_prof_rec[r].ev + 1]) != hipSuccess ||
            hipEventElapsedTime(&ms, g_prof_ev[g_prof_rec[r].ev], g_prof_ev[g_prof_rec[r].ev + 1]) !=
                hipSuccess)
            continue;
        int k = 0;
        while (k < n && strncmp(names + 64 * k, g_prof_rec[r].name, 63) != 0)
            ++k;
        if (k == n) {
            if (n >= max_entries)
                continue;
            strncpy(names + 64 * k, g_prof_rec[r].name, 63);
            names[64 * k + 63] = 0;
            counts[k] = 0;
            total_ms[k] = 0.0;
            ++n;
        }
        counts[k] += 1;
        total_ms[k] += ms;
    }
    return n;
}

}  // extern "C"
