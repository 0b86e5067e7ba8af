/*
 * filt.h -- C ABI of the MI355X (gfx950) direct-form filter library libfilt.so.
 *
 * The library computes the direct-form IIR recursion of
 * Yu & Fazekas, "Accelerating Automatic Differentiation of Direct Form
 * Digital Filters" (arXiv 2511.14390), Sec. 2 Eq. 1 read as a difference
 * equation with per-sample coefficients and initial conditions,
 *
 *     y[n] = sum_{k=0..M} b_k[n] x[n-k] - sum_{k=1..N} a_k[n] y[n-k],
 *
 * and its closed-form backward (Sec. 3.1 Eqs. 6-9, Appendix A): an adjoint
 * filter run in reverse time with the same coefficients plus reductions for
 * the coefficient and initial-condition gradients.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array pointer is a DEVICE pointer (hipMalloc'd or torch-owned GPU
 *   memory) unless marked (host).  The caller owns every buffer; the library
 *   keeps no reference after a call returns.
 * - Every call is asynchronous on `stream` (a hipStream_t passed as void*;
 *   NULL = the default stream).  The calls never allocate device memory,
 *   never synchronise and never read device memory from the host, so they may
 *   be captured into a HIP graph.  Scratch space is the caller's workspace.
 * - Signals are FP32 (float) in layout FILT_LAYOUT_TB ([T][B], x[t*B+b]) or
 *   FILT_LAYOUT_BT ([B][T], x[b*T+t]), dense.
 * - Coefficients: a holds a_1..a_N (a_0 = 1 is implicit, sign as in Eq. 1;
 *   callers normalise by a_0), b holds b_0..b_M.  Time-invariant: a[B][N],
 *   b[B][M+1].  Per-sample (time_varying = 1): the signal layout with the tap
 *   index innermost, [T][B][K] (TB) or [B][T][K] (BT).  Frame-held
 *   (time_varying = h >= 2, the parameter-varying case of the paper's closing
 *   remarks): one row per frame of h samples, frame f applying to samples
 *   [f h, min((f + 1) h, T)), F = ceil(T / h) rows per channel laid out as
 *   [F][B][K] (TB) or [B][F][K] (BT); needs T < 2^31.  The gradients of
 *   frame-held rows have the same shapes and are the per-sample gradients
 *   summed over each frame's samples (the chain rule through the hold).
 * - Initial conditions, most recent first: xi[B][M] with xi[b][j-1] = x[-j],
 *   yi[B][N] with yi[b][j-1] = y[-j].  NULL means zero.
 * - Errors: the return value; a thread-local message is available from
 *   filt_last_error().  Argument errors are detected on the host before any
 *   GPU work is queued (nothing is written).  FILT_EHIP reports a failed
 *   launch; outputs are then undefined.
 */
#ifndef FILT_H
#define FILT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FILT_OK = 0,
    FILT_EINVAL = 1,       /* bad argument (NULL where required, bad size/layout) */
    FILT_EUNSUPPORTED = 2, /* valid but not implemented (e.g. order above 16) */
    FILT_EWORKSPACE = 3,   /* workspace NULL or smaller than filt_workspace_bytes */
    FILT_EHIP = 4          /* a HIP runtime call or kernel launch failed */
} filt_status;

typedef enum { FILT_LAYOUT_TB = 0, FILT_LAYOUT_BT = 1 } filt_layout;

/* flags.  By default every recursion runs in FP64 registers (I/O stays
 * FP32): on gfx950 an FP64 FMA issues at the rate of an unpacked FP32 FMA, and
 * FP32 state misses the 1e-4 output tolerance on high-order filters whose
 * poles cluster near the unit circle.  FILT_F32_STATE runs the per-sample
 * output pass in FP32 instead (the chunk transitions and the carry stay FP64). */
#define FILT_F32_STATE 0x2
/* FILT_TOEPLITZ: time-invariant problems in the [B][T] layout (FP32 entry
 * points) run the chunked scan with each chunk's response computed as a
 * lower-triangular Toeplitz matrix product on the FP32 matrix cores (chunks
 * of 64 samples; chunk must be 0 or 64) and the chunk carry in FP64.  Its
 * error is that of FP32 sums in which the entering state's response can
 * cancel: about 1e-6 relative for moderate poles, but up to 5e-4 for two
 * pole pairs of radius near 0.99 (one draw in twelve of that domain), so it
 * is opt-in.  By default (and with FILT_RECURRENCE, kept for compatibility)
 * every problem runs the per-lane recurrence with FP64 state. */
#define FILT_RECURRENCE 0x4
#define FILT_TOEPLITZ 0x8

typedef struct {
    int64_t B;            /* channels (>= 0); B == 0 or T == 0 writes no signal (see
                             filt_backward for the per-channel gradients then) */
    int64_t T;            /* samples per channel (>= 0) */
    int32_t M;            /* feed-forward order: b_0..b_M, 0 <= M <= 16 */
    int32_t N;            /* feedback order: a_1..a_N, 0 <= N <= 16 */
    int32_t time_varying; /* 0: coefficients per channel; 1: per sample; h >= 2: per
                             frame of h samples (see the conventions above) */
    int32_t layout;       /* filt_layout of x, y, gy, gx (and per-sample coefficients) */
    int32_t flags;        /* FILT_F32_STATE | FILT_RECURRENCE | FILT_TOEPLITZ, or 0 */
    int32_t chunk;        /* time-chunk length for the parallel scan; 0 = automatic,
                             else a multiple of 32 */
} filt_problem;

/* Size in bytes of the workspace that filt_forward / filt_backward need for
 * problem *p (the larger of the two).  bytes is a host pointer. */
filt_status filt_workspace_bytes(const filt_problem *p, size_t *bytes);

/* Forward filter (Eq. 1 as a difference equation).
 *   x   [layout]        input signal
 *   b   coefficients    NULL => b = [1] (then M must be 0)
 *   a   coefficients    may be NULL only when N == 0
 *   xi  [B][M] or NULL, yi [B][N] or NULL
 *   y   [layout]        output, written in full
 *   ws  workspace of at least filt_workspace_bytes(p) bytes (device) */
filt_status filt_forward(const filt_problem *p, const float *x, const float *b, const float *a,
                         const float *xi, const float *yi, float *y, void *ws, size_t ws_bytes,
                         void *stream);

/* Closed-form backward (Eqs. 6-9, App. A), given gy = dL/dy:
 *   ybar[n] = gy[n] - sum_k a_k[n+k] ybar[n+k]     (reverse time, zero past T-1)
 *   gx[n]   = sum_k b_k[n+k] ybar[n+k]
 *   gb_k[n] = ybar[n] x[n-k],  ga_k[n] = -ybar[n] y[n-k]
 *             (summed over n when time_varying == 0, over each frame's
 *             samples when it is a hop h >= 2)
 *   gxi[j-1] = sum_{k>=j} b_k[k-j] ybar[k-j],  gyi[j-1] = -sum_{k>=j} a_k[k-j] ybar[k-j]
 * x, xi are read only when gb is requested or M > 0 matters for it; y, yi
 * only when ga is requested.  Each of gx, gb, ga, gxi, gyi may be NULL (not
 * computed); the others are written in full with the shapes of x, b, a, xi,
 * yi.  With T == 0 (and B > 0) no output depends on any input: the
 * per-channel outputs (gxi, gyi and the time-invariant gb, ga) are set to
 * zero by a kernel on the stream and FILT_OK is returned. */
filt_status filt_backward(const filt_problem *p, const float *gy, const float *x, const float *y,
                          const float *b, const float *a, const float *xi, const float *yi,
                          float *gx, float *gb, float *ga, float *gxi, float *gyi, void *ws,
                          size_t ws_bytes, void *stream);

/* filt_forward without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Arguments as filt_forward.  The workspace is a
 * static device array of the library (64 MiB on every device it runs on,
 * held until the process ends); the call allocates nothing.  Problems whose
 * workspace (filt_workspace_bytes) exceeds 64 MiB are rejected on the host
 * with FILT_EWORKSPACE.  Every call on one device shares that array and
 * leaves its contents behind: calls that overlap on one device (concurrent
 * streams, or threads) race and must be serialised by the caller. */
filt_status filt_forward_noalloc(const filt_problem *p, const float *x, const float *b,
                                 const float *a, const float *xi, const float *yi, float *y,
                                 void *stream);

/* Forward-mode derivative (Jacobian-vector product): the tangent dy of the
 * output along tangents of the inputs,
 *   dy[n] = sum_k b_k[n] dx[n-k] + sum_k db_k[n] x[n-k]
 *           - sum_k da_k[n] y[n-k] - sum_k a_k[n] dy[n-k],
 * with dx[-j] = dxi[j-1], dy[-j] = dyi[j-1] and the histories of x and y from
 * xi and yi (Eq. 1 differentiated; the same recursion as the forward, run on
 * the tangent input).  x, y (= filt_forward's output), b, a, xi, yi as for
 * filt_backward; each tangent dx, db, da, dxi, dyi has the shape of its
 * input and may be NULL (zero).  x is read only with db, y and yi only with
 * da.  dy [layout] is written in full.  ws: at least
 * filt_jvp_workspace_bytes(p) bytes. */
filt_status filt_jvp_workspace_bytes(const filt_problem *p, size_t *bytes);
filt_status filt_jvp(const filt_problem *p, const float *x, const float *y, const float *b,
                     const float *a, const float *xi, const float *yi, const float *dx,
                     const float *db, const float *da, const float *dxi, const float *dyi,
                     float *dy, void *ws, size_t ws_bytes, void *stream);

/* Derivative of the backward pass (reverse over reverse: Hessian-vector
 * products for the second-order optimisation the paper's closing remarks
 * point to).  filt_backward maps (gy, x, y, a, b, xi, yi), y taken as an
 * input of its own, to (gx, gb, ga, gxi, gyi); for cotangents vx, vb, va,
 * vxi, vyi of those outputs (shapes of gx, gb, ga, gxi, gyi; each may be
 * NULL = zero) this writes the gradients of
 *   Q = <vx, gx> + <vb, gb> + <va, ga> + <vxi, gxi> + <vyi, gyi>:
 *   wgy = dy, the forward-mode tangent along the cotangents (filt_jvp),
 *   wx[m]     = sum_{k=0..M} vb_k[m+k] ybar[m+k],   wxi likewise,
 *   wb_k[n]   = ybar[n] vx[n-k]   (history vxi),
 *   wy[m]     = -sum_{k=1..N} va_k[m+k] ybar[m+k],  wyi likewise,
 *   wa_k[n]   = -ybar[n] dy[n-k]  (history vyi),
 * ybar the adjoint of gy; time-invariant wb / wa summed over n, frame-held
 * ones over each frame.  Shapes: wgy, wx, wy [layout]; wb, wa, wxi, wyi as
 * b, a, xi, yi.  Every output may be NULL (not computed).  b == NULL (b =
 * [1]) needs M == 0 and vb, wb NULL; N == 0 needs va, wa NULL; vb needs x,
 * va needs y.  T == 0 with B > 0 zero-fills the per-channel outputs given.
 * FP32 entry point; async on stream, no allocation.  ws: at least
 * filt_backward2_workspace_bytes(p) bytes (three signals, three coefficient
 * arrays and the largest workspace of the passes it runs). */
filt_status filt_backward2_workspace_bytes(const filt_problem *p, size_t *bytes);
filt_status filt_backward2(const filt_problem *p, const float *gy, const float *x,
                           const float *y, const float *b, const float *a, const float *xi,
                           const float *yi, const float *vx, const float *vb, const float *va,
                           const float *vxi, const float *vyi, float *wgy, float *wx, float *wy,
                           float *wb, float *wa, float *wxi, float *wyi, void *ws,
                           size_t ws_bytes, void *stream);

/* Matrix recurrence (the state-space recursion of Sec. 2 Eq. 4 with the
 * input already in state space; the operator of App. B), per channel b:
 *   v(n+1) = A v(n) + z(n),  n = 0 .. T-1,  v(0) = v0,
 * output v(1) .. v(T).  The problem takes p->N = K, the state size
 * (1 <= K <= 16), p->M = 0, p->time_varying = 0; p->chunk as for the filters.
 * A [B][K][K] row-major (v_i(n+1) = sum_j A[b][i][j] v_j(n) + z_i(n)),
 * v0 [B][K] or NULL (zero); z, v [B][T][K] (FILT_LAYOUT_BT) or [T][B][K]
 * (FILT_LAYOUT_TB), v[.., n, ..] = v(n+1).  The state runs in FP64.
 * Backward (Sec. 3.1 Eqs. 7 and 9 for this operator), given gv = dL/dv:
 *   gz(n) = gv(n) + A^T gz(n+1) (gz(T) = 0),  gv0 = A^T gz(0),
 *   gA = sum_n gz(n) v(n)^T  (v(0) = v0),
 * gz [layout] required, gA [B][K][K] and gv0 [B][K] may be NULL; v is
 * filt_mr_forward's output.  T == 0 with B > 0: the backward zero-fills gA
 * and gv0.  ws: at least filt_mr_workspace_bytes(p) bytes. */
filt_status filt_mr_workspace_bytes(const filt_problem *p, size_t *bytes);
filt_status filt_mr_forward(const filt_problem *p, const float *A, const float *v0,
                            const float *z, float *v, void *ws, size_t ws_bytes, void *stream);
filt_status filt_mr_backward(const filt_problem *p, const float *A, const float *v0,
                             const float *v, const float *gv, float *gz, float *gA, float *gv0,
                             void *ws, size_t ws_bytes, void *stream);

/* Transposed direct form II with an initial state (Sec. 2: the state-space
 * form of Eqs. 4-5 with the companion matrix transposed and B, C swapped;
 * SciPy's lfilter(b, a, x, zi)), time-invariant coefficients only
 * (p->time_varying must be 0; FILT_EUNSUPPORTED otherwise).  With
 * K = max(M, N) (at least 1), b_j = 0 past M and a_j = 0 past N:
 *   y(n) = b_0 x(n) + z_0(n-1),
 *   z_i(n) = b_{i+1} x(n) - a_{i+1} y(n) + z_{i+1}(n-1),  z(-1) = zi,
 * x and y zero before time 0.  b [B][M+1] is required (b = [1] is a row of
 * one 1), a [B][N] may be NULL only when N == 0, zi [B][K] may be NULL
 * (zero state).  Signals in p->layout.  The backward (Sec. 3.1 Eqs. 6-9 for
 * this realisation) writes gx [layout], gb [B][M+1], ga [B][N] (needs y and
 * N > 0), gzi [B][K]; each may be NULL.  x is read only for gb.  T == 0 with
 * B > 0 zero-fills the per-channel gradients it was given.  ws: at least
 * filt_tdf_workspace_bytes(p) bytes. */
filt_status filt_tdf_workspace_bytes(const filt_problem *p, size_t *bytes);
filt_status filt_tdf_forward(const filt_problem *p, const float *x, const float *b,
                             const float *a, const float *zi, float *y, void *ws, size_t ws_bytes,
                             void *stream);
filt_status filt_tdf_backward(const filt_problem *p, const float *gy, const float *x,
                              const float *y, const float *b, const float *a, const float *zi,
                              float *gx, float *gb, float *ga, float *gzi, void *ws,
                              size_t ws_bytes, void *stream);

/* Cascades of nsec second-order sections (biquads; the structure used for
 * higher orders to keep rounding errors small, Sec. 4), SciPy's sosfilt
 * semantics: section k filters section k-1's output (x for k = 0) in the
 * transposed direct form II above with its own initial state.  p->M and
 * p->N must be 2 and p->time_varying 0; coefficients are section-major:
 * b [nsec][B][3] (b_0 b_1 b_2), a [nsec][B][2] (a_1 a_2, a_0 = 1 implied),
 * zi [nsec][B][2] or NULL (zero states).  The backward writes gx [layout]
 * and gb, ga, gzi in the shapes of b, a, zi (each may be NULL); it needs x
 * and y (the forward's output) and recomputes the sections' inputs.
 * ws: at least filt_sos_workspace_bytes(p, nsec) bytes (nsec + 1 signals
 * plus one section's workspace). */
filt_status filt_sos_workspace_bytes(const filt_problem *p, int32_t nsec, size_t *bytes);
filt_status filt_sos_forward(const filt_problem *p, int32_t nsec, const float *x, const float *b,
                             const float *a, const float *zi, float *y, void *ws, size_t ws_bytes,
                             void *stream);
filt_status filt_sos_backward(const filt_problem *p, int32_t nsec, const float *gy,
                              const float *x, const float *y, const float *b, const float *a,
                              const float *zi, float *gx, float *gb, float *ga, float *gzi,
                              void *ws, size_t ws_bytes, void *stream);

/* The same two operations on FP64 data, computed in FP64 (for numerical
 * gradient checks).  Arguments as above with double in place of float. */
filt_status filt_forward_f64(const filt_problem *p, const double *x, const double *b,
                             const double *a, const double *xi, const double *yi, double *y,
                             void *ws, size_t ws_bytes, void *stream);
filt_status filt_backward_f64(const filt_problem *p, const double *gy, const double *x,
                              const double *y, const double *b, const double *a,
                              const double *xi, const double *yi, double *gx, double *gb,
                              double *ga, double *gxi, double *gyi, void *ws, size_t ws_bytes,
                              void *stream);

/* ------------------------------------------------------------------------
 * Batched ragged filtering: many independent all-pole filters (M = 0,
 * b = [1]) with per-sample coefficients, of different lengths and orders,
 * packed into flat arrays and run by one plan.  This is the batching of the
 * method across uneven filters (one launch per phase and order bucket,
 * optionally replayed as one HIP graph) with chunk lengths picked by an
 * autotuner; each filter computes exactly what filt_forward / filt_backward
 * compute for it with B = 1 in the [B][T] layout.
 *
 * Segment i covers samples [x_off, x_off + T) of x / y / gy / gx, its
 * coefficient rows a[a_off + r*N .. a_off + r*N + N) (a_1..a_N) and its
 * initial conditions yi[ic_off .. ic_off + N) (y[-1] first).  With hop 0 or 1
 * the rows are per sample (r = t < T); with hop h >= 2 they are frame-held
 * (r = t / h < ceil(T / h)), and ga holds per-frame gradients (each the sum
 * over the frame's samples), as filt_backward with time_varying = h.
 * Segments must not overlap in the outputs.  Coefficient blocks that start on
 * a multiple of 4 floats (16 bytes) are read as whole vectors.
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t x_off;  /* first sample in x, y, gy, gx */
    int64_t T;      /* samples (>= 0) */
    int64_t a_off;  /* first coefficient in a / ga */
    int64_t ic_off; /* first initial condition in yi / gyi */
    int32_t N;      /* order, 0 <= N <= 16 */
    int32_t hop;    /* 0 or 1: a row per sample; h >= 2: a row per frame of h samples */
} filt_segment;

typedef struct filt_plan filt_plan;

/* Build a plan (host call; allocates its device tables and workspace and
 * synchronises).  segs is a host array of nseg segments.  chunks: NULL for
 * the defaults, else a host array of 5 entries for the order buckets
 * N <= 1, 2, 4, 8, 16: -1 runs the bucket's single-pass kernel (one launch
 * per direction, tiles chained by decoupled look-back), a positive multiple
 * of 32 the three-phase scan (summaries, carry, apply) with that chunk
 * length, 0 the default (single pass for orders up to 4, else the three-phase
 * scan at its default chunk). */
filt_status filt_plan_create(const filt_segment *segs, int32_t nseg, const int32_t *chunks,
                             filt_plan **out);
void filt_plan_destroy(filt_plan *p);

/* Forward / backward of every segment, asynchronous on stream, no
 * allocation.  Backward: ga (the layout of a: per sample or per frame) and
 * gyi may be NULL; y is needed for ga.  gx may be NULL. */
filt_status filt_plan_forward(filt_plan *p, const float *x, const float *a, const float *yi,
                              float *y, void *stream);
filt_status filt_plan_backward(filt_plan *p, const float *gy, const float *y, const float *a,
                               const float *yi, float *gx, float *ga, float *gyi, void *stream);

/* Autotuner: for each order bucket, time forward + backward of that bucket's
 * segments with the single-pass kernel and with the three-phase scan at
 * several chunk lengths (HIP events, median of 3) and keep the fastest; then
 * re-lay the plan.  Synchronises; the outputs are scratch.  get_chunks
 * reports the choice in the form filt_plan_create takes (-1: single pass). */
filt_status filt_plan_tune(filt_plan *p, const float *x, const float *a, const float *yi,
                           const float *gy, float *y, float *gx, float *ga, float *gyi,
                           void *stream);
filt_status filt_plan_get_chunks(const filt_plan *p, int32_t *chunks /* host, 5 */);

/* Capture forward + backward on these buffers into a HIP graph (the stream
 * must not be capturing already), and replay it.  In the graph each order
 * bucket's backward follows its own forward directly (one fork and one join
 * for the step), so buckets overlap across the two directions; the results
 * equal filt_plan_forward followed by filt_plan_backward. */
filt_status filt_plan_capture(filt_plan *p, const float *x, const float *a, const float *yi,
                              const float *gy, float *y, float *gx, float *ga, float *gyi,
                              void *stream);
filt_status filt_plan_replay(filt_plan *p, void *stream);

/* Chunk length the library picks for *p when p->chunk == 0 (for tests and
 * tuning).  Host-only; returns 0 for an invalid problem. */
int64_t filt_auto_chunk(const filt_problem *p);

/* Diagnostics for benchmarking: per-kernel GPU time.  While enabled, the
 * library records a HIP event pair on the launch stream around every kernel
 * it launches (no synchronisation).  filt_profile_enable(1) creates the
 * events on the host (not to be called during graph capture) and clears the
 * previous records; filt_profile_enable(0) stops recording.
 * filt_profile_read synchronises the recorded events and fills, per kernel
 * name, the launch count and the total milliseconds; names is a host buffer
 * of max_entries * 64 chars, counts / total_ms host arrays of max_entries.
 * Returns the number of entries filled.  Not thread-safe. */
filt_status filt_profile_enable(int on);
/* Restrict the recording to launches of one kernel name (as reported by
 * filt_profile_read), so that a timed loop carries two events per launch of
 * that kernel only; NULL (or "") records every launch again.  name is a host
 * string of at most 63 characters, copied; FILT_EINVAL if longer. */
filt_status filt_profile_only(const char *name);
int filt_profile_read(char *names, int32_t *counts, double *total_ms, int max_entries);

/* Text of a status code, and the last error message of the calling thread. */
const char *filt_strerror(filt_status s);
const char *filt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FILT_H */
