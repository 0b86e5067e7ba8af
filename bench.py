"""Benchmark: forward + backward throughput of the direct-form filter on one GPU.

Default workload (``batched-ragged``): 512 independent all-pole filters of
uneven lengths T ~ U{1000..200000} and orders N in {1, 2, 4, 8, 16}, with
per-sample coefficients from frame-held (hop 128) reflection coefficients,
random initial states, FP32 I/O, packed into flat arrays (51.6 M samples).
One step = forward plus the full backward (gradients of x, of the per-sample
coefficients and of the initial states) of every filter, through the batched
plan with its autotuned chunk lengths, replayed as one HIP graph, with all
inputs already resident in HBM.  Also timed: the same work as plain
per-filter calls of the dense C ABI (eager, and the loop captured in a
graph), and the FP64 CPU oracle on the host's cores.

The other workloads (``--workload``): the per-sample order-16 filter
(64 x 48000), the time-invariant M = N = 4 filter on [65536, 1024] and the
long narrow order-4 filter (2 x 2^22), through the autograd.Function.
``--frames`` runs the per-sample workloads (batched-ragged, ltv-allpole-n16)
with their coefficients given as frame rows (one row per hop, the gradients
of the coefficients per frame) instead of per-sample rows.

Prints one JSON line with the dominant kernel's achieved HBM bandwidth
(algorithmic bytes per launch / its average duration, timed with HIP events
on the stream it runs on) and its HBM traffic as counted by rocprofv3 (from
the committed counter summary, only while the kernel sources are unchanged
since the count).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, 8 TB/s
FP64_VALU_PEAK_TFLOPS = 78.6   # MI355X FP64 vector: 256 CUs x 4 SIMD x 16 lanes x 2 x 2.4 GHz


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batched-ragged",
                    choices=["ltv-allpole-n16", "lti-allpole-n2", "lti-df-m4n4",
                             "lti-allpole-n4-long", "batched-ragged"])
    ap.add_argument("--plain-steps", type=int, default=3,
                    help="steps of the per-filter launch loop timed for comparison")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--bucket-chunks", default="",
                    help="batched-ragged: fixed chunk lengths for the five order buckets "
                         "(comma separated) instead of tuning")
    ap.add_argument("--layout", choices=["TB", "BT"], default=None,
                    help="signal layout (default: the workload's own)")
    ap.add_argument("--f32-state", action="store_true")
    ap.add_argument("--toeplitz", action="store_true",
                    help="time-invariant [B, T] workloads: the opt-in FP32 matrix-core path")
    ap.add_argument("--frames", action="store_true",
                    help="batched-ragged: the coefficients as frame rows (one per hop of 128 "
                         "samples, gradients per frame) instead of per-sample rows")
    ap.add_argument("--tdf", action="store_true",
                    help="lti-df-m4n4: the transposed direct form II with an initial state "
                         "(zi drawn like the workload's initial conditions) instead of the "
                         "direct form with input / output histories")
    ap.add_argument("--paper-sweep", action="store_true",
                    help="the paper's own benchmark: the state-space recursion "
                         "v(n+1) = A v(n) + z(n) with a 2-dimensional state, one signal of "
                         "T = 2^14 .. 2^20 samples, forward and forward + backward times, "
                         "beside the same lengths of the order-2 all-pole direct form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (a known-size kernel for "
                         "calibrating hardware byte counters)")
    return ap.parse_args()


def make_problem(name, frames=False):
    from paper_2511_14390_amd import workloads as W

    if frames:
        if name != "ltv-allpole-n16":
            raise SystemExit("--frames applies to the per-sample workloads (ltv-allpole-n16, "
                             "batched-ragged)")
        return W.config2(frames=True)
    return {"ltv-allpole-n16": W.config2, "lti-allpole-n2": W.config1,
            "lti-df-m4n4": W.config3, "lti-allpole-n4-long": W.config4}[name]()


def to_layout(p, layout):
    """The same problem with signals (and per-sample coefficients) transposed
    between [B, T] and [T, B]."""
    import numpy as np

    from paper_2511_14390_amd import workloads as W

    sw = lambda v: None if v is None else np.ascontiguousarray(np.swapaxes(v, 0, 1))
    a = sw(p.a) if p.a.ndim == 3 else p.a
    b = (sw(p.b) if p.b.ndim == 3 else p.b) if p.b is not None else None
    return W.Problem(p.name, layout, sw(p.x), a, b, p.xi, p.yi, sw(p.gy), dict(p.meta))


def kernel_bytes(p, name):
    """Algorithmic bytes per sample of each library kernel: the tensors of the
    algorithm that the kernel's phase must move, each counted once.  Signals
    are 4 B/sample; per-sample coefficients 4*K B/sample."""
    K_a = p.N
    K_b = (p.M + 1) if p.b is not None else 0
    # per-sample rows, or frame rows (one per hop samples)
    hop = int(p.meta.get("hop", 1)) if p.meta.get("frames") else 1
    coef = 4 * (K_a + K_b) / hop if p.time_varying else 0
    fir = 4 if p.M > 0 else 0
    W = 1
    while W < max(p.N, p.M + 1):
        W *= 2
    # order-16 bucket: with an FIR part or per-sample gains b the adjoint pass
    # leaves the coefficient products to a separate pass; without them it
    # forms ga itself
    split = W >= 16 and (p.M > 0 or p.b is not None)
    table = {
        # time-invariant [B, T] problems on the matrix cores: the tile kernels
        # move only signals (the per-channel matrices stay in L2)
        "tz_fwd_apply": 4 + 4,
        "tz_bwd_apply": 4 + 4 + 4 + (4 if (p.M > 0 and p.b is not None) else 0),
        "tz_fwd_summary": 4,
        "tz_bwd_summary": 4,
        # forward: read x (+ coefficients), write y
        "fwd_apply": 4 + 4 + coef,
        "stream_fwd_apply": 4 + 4 + coef,
        # backward adjoint pass that leaves the coefficient products to a
        # separate pass: read gy and the row, write gx (= ybar)
        "stream_bwd_apply": 4 + coef + 4,
        # per-sample coefficient gradients: read ybar and y, write the rows
        "coef_grads": 4 + 4 + coef,
        # frame-held rows: read ybar and y (x too with an FIR part), write
        # one row per frame
        "frame_coef_grads": 4 + 4 + fir + coef,
        # backward: read gy, y (+ x for M > 0) and coefficients; write gx and
        # the per-sample coefficient gradients (split: read gy, the row, write
        # gx, the products left to coef_grads)
        "bwd_apply": (4 + coef + 4 + fir) if (split and p.time_varying)
                     else (4 + 4 + fir + 4 + 2 * coef),
        # chunk summaries read their phase's inputs once
        "fwd_summary": 4 + coef,
        "bwd_summary": 4 + coef,
        # transposed form: the feed-forward input (read x, write u), the
        # feed-forward adjoint (read ybar, write gx; in [T, B] it also reads x
        # for the gb partial sums) and the separate gb partial sums of [B, T]
        # (read ybar and x)
        "tdf_input": 8,
        "tdf_fir_adjoint": 12 if p.layout == "TB" else 8,
        "tdf_gb_partial": 8,
    }
    return table.get(name)


def kernel_flops(p, name, chunk):
    """FP64 FLOPs per sample of the kernels bound by vector arithmetic: the
    per-sample chunk summaries solve N homogeneous recursions and one driven
    one of N FMAs each per sample, over every chunk but the one with no
    successor (forward) / predecessor (backward)."""
    if name not in ("fwd_summary", "bwd_summary") or not p.time_varying:
        return None
    C = -(-p.T // chunk)
    return 2.0 * (p.N + 1) * (p.N + p.M) * (C - 1) / C


def source_digest():
    """Digest of the library's kernel sources: a counted traffic figure is
    used only for the sources it was counted on."""
    import glob
    import hashlib

    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2511_14390_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def counted_traffic(workload, layout, chunk, kernel):
    """HBM bytes per launch of `kernel` from a `traffic-record:` line of the
    counter summaries in profiles/ (FETCH_SIZE and WRITE_SIZE, each scaled by
    the same counter's reading for a 1 GiB copy), or None when no record
    matches this workload, layout, chunk and the current sources."""
    import glob

    digest = source_digest()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_hbm_counters.md"))):
        for line in open(f):
            if not line.startswith("traffic-record:"):
                continue
            kv = dict(t.split("=", 1) for t in line.split()[1:])
            if (kv.get("workload") == workload and kv.get("layout") == layout
                    and int(kv.get("chunk", -1)) == chunk and kv.get("kernel") == kernel
                    and kv.get("sources") == digest):
                return int(kv["read_bytes"]) + int(kv["write_bytes"])
    return None


def batched_kernel_bytes(s, chunks, name):
    """Algorithmic bytes of one launch of a batched kernel (name ends in the
    order bucket, e.g. ``batched_fwd_apply_w16``): the bytes of that phase
    (signals 4 B per sample, coefficient rows 4 N B per row: one row per
    sample, or per frame of hop samples for frame-held rows) summed over the
    bucket's segments and the samples the phase covers.  None for the carry
    kernels (they move O(N^2) doubles per chunk, not samples)."""
    import numpy as np

    kind, _, w = name.rpartition("_w")
    if not w.isdigit():
        return None
    W = int(w)
    bucket = {1: 0, 2: 1, 4: 2, 8: 3, 16: 4}[W]
    L = max(chunks[bucket], 1)
    Wb = np.maximum(1, 2 ** np.ceil(np.log2(np.maximum(s.N, 1)))).astype(np.int64)
    sel = Wb == W
    T = s.T[sel].astype(np.float64)
    N = s.N[sel].astype(np.float64)
    rows = np.asarray(s.rows, np.float64)[sel] / np.maximum(T, 1)  # rows per sample
    C = np.ceil(T / L)
    # the forward summarises chunks 0..C-2, the adjoint chunks 1..C-1
    summ = np.maximum(T - L, 0) * (C > 1)
    frames = bool(s.meta.get("frames"))
    per = {
        # read the signal and the coefficient rows
        "batched_fwd_summary": (summ, 4, 4),
        "batched_bwd_summary": (summ, 4, 4),
        # read x and the rows, write y
        "batched_fwd_apply": (T, 8, 4),
        "batched_stream_fwd": (T, 8, 4),
        "batched_onepass_fwd": (T, 8, 4),
        # read gy and the rows, write gx (= ybar for b = [1]); the per-sample
        # products go to coef_grads
        "batched_bwd_apply": (T, 8, 4),
        "batched_stream_bwd": (T, 8, 4),
        # single pass: read gy and the rows, write gx and (per-sample rows)
        # the ga rows, reading y for them
        "batched_onepass_bwd": (T, 8 if frames else 12, 4 if frames else 8),
        # read ybar and y, write the ga rows
        "batched_coef_grads": (T, 8, 4),
        "batched_frame_grads": (T, 8, 4),
    }.get(kind)
    if per is None:
        return None
    if kind == "batched_bwd_apply" and W == 16 and not frames:
        # the staged order-16 adjoint forms the per-sample ga rows itself
        # (reads y, writes the rows): no separate coef_grads pass
        per = (T, 12, 8)
    n, sig, coef = per
    return float((n * (sig + coef * N * rows)).sum())


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def batched_cpu_baseline(s, seconds):
    """The FP64 oracle over every segment of the batched workload (forward +
    backward with the gradients of x, a and yi), once on one thread and
    repeated on all host cores (one segment per task)."""
    import concurrent.futures as cf

    import numpy as np

    import oracle

    hop = int(s.meta["hop"]) if s.meta.get("frames") else 1

    def one(i):
        x, a, yi, gy = s.segment(i)
        x64, a64, gy64 = (np.asarray(v, np.float64)[None] for v in (x, a, gy))
        yi64 = np.asarray(yi, np.float64)[None] if len(yi) else None
        if hop > 1:
            y = oracle.forward_frames(x64, a64, None, None, yi64, hop=hop, layout="BT",
                                      nthreads=1)
            oracle.backward_frames(gy64, x64, y, a64, None, None, yi64, hop=hop, layout="BT",
                                   want=("x", "a", "yi"), nthreads=1)
            return
        y = oracle.forward(x64, a64, None, None, yi64, layout="BT", nthreads=1)
        oracle.backward(gy64, x64, y, a64, None, None, yi64, layout="BT", want=("x", "a", "yi"),
                        nthreads=1)

    samples = int(s.T.sum())
    order = list(np.argsort(-s.T))   # longest first
    c0 = time.perf_counter()
    for i in order:
        one(i)
    one_thread = samples / (time.perf_counter() - c0) / 1e9
    cores = len(os.sched_getaffinity(0))
    reps, c0 = 0, time.perf_counter()
    with cf.ThreadPoolExecutor(cores) as ex:
        while True:
            list(ex.map(one, order))
            reps += 1
            if time.perf_counter() - c0 >= seconds:
                break
    dt = time.perf_counter() - c0
    return {"value": round(samples * reps / dt / 1e9, 6), "unit": "Gsamples/s", "cores": cores,
            "kind": "oracle", "value_1_thread": round(one_thread, 6), "cpu_model": cpu_model(),
            "sample": f"the whole workload ({len(s.T)} segments, {samples} samples, fwd + bwd "
                      f"with grads of x, a and yi), FP64; once on 1 thread, then {reps}x on "
                      f"{cores} threads (one segment per task) in {dt:.1f} s"}


def batched_main(args):
    """Many uneven per-sample all-pole filters: the batched plan (autotuned
    chunk lengths, forward + backward replayed as a HIP graph) against plain
    per-filter calls of the dense C ABI on the same stream (eager, and the
    same loop captured in a graph)."""
    import numpy as np
    import torch

    from paper_2511_14390_amd import filt as F
    from paper_2511_14390_amd import workloads as W

    dev = torch.device("cuda:0")
    s = W.config5(frames=args.frames)
    hop = int(s.meta["hop"]) if args.frames else 1
    workload = "batched-ragged-frames" if args.frames else "batched-ragged"
    t = lambda v: torch.from_numpy(v).to(dev)
    x, a, yi, gy = t(s.x), t(s.a), t(s.yi), t(s.gy)
    samples = int(s.T.sum())
    if args.chunk > 0 or args.bucket_chunks:
        # fixed chunk lengths (no tuning)
        fixed = ([int(v) for v in args.bucket_chunks.split(",")] if args.bucket_chunks
                 else [args.chunk] * 5)
        plan = F.BatchedFilter(s.T, s.N, s.x_off, s.a_off, s.ic_off, chunks=fixed, hop=hop)
        chunks = plan.chunks
    else:
        plan = F.BatchedFilter(s.T, s.N, s.x_off, s.a_off, s.ic_off, hop=hop)
        chunks = plan.tune(x, a, yi, gy)
    y = torch.empty_like(x)
    gx = torch.empty_like(x)
    ga = torch.zeros_like(a)
    gyi = torch.zeros_like(yi)

    def eager_step():
        plan.forward(x, a, yi, out=y)
        plan.backward(gy, y, a, yi, out={"x": gx, "a": ga, "yi": gyi})

    # warm-up: eager steps, every launch between an event pair (first one
    # unrecorded) for the per-kernel breakdown and the dominant kernel
    eager_step()
    torch.cuda.synchronize()
    F.profile_only(None)
    F.profile_enable(True)
    wsteps = max(args.warmup, 1)
    for _ in range(wsteps):
        eager_step()
    torch.cuda.synchronize()
    F.profile_enable(False)
    prof = F.profile_read()
    kern = {k: {"launches": c // wsteps, "avg_us": round(1e3 * ms / c, 2),
                "total_ms_per_step": round(ms / wsteps, 4)} for k, (c, ms) in prof.items()}
    # the dominant kernel among those moving a per-sample volume (the carry
    # kernels, several small launches per step, have no per-sample figure)
    sized = [k for k in kern if batched_kernel_bytes(s, chunks, k) is not None]
    pool = sized or list(kern)
    dom = max(pool, key=lambda k: kern[k]["total_ms_per_step"]) if pool else None

    if args.calib_copy_mib > 0:
        src = torch.empty(args.calib_copy_mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # timed region 1: graph replays of the whole step (value)
    plan.capture(x, a, yi, gy, y, gx, ga, gyi)
    for _ in range(max(1, args.warmup)):
        plan.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    value = samples / (ms * 1e-3) / 1e9

    # timed region 2: the same steps launched eagerly with one HIP event pair
    # per launch of the dominant kernel only, recorded on the stream it runs
    # on (roofline.achieved); event pairs around every launch slow the
    # kernels they bracket, so the breakdown above is only used to pick it
    F.profile_only(dom)
    F.profile_enable(True)
    torch.cuda.synchronize()
    e0 = time.perf_counter()
    for _ in range(args.steps):
        eager_step()
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - e0) * 1e3 / args.steps
    F.profile_enable(False)
    live = F.profile_read()
    F.profile_only(None)

    roofline = None
    if dom in live:
        c, dms = live[dom]
        avg_us = 1e3 * dms / c
        kern[dom]["eager_region_avg_us"] = round(avg_us, 2)
        kern[dom]["eager_region_launches"] = c
        per_launch = batched_kernel_bytes(s, chunks, dom)
        if per_launch is not None:
            ach = per_launch / (avg_us * 1e-6) / 1e9
            roofline = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(ach / HBM_PEAK_GBS, 4),
                        "traffic": counted_traffic(workload, "packed", chunks[4], dom),
                        "bytes_per_launch": per_launch, "avg_launch_us": round(avg_us, 2)}
            # the launch time above is a wall time while the other buckets'
            # streams share the GPU; the same kernel with its bucket alone (a
            # plan over that bucket's segments, same chunk lengths, eager
            # steps, events around its launches) for context
            Wd = int(dom.rpartition("_w")[2])
            Wb = np.maximum(1, 2 ** np.ceil(np.log2(np.maximum(s.N, 1)))).astype(np.int64)
            sel = np.nonzero(Wb == Wd)[0]
            solo = F.BatchedFilter(s.T[sel], s.N[sel], s.x_off[sel], s.a_off[sel],
                                   s.ic_off[sel], chunks=chunks, hop=hop)

            def solo_step():
                solo.forward(x, a, yi, out=y)
                solo.backward(gy, y, a, yi, out={"x": gx, "a": ga, "yi": gyi})

            solo_step()
            torch.cuda.synchronize()
            F.profile_only(dom)
            F.profile_enable(True)
            for _ in range(args.steps):
                solo_step()
            torch.cuda.synchronize()
            F.profile_enable(False)
            alone = F.profile_read()
            F.profile_only(None)
            solo.close()
            if dom in alone:
                c1, ms1 = alone[dom]
                us1 = 1e3 * ms1 / c1
                roofline["alone"] = {"avg_launch_us": round(us1, 2),
                                     "achieved": round(per_launch / (us1 * 1e-6) / 1e9, 1),
                                     "frac": round(per_launch / (us1 * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                                     "what": "the kernel's bucket alone on the GPU"}

    # plain: one dense forward + backward call per filter, eager and captured
    segs = [(int(s.T[i]), int(s.N[i]), int(s.x_off[i]), int(s.a_off[i]), int(s.ic_off[i]),
             int(s.rows[i])) for i in range(len(s.T))]

    def plain_step():
        for (tt, n, xo, ao, io, r) in segs:
            xs = x[xo:xo + tt][None]
            as_ = a[ao:ao + r * n].view(1, r, n)
            yis = yi[io:io + n][None]
            ys = F.filt_forward(xs, as_, None, None, yis, layout="BT", hop=hop)
            F.filt_backward(gy[xo:xo + tt][None], xs, ys, as_, None, None, yis, layout="BT",
                            hop=hop, want=("x", "a", "yi"))

    plain_ms = plain_graph_ms = None
    if args.plain_steps > 0:
        plain_step()
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for _ in range(args.plain_steps):
            plain_step()
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - p0) * 1e3 / args.plain_steps
        try:
            g = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                plain_step()
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            with torch.cuda.graph(g):
                plain_step()
            g.replay()
            torch.cuda.synchronize()
            p0 = time.perf_counter()
            for _ in range(args.plain_steps):
                g.replay()
            torch.cuda.synchronize()
            plain_graph_ms = (time.perf_counter() - p0) * 1e3 / args.plain_steps
            del g
        except Exception as e:  # reported, not fatal
            print(f"plain loop graph capture failed: {e}", file=sys.stderr, flush=True)

    coef = 4 * float((np.asarray(s.rows) * s.N).sum())
    # forward: x, y, the rows; backward: gy, y, gx, the rows read, ga written
    algo = 4 * samples * 2 + coef + (4 * samples * 3 + 2 * coef)
    cpu = None if args.no_cpu_baseline else batched_cpu_baseline(s, args.cpu_seconds)
    rec = {
        "metric": "fwd+bwd Gsamples/s & % HBM roofline, batched vs plain, rel err <=1e-4 vs FP64",
        "value": round(value, 4), "unit": "Gsamples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": workload, "io": "f32", "segments": len(s.T),
                   "samples": samples, "T_range": [int(s.T.min()), int(s.T.max())],
                   "orders": sorted(set(int(n) for n in s.N)), "hop": s.meta["hop"],
                   "coefficients": ("frame rows (one per hop, gradients per frame)"
                                    if args.frames else "per-sample rows"),
                   "chunks_by_order_bucket": chunks, "timed": "hip graph replay",
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "eager_ms_per_step": round(eager_ms, 4),
        "whole_step_algorithmic_bytes": algo,
        "whole_step_hbm_frac": round(algo / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
        "plain_ms_per_step": round(plain_ms, 3) if plain_ms else None,
        "plain_graph_ms_per_step": round(plain_graph_ms, 3) if plain_graph_ms else None,
        "batched_speedup_vs_plain": round(plain_ms / ms, 2) if plain_ms else None,
        "batched_speedup_vs_plain_graph": (round(plain_graph_ms / ms, 2)
                                           if plain_graph_ms else None),
        "kernels": kern,
    }
    print(json.dumps(rec), flush=True)


# The paper's Figure 1 (RTX 5060 Ti, FP32, batch unstated): its custom
# operator's forward and "backprop" runtimes in microseconds at
# T = 2^14, 2^16, 2^18, 2^20.
PAPER_FIG1_GPU_US = {"fwd": [135.0, 141.0, 155.3, 213.6], "backprop": [451.5, 463.0, 709.6,
                                                                          2394.9]}


def paper_sweep_main(args):
    """The state-space recursion of the paper's benchmark (2-dimensional
    state, time-invariant, one signal) through the autograd functions:
    median forward and forward + backward times over the timed repeats,
    each bracketed by events on the current stream."""
    import math

    import numpy as np
    import torch

    from paper_2511_14390_amd import autograd as AG

    dev = torch.device("cuda:0")
    rng = np.random.default_rng(2024)
    # a stable 2 x 2 transition with complex poles (radius 0.95, angle 0.3)
    r, th = 0.95, 0.3
    A = np.array([[[r * math.cos(th), -r * math.sin(th)], [r * math.sin(th), r * math.cos(th)]]],
                 np.float32)
    rows = []
    for e, T in enumerate((1 << 14, 1 << 16, 1 << 18, 1 << 20)):
        z = torch.from_numpy(rng.standard_normal((1, T, 2)).astype(np.float32)).to(dev)
        gv = torch.from_numpy(rng.standard_normal((1, T, 2)).astype(np.float32)).to(dev)
        At = torch.from_numpy(A).to(dev)
        x = torch.from_numpy(rng.standard_normal((1, T)).astype(np.float32)).to(dev)
        gy = torch.from_numpy(rng.standard_normal((1, T)).astype(np.float32)).to(dev)
        a = torch.tensor([[-2 * r * math.cos(th), r * r]], dtype=torch.float32, device=dev)

        def timed(fn):
            for _ in range(args.warmup):
                fn()
            ts = []
            for _ in range(args.steps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                e1.synchronize()
                ts.append(e0.elapsed_time(e1) * 1e3)
            return float(np.median(ts))

        zr, Ar, xr, ar = (v.clone().requires_grad_(True) for v in (z, At, x, a))
        mr_f = timed(lambda: AG.matrix_recurrence(At, z))
        mr_fb = timed(lambda: torch.autograd.grad(AG.matrix_recurrence(Ar, zr), [Ar, zr], gv))
        df_f = timed(lambda: AG.lfilter(x, a))
        df_fb = timed(lambda: torch.autograd.grad(AG.lfilter(xr, ar), [xr, ar], gy))
        rows.append({"T": T, "mr_fwd_us": round(mr_f, 1), "mr_fwd_bwd_us": round(mr_fb, 1),
                     "df_fwd_us": round(df_f, 1), "df_fwd_bwd_us": round(df_fb, 1),
                     "paper_fwd_us": PAPER_FIG1_GPU_US["fwd"][e],
                     "paper_backprop_us": PAPER_FIG1_GPU_US["backprop"][e]})
    last = rows[-1]
    rec = {"metric": "the paper's Figure 1 workload: state-space recursion (2-dim state), "
                     "forward + backward time at T = 2^20",
           "value": last["mr_fwd_bwd_us"], "unit": "us", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(last["mr_fwd_bwd_us"] * 1e-3, 4),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "paper-fig1-state-space-m2", "io": "f32", "B": 1,
                      "K": 2, "parallelism": "single GPU",
                      "paper_hardware": "RTX 5060 Ti (the paper's; context only)"},
           "sweep": rows, "roofline": None, "cpu_baseline": None}
    # roofline of the forward + backward at T = 2^20 as a whole: algorithmic
    # bytes (z in, v out; gv, v in, gz out: 4 K each per step) over its time;
    # one signal is bound by the per-step latency of the recurrence, so the
    # fraction is small
    Tl, K = rows[-1]["T"], 2
    by = Tl * 4 * K * (2 + 3)
    ach = by / (last["mr_fwd_bwd_us"] * 1e-6) / 1e9
    rec["roofline"] = {"bound": "hbm", "kernel": "matrix recurrence forward + backward",
                       "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None,
                       "bytes_per_launch": by}
    if not args.no_cpu_baseline:
        import oracle

        # the oracle's matrix recurrence (FP64 NumPy loop over time, one
        # thread) on a bounded sample: 2^16 steps of the same recurrence
        Ts = 1 << 16
        zs = rng.standard_normal((1, Ts, 2))
        gs = rng.standard_normal((1, Ts, 2))
        reps, c0 = 0, time.perf_counter()
        while True:
            vo = oracle.mr_forward(A.astype(np.float64), None, zs)
            oracle.mr_backward(gs, A.astype(np.float64), None, vo)
            reps += 1
            if time.perf_counter() - c0 >= min(args.cpu_seconds, 10.0):
                break
        dt = time.perf_counter() - c0
        rec["cpu_baseline"] = {"value": round(Ts * reps / dt / 1e9, 6), "unit": "Gsamples/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"forward + backward of one 2^16-step signal, FP64 "
                                         f"NumPy loop, repeated {reps}x in {dt:.1f} s",
                               "gpu_at_2^20_gsamples_s": round(Tl / (last["mr_fwd_bwd_us"]
                                                                     * 1e-6) / 1e9, 4)}
    print(json.dumps(rec), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.paper_sweep:
        return paper_sweep_main(args)
    if args.workload == "batched-ragged":
        return batched_main(args)
    import numpy as np
    import torch

    from paper_2511_14390_amd import autograd as AG
    from paper_2511_14390_amd import filt as F

    dev = torch.device("cuda:0")
    p = make_problem(args.workload, args.frames)
    hop = int(p.meta["hop"]) if args.frames else 1
    # the per-sample workload runs channel-interleaved ([T, B]): one wavefront
    # then reads 64 channels' coefficient rows of one time step as one block
    layout = args.layout or ("TB" if args.workload == "ltv-allpole-n16" else p.layout)
    if layout != p.layout:
        p = to_layout(p, layout)
    t = lambda v, rg=False: None if v is None else torch.from_numpy(v).to(dev).requires_grad_(rg)
    x = t(p.x, True)
    a = t(p.a, True)
    b = t(p.b, p.b is not None)
    xi = t(p.xi, p.xi is not None)
    yi = t(p.yi, p.yi is not None)
    gy = t(p.gy)
    samples = p.B * p.T

    if args.tdf:
        if args.workload != "lti-df-m4n4":
            raise SystemExit("--tdf applies to lti-df-m4n4")
        # the transposed form's state zi [B, max(M, N)] from the same draw as
        # the workload's output history
        zi = t(p.yi, True)

    def step():
        if args.tdf:
            y = AG.lfilter_tdf(x, b, a, zi, layout=p.layout, chunk=args.chunk)
            torch.autograd.grad(y, [x, b, a, zi], gy)
            return
        y = AG.lfilter(x, a, b, xi, yi, layout=p.layout, chunk=args.chunk,
                       f32_state=args.f32_state, toeplitz=args.toeplitz, hop=hop)
        inputs = [v for v in (x, a, b, xi, yi) if v is not None]
        torch.autograd.grad(y, inputs, gy)

    # warmup: the first step untimed and unrecorded, the rest with an event
    # pair around every library launch for the per-kernel breakdown
    step()
    torch.cuda.synchronize()
    F.profile_only(None)
    F.profile_enable(True)
    wsteps = max(args.warmup - 1, 1)
    for _ in range(wsteps):
        step()
    torch.cuda.synchronize()
    F.profile_enable(False)
    prof = F.profile_read()
    kern = {k: {"launches": c // wsteps, "avg_us": 1e3 * ms / c, "total_ms_per_step": ms / wsteps}
            for k, (c, ms) in prof.items()}
    dom = max(kern, key=lambda k: kern[k]["total_ms_per_step"]) if kern else None
    if args.calib_copy_mib > 0:
        src = torch.empty(args.calib_copy_mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # timed region: events only around the dominant kernel's launches (on the
    # stream it runs on), so the step time carries two events per step
    # instead of two per launch
    F.profile_only(dom)
    F.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    F.profile_enable(False)
    live = F.profile_read()
    F.profile_only(None)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = samples / (ms_per_step * 1e-3) / 1e9
    if dom in live:
        c, ms = live[dom]
        kern[dom] = {"launches": c // args.steps, "avg_us": 1e3 * ms / c,
                     "total_ms_per_step": ms / args.steps, "timed_region": True}

    roofline = None
    chunk = F.auto_chunk(F.problem(x, a, b, p.layout, args.chunk, toeplitz=args.toeplitz,
                                   hop=hop))
    pk = p  # the problem whose per-sample bytes the library's kernels move
    if args.tdf:
        # the transposed form runs the all-pole kernels on the formed input
        from paper_2511_14390_amd import workloads as W

        pk = W.Problem(p.name, p.layout, p.x, p.a, None, None, None, p.gy, dict(p.meta))
    if dom is not None and kernel_flops(pk, dom, chunk) is not None:
        # the dominant kernel is bound by FP64 vector arithmetic (SQ counters:
        # VALU issue), so it is measured against the FP64 vector peak
        flop = kernel_flops(pk, dom, chunk) * samples
        ach = flop / (kern[dom]["avg_us"] * 1e-6) / 1e12
        roofline = {"bound": "alu", "kernel": dom, "achieved": round(ach, 2),
                    "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(ach / FP64_VALU_PEAK_TFLOPS, 4),
                    "traffic": counted_traffic(args.workload + ("-frames" if hop > 1 else ""),
                                               p.layout, chunk, dom),
                    "flops_per_launch": flop, "avg_launch_us": round(kern[dom]["avg_us"], 2)}
    elif dom is not None and kernel_bytes(pk, dom) is not None:
        per_launch = kernel_bytes(pk, dom) * samples
        ach = per_launch / (kern[dom]["avg_us"] * 1e-6) / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                    "traffic": counted_traffic(args.workload + ("-frames" if hop > 1 else ""),
                                               p.layout, chunk, dom),
                    "bytes_per_launch": per_launch,
                    "avg_launch_us": round(kern[dom]["avg_us"], 2)}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        cores = len(os.sched_getaffinity(0))
        nthreads = max(1, min(cores, p.B))
        f64 = lambda v: None if v is None else np.ascontiguousarray(v, dtype=np.float64)
        xs, as_, bs, xis, yis, gys = map(f64, (p.x, p.a, p.b, p.xi, p.yi, p.gy))
        sub = None
        if args.tdf:
            # the transposed form's oracle is a NumPy loop over time: a
            # bounded sample of 16 channels
            sub = np.arange(16)
            pick = (lambda v: v[:, sub]) if p.layout == "TB" else (lambda v: v[sub])
            xs, gys = pick(xs), pick(gys)
            bs, as_, zis = bs[sub], as_[sub], f64(p.yi)[sub]
        reps, c0 = 0, time.perf_counter()
        while True:
            if args.tdf:
                yo = oracle.tdf_forward(xs, bs, as_, zis, layout=p.layout)
                oracle.tdf_backward(gys, xs, bs, as_, zis, layout=p.layout)
            elif hop > 1:
                yo = oracle.forward_frames(xs, as_, bs, xis, yis, hop=hop, layout=p.layout,
                                           nthreads=nthreads)
                oracle.backward_frames(gys, xs, yo, as_, bs, xis, yis, hop=hop, layout=p.layout,
                                       nthreads=nthreads)
            else:
                yo = oracle.forward(xs, as_, bs, xis, yis, layout=p.layout, nthreads=nthreads)
                oracle.backward(gys, xs, yo, as_, bs, xis, yis, layout=p.layout,
                                nthreads=nthreads)
            reps += 1
            if time.perf_counter() - c0 >= args.cpu_seconds:
                break
        dt = time.perf_counter() - c0
        if sub is not None:
            cpu = {"value": round(len(sub) * p.T * reps / dt / 1e9, 6), "unit": "Gsamples/s",
                   "cores": 1, "kind": "oracle",
                   "sample": f"{len(sub)} of the {p.B} channels (fwd+bwd of the transposed "
                             f"form, FP64 NumPy state-space loop, 1 thread) repeated {reps}x, "
                             f"{dt:.1f} s"}
        else:
            cpu = {"value": round(samples * reps / dt / 1e9, 6), "unit": "Gsamples/s",
                   "cores": nthreads, "kind": "oracle",
                   "sample": f"the whole workload (fwd+bwd, all {p.B} channels) repeated "
                             f"{reps}x, FP64, {nthreads} threads over channels, {dt:.1f} s"}

    rec = {
        "metric": "fwd+bwd Gsamples/s & % HBM roofline, batched vs plain, rel err <=1e-4 vs FP64",
        "value": round(value, 4), "unit": "Gsamples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-state" if args.f32_state else ("f32-mfma" if args.toeplitz else "f64"),
        "data": "synthetic",
        "config": {"workload": p.name + ("-frames" if hop > 1 else "") + ("-tdf" if args.tdf
                                                                          else ""),
                   "io": "f32", "B": p.B,
                   "T": p.T, "M": p.M, "N": p.N,
                   "time_varying": bool(p.time_varying), "hop": hop, "layout": p.layout,
                   "chunk": chunk,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kern,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
