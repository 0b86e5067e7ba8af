"""GPU tests of the batched ragged plan (many uneven all-pole filters).

Each segment is checked against the FP64 oracle run on that segment alone,
and against the dense per-filter C-ABI call on the same segment; graph replay
is checked against eager execution.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2511_14390_amd import filt as F
from paper_2511_14390_amd import workloads as W
from tests.helpers import chan_rel_err, vec_rel_err

pytestmark = pytest.mark.gpu

TIGHT = 2e-6   # FP64 recursion, FP32 I/O


def _to(dev, *arrs):
    return [None if v is None else torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in arrs]


def _oracle_segment(s, i):
    x, a, yi, gy = s.segment(i)
    y = oracle.forward(x[None], a[None], None, None, yi[None] if len(yi) else None, layout="BT")
    g = oracle.backward(gy[None], x[None], y, a[None], None, None,
                        yi[None] if len(yi) else None, layout="BT", want=("x", "a", "yi"))
    return y[0], g


def _run_plan(s, dev, chunks=None):
    x, a, yi, gy = _to(dev, s.x, s.a, s.yi, s.gy)
    plan = F.BatchedFilter(s.T, s.N, s.x_off, s.a_off, s.ic_off, chunks=chunks)
    y = plan.forward(x, a, yi)
    g = plan.backward(gy, y, a, yi)
    torch.cuda.synchronize()
    return plan, (x, a, yi, gy), y, g


def _check_segments(s, y, g, tol, which=None):
    y = y.cpu().numpy()
    gx, ga, gyi = (g[k].cpu().numpy() for k in ("x", "a", "yi"))
    worst = 0.0
    for i in (which if which is not None else range(len(s.T))):
        t, n = int(s.T[i]), int(s.N[i])
        xo, ao, io = int(s.x_off[i]), int(s.a_off[i]), int(s.ic_off[i])
        yo, go = _oracle_segment(s, i)
        e = [chan_rel_err(y[xo:xo + t][None], yo[None], "BT"),
             chan_rel_err(gx[xo:xo + t][None], go["x"], "BT")]
        if n > 0:
            e.append(chan_rel_err(ga[ao:ao + t * n].reshape(1, t, n), go["a"], "BT"))
            e.append(vec_rel_err(gyi[io:io + n][None], go["yi"]))
        worst = max(worst, max(e))
        assert max(e) <= tol, (i, t, n, e)
    print(f"[batched] {len(s.T)} segments, worst rel err {worst:.2e}", flush=True)


def test_batched_matches_oracle_per_segment(gpu_device):
    s = W.config5(nseg=24, Tmin=1000, Tmax=20000)
    _, _, y, g = _run_plan(s, gpu_device)
    _check_segments(s, y, g, TIGHT)


def test_batched_short_empty_and_passthrough_segments(gpu_device):
    # T < chunk, T = 1, T = 0 and an order-0 (y = x) segment among normal ones
    T = np.array([1, 0, 40, 300, 33, 257], dtype=np.int64)
    N = np.array([2, 4, 0, 16, 1, 8], dtype=np.int32)
    # rebuild a packed problem with these sizes from the generator's values
    rng = np.random.default_rng(5)
    x_off = np.concatenate([[0], np.cumsum(T)[:-1]]).astype(np.int64)
    a_len = (T * N + 3) // 4 * 4
    a_off = np.concatenate([[0], np.cumsum(a_len)[:-1]]).astype(np.int64)
    ic_off = np.concatenate([[0], np.cumsum(N)[:-1]]).astype(np.int64)
    a = np.zeros(int(a_len.sum()), np.float32)
    for i in range(6):
        t, n = int(T[i]), int(N[i])
        if t and n:
            k = rng.uniform(-0.9, 0.9, (-(-t // 16), n))
            frames = W.bandwidth_expand(W.reflection_to_direct(k), 0.95)
            a[a_off[i]:a_off[i] + t * n] = W.frame_held(frames, t, 16, 0).reshape(-1)
    s = W.Segments(T, N, x_off, a_off, ic_off, rng.standard_normal(int(T.sum())).astype(np.float32),
                   a, rng.normal(0, 0.1, int(N.sum())).astype(np.float32),
                   rng.standard_normal(int(T.sum())).astype(np.float32))
    for chunks in ([32, 32, 32, 64, 64], [-1, -1, -1, -1, -1]):
        _, _, y, g = _run_plan(s, gpu_device, chunks=chunks)
        _check_segments(s, y, g, TIGHT, which=[0, 2, 3, 4, 5])


def _segments_of_orders(T, N, seed):
    """A packed problem with the given lengths and orders (per-sample rows
    from bandwidth-expanded reflection coefficients held over 16 samples)."""
    T = np.asarray(T, dtype=np.int64)
    N = np.asarray(N, dtype=np.int32)
    rng = np.random.default_rng(seed)
    x_off = np.concatenate([[0], np.cumsum(T)[:-1]]).astype(np.int64)
    a_len = (T * N + 3) // 4 * 4
    a_off = np.concatenate([[0], np.cumsum(a_len)[:-1]]).astype(np.int64)
    ic_off = np.concatenate([[0], np.cumsum(N)[:-1]]).astype(np.int64)
    a = np.zeros(int(a_len.sum()), np.float32)
    for i in range(len(T)):
        t, n = int(T[i]), int(N[i])
        if t and n:
            k = rng.uniform(-0.9, 0.9, (-(-t // 16), n))
            frames = W.bandwidth_expand(W.reflection_to_direct(k), 0.95)
            a[a_off[i]:a_off[i] + t * n] = W.frame_held(frames, t, 16, 0).reshape(-1)
    return W.Segments(T, N, x_off, a_off, ic_off,
                      rng.standard_normal(int(T.sum())).astype(np.float32), a,
                      rng.normal(0, 0.1, int(N.sum())).astype(np.float32),
                      rng.standard_normal(int(T.sum())).astype(np.float32))


@pytest.mark.parametrize("chunks", [[32, 32, 32, 64, 128], [-1, -1, -1, 256, 512]])
def test_batched_every_order_of_the_upper_buckets(gpu_device, chunks):
    # orders 5..16 (the order 5..8 and 9..16 buckets' row summaries, the
    # lanes past N zeroed), ragged lengths with a partial last chunk
    N = [5, 6, 7, 8, 9, 11, 13, 15, 16, 3]
    T = [3001, 2049, 1537, 4100, 2222, 1999, 3333, 1025, 2600, 1800]
    s = _segments_of_orders(T, N, seed=21)
    _, _, y, g = _run_plan(s, gpu_device, chunks=chunks)
    _check_segments(s, y, g, TIGHT)


def test_batched_equals_dense_per_filter_calls(gpu_device):
    s = W.config5(nseg=10, Tmin=2000, Tmax=9000, seed=11)
    plan, (x, a, yi, gy), y, g = _run_plan(s, gpu_device)
    chunks = plan.chunks
    for i in range(len(s.T)):
        t, n = int(s.T[i]), int(s.N[i])
        xo, ao, io = int(s.x_off[i]), int(s.a_off[i]), int(s.ic_off[i])
        L = max(chunks[max(n - 1, 0).bit_length()], 0)  # -1: single pass, dense auto chunk
        xs = x[xo:xo + t][None]
        as_ = a[ao:ao + t * n].view(1, t, n)
        yis = yi[io:io + n][None]
        yd = F.filt_forward(xs, as_, None, None, yis, layout="BT", chunk=L)
        gd = F.filt_backward(gy[xo:xo + t][None], xs, yd, as_, None, None, yis, layout="BT",
                             chunk=L, want=("x", "a", "yi"))
        torch.cuda.synchronize()
        assert chan_rel_err(y[xo:xo + t][None].cpu().numpy(), yd.cpu().numpy(), "BT") <= 1e-6
        assert chan_rel_err(g["x"][xo:xo + t][None].cpu().numpy(), gd["x"].cpu().numpy(),
                            "BT") <= 1e-6
        assert chan_rel_err(g["a"][ao:ao + t * n].view(1, t, n).cpu().numpy(),
                            gd["a"].cpu().numpy(), "BT") <= 1e-6


def test_graph_replay_matches_eager(gpu_device):
    s = W.config5(nseg=12, Tmin=1000, Tmax=12000, seed=12)
    plan, (x, a, yi, gy), y_ref, g_ref = _run_plan(s, gpu_device)
    y = torch.empty_like(x)
    gx = torch.empty_like(x)
    ga = torch.zeros_like(a)
    gyi = torch.zeros_like(yi)
    plan.capture(x, a, yi, gy, y, gx, ga, gyi)
    for rep in range(3):
        y.fill_(float("nan"))
        gx.fill_(float("nan"))
        plan.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref), rep
        assert torch.equal(gx, g_ref["x"]), rep
        assert torch.equal(ga, g_ref["a"]), rep
        assert torch.equal(gyi, g_ref["yi"]), rep
        # eager work on the stream between replays
        _ = plan.forward(x, a, yi)
        torch.cuda.synchronize()


def test_autotuner_picks_valid_chunks_and_stays_exact(gpu_device):
    s = W.config5(nseg=16, Tmin=1000, Tmax=30000, seed=13)
    x, a, yi, gy = _to(gpu_device, s.x, s.a, s.yi, s.gy)
    plan = F.BatchedFilter(s.T, s.N, s.x_off, s.a_off, s.ic_off)
    chunks = plan.tune(x, a, yi, gy)
    print(f"[batched] tuned chunks {chunks}", flush=True)
    # -1: the single-pass kernel; else the three-phase scan's chunk length
    assert all(c == -1 or (c >= 32 and c % 32 == 0) for c in chunks)
    y = plan.forward(x, a, yi)
    g = plan.backward(gy, y, a, yi)
    torch.cuda.synchronize()
    _check_segments(s, y, g, TIGHT)


def _check_segments_threaded(s, y, g, tol, label):
    """Per-segment comparison with the oracle, segments spread over host
    threads (the oracle's C calls release the interpreter lock)."""
    import concurrent.futures as cf
    import os

    y = y.cpu().numpy()
    gx, ga, gyi = (g[k].cpu().numpy() for k in ("x", "a", "yi"))

    def one(i):
        t, n = int(s.T[i]), int(s.N[i])
        xo, ao, io = int(s.x_off[i]), int(s.a_off[i]), int(s.ic_off[i])
        yo, go = _oracle_segment(s, i)
        e = [chan_rel_err(y[xo:xo + t][None], yo[None], "BT"),
             chan_rel_err(gx[xo:xo + t][None], go["x"], "BT")]
        if n > 0:
            e.append(chan_rel_err(ga[ao:ao + t * n].reshape(1, t, n), go["a"], "BT"))
            e.append(vec_rel_err(gyi[io:io + n][None], go["yi"]))
        return i, t, n, max(e)

    with cf.ThreadPoolExecutor(min(16, len(os.sched_getaffinity(0)))) as ex:
        res = list(ex.map(one, range(len(s.T))))
    worst = max(r[3] for r in res)
    print(f"[batched] {label}: {len(s.T)} segments, worst rel err {worst:.2e}", flush=True)
    bad = [r for r in res if r[3] > tol]
    assert not bad, bad[:5]


def test_batched_full_size_workload_per_segment(gpu_device):
    # the benchmark's workload at full size: 512 segments, T up to 200 000
    # (order-16 carries over about 520 chunks stage their records in several
    # rounds), with the chunk lengths the tuner picks on the device
    s = W.config5()
    x, a, yi, gy = _to(gpu_device, s.x, s.a, s.yi, s.gy)
    plan = F.BatchedFilter(s.T, s.N, s.x_off, s.a_off, s.ic_off)
    chunks = plan.tune(x, a, yi, gy)
    y = plan.forward(x, a, yi)
    g = plan.backward(gy, y, a, yi)
    torch.cuda.synchronize()
    _check_segments_threaded(s, y, g, TIGHT, f"full size, chunks {chunks}")


@pytest.mark.parametrize("chunks", [[192, 192, 192, 192, 192], [64, 64, 128, 128, 384],
                                    [-1, -1, -1, -1, -1], [-1, 128, -1, 256, -1]])
def test_batched_long_order16_segment(gpu_device, chunks):
    # an order-16 segment of 200 000 samples among shorter ones of every
    # order: about 1042 chunks at 192 (G = NB = 33) and 521 at 384
    T = np.array([200000, 150001, 3000, 70000, 99999, 1000], dtype=np.int64)
    N = np.array([16, 8, 16, 4, 2, 1], dtype=np.int32)
    s = _packed(T, N, seed=21)
    _, _, y, g = _run_plan(s, gpu_device, chunks=chunks)
    _check_segments_threaded(s, y, g, TIGHT, f"long order 16, chunks {chunks}")


def _packed(T, N, seed, hop=128):
    rng = np.random.default_rng(seed)
    x_off = np.concatenate([[0], np.cumsum(T)[:-1]]).astype(np.int64)
    a_len = (T * N + 3) // 4 * 4
    a_off = np.concatenate([[0], np.cumsum(a_len)[:-1]]).astype(np.int64)
    ic_off = np.concatenate([[0], np.cumsum(N)[:-1]]).astype(np.int64)
    a = np.zeros(int(a_len.sum()), np.float32)
    for i in range(len(T)):
        t, n = int(T[i]), int(N[i])
        if t and n:
            k = rng.uniform(-0.9, 0.9, (-(-t // hop), n))
            frames = W.bandwidth_expand(W.reflection_to_direct(k), 0.99)
            a[a_off[i]:a_off[i] + t * n] = W.frame_held(frames, t, hop, 0).reshape(-1)
    return W.Segments(T, N, x_off, a_off, ic_off,
                      rng.standard_normal(int(T.sum())).astype(np.float32), a,
                      rng.normal(0, 0.1, int(N.sum())).astype(np.float32),
                      rng.standard_normal(int(T.sum())).astype(np.float32))
