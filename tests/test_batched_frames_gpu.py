"""GPU tests of the batched plan with frame-held coefficients (segment hop
h >= 2: one row per frame of h samples, ga per frame).

Each segment is checked against the oracle on its frame-expanded rows with the
coefficient gradients reduced per frame (oracle.forward_frames /
oracle.backward_frames), in every kernel family of the plan (single-pass
tiles, three-phase scans with staged or quad applies), with per-sample and
frame-held segments mixed in one plan.
"""
import concurrent.futures as cf
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2511_14390_amd import filt as F
from paper_2511_14390_amd import workloads as W
from tests.helpers import chan_rel_err, vec_rel_err

pytestmark = pytest.mark.gpu

TIGHT = 2e-6   # FP64 recursion, FP32 I/O; the frame sums in FP64


def _to(dev, *arrs):
    return [None if v is None else torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in arrs]


def _mixed(T, N, hops, seed):
    """Packed segments with per-segment hop (1: per-sample rows)."""
    T = np.asarray(T, np.int64)
    N = np.asarray(N, np.int32)
    hops = np.asarray(hops, np.int64)
    R = np.where(hops > 1, (T + hops - 1) // np.maximum(hops, 1), T)
    x_off = np.concatenate([[0], np.cumsum(T)[:-1]]).astype(np.int64)
    a_len = (R * N + 3) // 4 * 4
    a_off = np.concatenate([[0], np.cumsum(a_len)[:-1]]).astype(np.int64)
    ic_off = np.concatenate([[0], np.cumsum(N)[:-1]]).astype(np.int64)
    a = np.zeros(int(a_len.sum()), np.float32)
    x = np.zeros(int(T.sum()), np.float32)
    gy = np.zeros(int(T.sum()), np.float32)
    yi = np.zeros(int(N.sum()), np.float32)
    for i in range(len(T)):
        t, n, h = int(T[i]), int(N[i]), int(hops[i])
        p = W.random_problem(seed + i, B=1, T=t, M=0, N=n, time_varying=True, layout="BT",
                             hop=max(h, 1) if h > 1 else 16, rho_max=0.97, with_b=False,
                             frames=h > 1)
        a[a_off[i]:a_off[i] + p.a.size] = p.a.reshape(-1)
        x[x_off[i]:x_off[i] + t] = p.x[0]
        gy[x_off[i]:x_off[i] + t] = p.gy[0]
        if n:
            yi[ic_off[i]:ic_off[i] + n] = p.yi[0]
    s = W.Segments(T, N, x_off, a_off, ic_off, x, a, yi, gy, {"hops": hops})
    return s, hops, R


def _run(s, hops, dev, chunks=None, want_gx=True):
    x, a, yi, gy = _to(dev, s.x, s.a, s.yi, s.gy)
    plan = F.BatchedFilter(s.T, s.N, s.x_off, s.a_off, s.ic_off, chunks=chunks, hop=hops)
    y = plan.forward(x, a, yi)
    want = ("x", "a", "yi") if want_gx else ("a", "yi")
    g = plan.backward(gy, y, a, yi, want=want)
    torch.cuda.synchronize()
    return plan, y, g


def _check(s, hops, R, y, g, tol, label, check_gx=True):
    y = y.cpu().numpy()
    gx = g["x"].cpu().numpy() if check_gx else None
    ga, gyi = g["a"].cpu().numpy(), g["yi"].cpu().numpy()

    def one(i):
        t, n, h, r = int(s.T[i]), int(s.N[i]), int(hops[i]), int(R[i])
        xo, ao, io = int(s.x_off[i]), int(s.a_off[i]), int(s.ic_off[i])
        xs = s.x[xo:xo + t][None]
        ar = s.a[ao:ao + r * n].reshape(1, r, n)
        yis = s.yi[io:io + n][None] if n else None
        if h > 1:
            yo = oracle.forward_frames(xs, ar, None, None, yis, hop=h, layout="BT")
            go = oracle.backward_frames(s.gy[xo:xo + t][None], xs, yo, ar, None, None, yis,
                                        hop=h, layout="BT", want=("x", "a", "yi"))
        else:
            yo = oracle.forward(xs, ar, None, None, yis, layout="BT")
            go = oracle.backward(s.gy[xo:xo + t][None], xs, yo, ar, None, None, yis,
                                 layout="BT", want=("x", "a", "yi"))
        e = [chan_rel_err(y[xo:xo + t][None], yo, "BT")]
        if check_gx:
            e.append(chan_rel_err(gx[xo:xo + t][None], go["x"], "BT"))
        if n > 0:
            e.append(chan_rel_err(ga[ao:ao + r * n].reshape(1, r, n), go["a"], "BT"))
            e.append(vec_rel_err(gyi[io:io + n][None], go["yi"]))
        return i, t, n, h, max(e)

    with cf.ThreadPoolExecutor(min(16, len(os.sched_getaffinity(0)))) as ex:
        res = list(ex.map(one, range(len(s.T))))
    worst = max(r[4] for r in res)
    print(f"[batched-frames] {label}: {len(s.T)} segments, worst rel err {worst:.2e}", flush=True)
    bad = [r for r in res if r[4] > tol]
    assert not bad, bad[:5]


PLANS = [None, [-1, -1, -1, -1, -1], [64, 64, 128, 256, 384], [-1, 128, -1, 192, 192],
         [32, 32, 32, 64, 64]]


@pytest.mark.parametrize("chunks", PLANS)
def test_batched_frames_every_kernel_family(gpu_device, chunks):
    # every order bucket, hops that divide the chunks and hops that do not,
    # short segments (T below one frame / one chunk) and per-sample segments
    T = [5000, 3001, 777, 12000, 9999, 40, 2500, 15000, 640, 20000, 1, 333]
    N = [1, 2, 4, 8, 16, 3, 16, 5, 12, 16, 2, 7]
    hops = [128, 7, 100, 240, 128, 64, 1, 33, 128, 2, 5, 1000]
    s, hops, R = _mixed(T, N, hops, seed=7700)
    _, y, g = _run(s, hops, gpu_device, chunks=chunks)
    _check(s, hops, R, y, g, TIGHT, f"chunks {chunks}")


def test_batched_frames_without_gx(gpu_device):
    # ga without gx: the plan stages the adjoint in its own buffer
    T = [4000, 6000, 3000, 9000, 7000]
    N = [1, 4, 8, 16, 16]
    hops = [128, 128, 1, 128, 64]
    s, hops, R = _mixed(T, N, hops, seed=7800)
    for chunks in (None, [-1, -1, -1, -1, -1], [64, 64, 64, 128, 256]):
        _, y, g = _run(s, hops, gpu_device, chunks=chunks, want_gx=False)
        _check(s, hops, R, y, g, TIGHT, f"no gx, chunks {chunks}", check_gx=False)


def test_batched_frames_graph_replay_matches_eager(gpu_device):
    s = W.config5(nseg=12, Tmin=1000, Tmax=12000, seed=12, frames=True)
    hop = s.meta["hop"]
    x, a, yi, gy = _to(gpu_device, s.x, s.a, s.yi, s.gy)
    plan = F.BatchedFilter(s.T, s.N, s.x_off, s.a_off, s.ic_off, hop=hop)
    y_ref = plan.forward(x, a, yi)
    g_ref = plan.backward(gy, y_ref, a, yi)
    y = torch.empty_like(x)
    gx = torch.empty_like(x)
    ga = torch.zeros_like(a)
    gyi = torch.zeros_like(yi)
    # the frame rows of every segment (blocks are padded to 16 bytes; the
    # padding is no output)
    rows = np.zeros(a.numel(), bool)
    for i in range(len(s.T)):
        ao = int(s.a_off[i])
        rows[ao:ao + int(s.rows[i]) * int(s.N[i])] = True
    rows = torch.from_numpy(rows).to(gpu_device)
    plan.capture(x, a, yi, gy, y, gx, ga, gyi)
    for rep in range(3):
        y.fill_(float("nan"))
        gx.fill_(float("nan"))
        ga.masked_fill_(rows, float("nan"))
        plan.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, y_ref), rep
        assert torch.equal(gx, g_ref["x"]), rep
        assert torch.equal(ga, g_ref["a"]), rep
        assert torch.equal(gyi, g_ref["yi"]), rep
        _ = plan.forward(x, a, yi)
        torch.cuda.synchronize()


def test_batched_frames_full_size_workload(gpu_device):
    # the batched workload with its frame rows (hop 128) instead of per-sample
    # rows: 512 segments, 51.6 M samples, tuned plan
    s = W.config5(frames=True)
    hop = s.meta["hop"]
    hops = np.full(len(s.T), hop, np.int64)
    x, a, yi, gy = _to(gpu_device, s.x, s.a, s.yi, s.gy)
    plan = F.BatchedFilter(s.T, s.N, s.x_off, s.a_off, s.ic_off, hop=hop)
    chunks = plan.tune(x, a, yi, gy)
    y = plan.forward(x, a, yi)
    g = plan.backward(gy, y, a, yi)
    torch.cuda.synchronize()
    _check(s, hops, s.rows, y, g, TIGHT, f"full size frames, chunks {chunks}")
