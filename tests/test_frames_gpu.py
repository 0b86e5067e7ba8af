"""GPU parity of frame-held coefficients (time_varying = hop >= 2): the HIP
path through the C ABI against the oracle on the frame-expanded inputs, with
the coefficient gradients reduced per frame (oracle.forward_frames /
oracle.backward_frames).

Tolerances as the other parity tests: outputs 1e-4, gradients 1e-3 (per
channel, max |err| / max |ref|); FP64 entry points 1e-9.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2511_14390_amd import filt as F
from paper_2511_14390_amd import workloads as W
from tests.test_parity_gpu import GRAD_TOL, OUT_TOL, _dev, compare

pytestmark = pytest.mark.gpu


def run_frames_gpu(p, hop, dev, chunk=0, dtype=torch.float32, want=("x", "a", "b", "xi", "yi")):
    t = lambda v: _dev(v, dev, dtype)
    x, a, b, xi, yi, gy = map(t, (p.x, p.a, p.b, p.xi, p.yi, p.gy))
    y = F.filt_forward(x, a, b, xi, yi, layout=p.layout, chunk=chunk, hop=hop)
    g = F.filt_backward(gy, x, y, a, b, xi, yi, layout=p.layout, chunk=chunk, hop=hop,
                        want=want)
    torch.cuda.synchronize()
    return y.cpu().numpy(), {k: v.cpu().numpy() for k, v in g.items()}


def run_frames_oracle(p, hop, nthreads=8):
    y = oracle.forward_frames(p.x, p.a, p.b, p.xi, p.yi, hop=hop, layout=p.layout,
                              nthreads=nthreads)
    g = oracle.backward_frames(p.gy, p.x, y, p.a, p.b, p.xi, p.yi, hop=hop, layout=p.layout,
                               nthreads=nthreads)
    return y, g


CASES = [
    # (M, N, layout, T, hop, chunk): frame edges inside chunks, chunk edges
    # inside frames, ragged last frames and chunks, hop above T
    (0, 2, "BT", 1000, 7, 64),
    (2, 3, "TB", 901, 5, 64),
    (4, 4, "BT", 1234, 128, 160),
    (0, 8, "TB", 1111, 100, 96),
    (0, 16, "BT", 2500, 240, 128),
    (1, 16, "TB", 700, 33, 64),
    (16, 16, "BT", 640, 64, 64),
    (0, 16, "TB", 2000, 240, 256),
    (0, 1, "BT", 3000, 128, 0),
    (0, 4, "BT", 5000, 128, 0),
    (3, 5, "TB", 999, 1000, 64),
    (2, 2, "BT", 500, 2, 32),
    (0, 12, "TB", 1500, 96, 0),
    (5, 0, "BT", 400, 16, 64),
]


@pytest.mark.parametrize("M,N,layout,T,hop,chunk", CASES)
def test_frames_match_oracle(M, N, layout, T, hop, chunk):
    dev = torch.device("cuda:0")
    seed = 9100 + 7 * M + 3 * N + T + hop
    p = W.random_problem(seed, B=3, T=T, M=M, N=N, time_varying=True, layout=layout, hop=hop,
                         rho_max=0.97, frames=True)
    print(f"[frames] seed={seed} M={M} N={N} layout={layout} T={T} hop={hop} chunk={chunk}",
          flush=True)
    yg, gg = run_frames_gpu(p, hop, dev, chunk=chunk)
    yo, go = run_frames_oracle(p, hop)
    assert gg["a"].shape == p.a.shape if N > 0 else True
    compare(p, yg, gg, yo, go, label=f"frames hop={hop} chunk={chunk}")


@pytest.mark.parametrize("layout", ["TB", "BT"])
def test_frames_fp64_entry_points(layout):
    dev = torch.device("cuda:0")
    p = W.random_problem(9200 + (layout == "TB"), B=2, T=700, M=2, N=5, time_varying=True,
                         layout=layout, hop=37, frames=True)
    yg, gg = run_frames_gpu(p, 37, dev, chunk=64, dtype=torch.float64)
    yo, go = run_frames_oracle(p, 37)
    compare(p, yg, gg, yo, go, out_tol=1e-9, grad_tol=1e-9, label="frames f64")


@pytest.mark.parametrize("want", [("a",), ("b",), ("x", "yi"), ("a", "b", "xi")])
def test_frames_gradient_subsets(want):
    dev = torch.device("cuda:0")
    p = W.random_problem(9300, B=2, T=900, M=3, N=4, time_varying=True, layout="TB", hop=50,
                         frames=True)
    yg, gg = run_frames_gpu(p, 50, dev, chunk=96, want=want)
    yo, go = run_frames_oracle(p, 50)
    assert set(gg) == {k for k in want if k in go}
    compare(p, yg, gg, yo, {k: go[k] for k in gg}, label=f"frames want={want}")


@pytest.mark.parametrize("layout", ["TB", "BT"])
def test_frames_lpc_workload_full_size(layout):
    # 64 channels x 48000 samples, order 16, coefficients held over frames of
    # 240 samples (200 frame rows per channel), in the bench's layout and the
    # other one; every channel against the oracle
    dev = torch.device("cuda:0")
    p = W.config2(frames=True)
    if layout == "TB":
        sw = lambda v: np.ascontiguousarray(np.swapaxes(v, 0, 1))
        p = W.Problem(p.name, "TB", sw(p.x), sw(p.a), None, None, None, sw(p.gy), dict(p.meta))
    print(f"[frames] lpc full size layout={layout}", flush=True)
    yg, gg = run_frames_gpu(p, 240, dev)
    yo, go = run_frames_oracle(p, 240, nthreads=16)
    compare(p, yg, gg, yo, go, label="frames lpc full")


def test_frames_agree_with_expanded_per_sample_rows():
    # the same filter given as frame rows (hop 128) and as per-sample rows
    dev = torch.device("cuda:0")
    p = W.random_problem(9400, B=4, T=3000, M=0, N=6, time_varying=True, layout="BT", hop=128,
                         with_b=False, frames=True)
    yf, gf = run_frames_gpu(p, 128, dev, chunk=256)
    a_s = oracle.frame_expand(p.a, p.T, 128, "BT").astype(np.float32)
    q = W.Problem(p.name, "BT", p.x, a_s, None, None, p.yi, p.gy, dict(p.meta))
    t = lambda v: _dev(v, dev)
    x, a, yi, gy = map(t, (q.x, q.a, q.yi, q.gy))
    y = F.filt_forward(x, a, None, None, yi, layout="BT", chunk=256)
    g = F.filt_backward(gy, x, y, a, None, None, yi, layout="BT", chunk=256)
    np.testing.assert_allclose(yf, y.cpu().numpy(), rtol=0, atol=1e-5 * np.abs(yf).max())
    ga = oracle.frame_reduce(g["a"].cpu().numpy(), 128, "BT")
    np.testing.assert_allclose(gf["a"], ga, rtol=0, atol=1e-4 * np.abs(ga).max())


def test_frames_empty_signal():
    dev = torch.device("cuda:0")
    x = torch.zeros((3, 0), device=dev)
    a = torch.zeros((3, 0, 2), device=dev)
    yi = torch.ones((3, 2), device=dev)
    y = F.filt_forward(x, a, None, None, yi, layout="BT", hop=16)
    g = F.filt_backward(torch.zeros_like(x), x, y, a, None, None, yi, layout="BT", hop=16)
    torch.cuda.synchronize()
    assert y.shape == (3, 0) and g["a"].shape == (3, 0, 2)
    assert float(g["yi"].abs().max()) == 0.0


def test_frames_jvp_matches_oracle_directional_difference():
    dev = torch.device("cuda:0")
    hop = 20
    p = W.random_problem(9500, B=2, T=600, M=2, N=4, time_varying=True, layout="BT", hop=hop,
                         frames=True)
    rng = np.random.default_rng(9501)
    da = (0.01 * rng.standard_normal(p.a.shape)).astype(np.float32)
    db = (0.1 * rng.standard_normal(p.b.shape)).astype(np.float32)
    t = lambda v: _dev(v, dev)
    x, a, b, xi, yi = map(t, (p.x, p.a, p.b, p.xi, p.yi))
    y = F.filt_forward(x, a, b, xi, yi, layout="BT", hop=hop)
    dy = F.filt_jvp(x, y, a, b, xi, yi, da=t(da), db=t(db), layout="BT", hop=hop)
    torch.cuda.synchronize()
    eps = 1e-6
    f = lambda s: oracle.forward_frames(p.x, p.a.astype(np.float64) + s * da,
                                        p.b.astype(np.float64) + s * db, p.xi, p.yi, hop=hop,
                                        layout="BT")
    ref = (f(eps) - f(-eps)) / (2 * eps)
    err = np.abs(dy.cpu().numpy() - ref).max() / np.abs(ref).max()
    print(f"[frames] jvp rel err {err:.2e}", flush=True)
    assert err <= GRAD_TOL
