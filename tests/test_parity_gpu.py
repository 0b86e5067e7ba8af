"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (per channel, max |err| / max |ref|): outputs 1e-4, gradients
1e-3 (per-sample gradients per channel; per-channel coefficient and
initial-condition gradients per row).  Inputs are the seeded synthetic
workloads of ``paper_2511_14390_amd.workloads``.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2511_14390_amd import filt as F
from paper_2511_14390_amd import workloads as W
from tests.helpers import chan_rel_err, vec_rel_err

pytestmark = pytest.mark.gpu

OUT_TOL = 1e-4
GRAD_TOL = 1e-3


def _dev(v, dev, dtype=torch.float32):
    return None if v is None else torch.from_numpy(np.ascontiguousarray(v)).to(dev, dtype)


def run_gpu(p, dev, chunk=0, f32_state=False, dtype=torch.float32,
            want=("x", "a", "b", "xi", "yi"), recurrence=False):
    t = lambda v: _dev(v, dev, dtype)
    x, a, b, xi, yi, gy = map(t, (p.x, p.a, p.b, p.xi, p.yi, p.gy))
    y = F.filt_forward(x, a, b, xi, yi, layout=p.layout, chunk=chunk, f32_state=f32_state,
                       recurrence=recurrence)
    g = F.filt_backward(gy, x, y, a, b, xi, yi, layout=p.layout, chunk=chunk,
                        f32_state=f32_state, recurrence=recurrence, want=want)
    torch.cuda.synchronize()
    return y.cpu().numpy(), {k: v.cpu().numpy() for k, v in g.items()}


def run_oracle(p, nthreads=8):
    y = oracle.forward(p.x, p.a, p.b, p.xi, p.yi, layout=p.layout, nthreads=nthreads)
    g = oracle.backward(p.gy, p.x, y, p.a, p.b, p.xi, p.yi, layout=p.layout, nthreads=nthreads)
    return y, g


def compare(p, yg, gg, yo, go, out_tol=OUT_TOL, grad_tol=GRAD_TOL, label=""):
    errs = {"y": chan_rel_err(yg, yo, p.layout)}
    for k, v in gg.items():
        ref = go[k]
        if k == "x" or (k in ("a", "b") and p.time_varying):
            errs[k] = chan_rel_err(v, ref, p.layout)
        else:
            errs[k] = vec_rel_err(v, ref)
    print(f"[parity] {label} {p.name} B={p.B} T={p.T} M={p.M} N={p.N} tv={p.time_varying} "
          f"layout={p.layout} errs={ {k: f'{e:.2e}' for k, e in errs.items()} }", flush=True)
    assert errs["y"] <= out_tol, errs
    for k, e in errs.items():
        if k != "y":
            assert e <= grad_tol, (k, errs)
    return errs


CASES = [
    # (M, N, tv, layout, T, chunk)
    (0, 1, False, "BT", 1000, 64),
    (0, 2, False, "TB", 1000, 32),
    (2, 2, False, "BT", 777, 64),
    (4, 4, False, "TB", 1500, 128),
    (3, 5, False, "BT", 999, 96),
    (0, 16, False, "BT", 2000, 256),
    (0, 2, True, "BT", 1000, 64),
    (2, 3, True, "TB", 901, 64),
    (4, 4, True, "BT", 1234, 160),
    (0, 8, True, "TB", 1111, 96),
    (0, 16, True, "BT", 2500, 128),
    (1, 16, True, "TB", 700, 64),
    (16, 16, True, "BT", 640, 64),
    (0, 12, True, "TB", 1000, 96),
    (2, 13, True, "BT", 845, 64),
    (16, 2, False, "TB", 500, 32),
    (5, 0, False, "BT", 400, 64),
    (3, 0, True, "TB", 300, 32),
]


def _case(M, N, tv, layout, T):
    # frame-held per-sample coefficients switch every `hop` samples; long frames
    # and a lower pole radius for high orders keep the time-varying system well
    # conditioned (the FP32 tolerance applies to stable, well-conditioned filters)
    hop = 64 if N < 8 else 128
    rho = 0.95 if N < 8 else 0.9
    return W.random_problem(1000 + 31 * M + 7 * N + T, B=5, T=T, M=M, N=N, time_varying=tv,
                            layout=layout, hop=hop, rho_max=rho)


@pytest.mark.parametrize("M,N,tv,layout,T,chunk", CASES)
def test_random_problems_several_chunks_ragged_tail(gpu_device, M, N, tv, layout, T, chunk):
    # FP64 state with FP32 I/O (the per-lane recurrence, also for time-invariant
    # [B, T] problems): only the final FP32 rounding differs from the oracle, so
    # any algorithmic slip (wrong carry, index or boundary) shows up well above
    # this tolerance
    p = _case(M, N, tv, layout, T)
    yg, gg = run_gpu(p, gpu_device, chunk=chunk, recurrence=True)
    yo, go = run_oracle(p)
    compare(p, yg, gg, yo, go, out_tol=2e-6, grad_tol=2e-6, label=f"chunk={chunk}")


@pytest.mark.parametrize("M,N,tv,layout,T,chunk", CASES)
def test_random_problems_fp32_state(gpu_device, M, N, tv, layout, T, chunk):
    # opt-in FP32 state: 1e-4 on outputs, 1e-3 on gradients, on well-conditioned filters
    p = _case(M, N, tv, layout, T)
    yg, gg = run_gpu(p, gpu_device, chunk=chunk, f32_state=True)
    yo, go = run_oracle(p)
    compare(p, yg, gg, yo, go, label=f"f32state chunk={chunk}")


@pytest.mark.parametrize("T", [1, 2, 5, 31, 32, 33, 95])
def test_short_signals(gpu_device, T):
    p = W.random_problem(2000 + T, B=3, T=T, M=3, N=5, time_varying=True, layout="BT", hop=4)
    yg, gg = run_gpu(p, gpu_device, chunk=32)
    yo, go = run_oracle(p)
    compare(p, yg, gg, yo, go, label="short")


def test_no_b_no_initial_conditions(gpu_device):
    p = W.random_problem(3001, B=4, T=600, M=0, N=4, time_varying=True, layout="TB",
                         with_b=False, with_yi=False)
    yg, gg = run_gpu(p, gpu_device, chunk=64)
    yo, go = run_oracle(p)
    compare(p, yg, gg, yo, go, label="no-b")


def test_chunk_length_invariance(gpu_device):
    p = W.random_problem(3002, B=6, T=3000, M=2, N=6, time_varying=True, layout="BT")
    ref_y, ref_g = run_gpu(p, gpu_device, chunk=32)
    for chunk in (64, 160, 512, 4096):
        y, g = run_gpu(p, gpu_device, chunk=chunk)
        assert chan_rel_err(y, ref_y, "BT") <= 1e-5
        for k in g:
            assert chan_rel_err(g[k], ref_g[k], "BT") <= 1e-4, k


@pytest.mark.parametrize("M,N,layout,T,chunk", [(3, 4, "TB", 120000, 32), (0, 9, "BT", 50000, 32),
                                                (2, 16, "BT", 40000, 64)])
def test_time_invariant_carry_over_many_tiles(gpu_device, M, N, layout, T, chunk):
    # more than 256 chunk steps: the log-depth time-invariant carry sums
    # 256-step tiles, scans the tiles and refills them (with the FIR adjoint
    # state for M > 0), on the FP64-state recurrence path
    p = W.random_problem(3100 + N, B=3, T=T, M=M, N=N, time_varying=False, layout=layout,
                         rho_max=0.95)
    yg, gg = run_gpu(p, gpu_device, chunk=chunk, recurrence=True)
    yo, go = run_oracle(p)
    compare(p, yg, gg, yo, go, out_tol=2e-6, grad_tol=2e-6, label=f"lti-tiles chunk={chunk}")


def test_config1_full(gpu_device):
    p = W.config1()
    yg, gg = run_gpu(p, gpu_device, want=("x", "a", "yi"))
    yo, go = run_oracle(p)
    compare(p, yg, gg, yo, go, label="config1")


def test_config2_reduced(gpu_device):
    p = W.config2(B=8, T=4800)
    yg, gg = run_gpu(p, gpu_device, want=("x", "a", "yi"))
    yo, go = run_oracle(p)
    compare(p, yg, gg, yo, go, label="config2-reduced")


def test_config2_full(gpu_device):
    p = W.config2()
    yg, gg = run_gpu(p, gpu_device, want=("x", "a"))
    yo, go = run_oracle(p)
    compare(p, yg, gg, yo, go, label="config2")


def test_config3_reduced(gpu_device):
    p = W.config3(B=64, T=8192)
    yg, gg = run_gpu(p, gpu_device)
    yo, go = run_oracle(p)
    compare(p, yg, gg, yo, go, label="config3-reduced")


def test_config3_full(gpu_device):
    p = W.config3()
    yg, gg = run_gpu(p, gpu_device)
    yo, go = run_oracle(p)
    compare(p, yg, gg, yo, go, label="config3")


def test_config4_full(gpu_device):
    p = W.config4()
    yg, gg = run_gpu(p, gpu_device, want=("x", "a"))
    yo, go = run_oracle(p)
    compare(p, yg, gg, yo, go, label="config4")


def test_fp64_io_path_matches_oracle_tightly(gpu_device):
    p = W.random_problem(4001, B=3, T=700, M=2, N=3, time_varying=True, layout="BT")
    yg, gg = run_gpu(p, gpu_device, dtype=torch.float64, chunk=64)
    yo, go = run_oracle(p)
    compare(p, yg, gg, yo, go, out_tol=1e-10, grad_tol=1e-9, label="f64")
