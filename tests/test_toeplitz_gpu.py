"""GPU parity of the matrix-core path for time-invariant [B, T] problems
(opt-in with FILT_TOEPLITZ; the default is the FP64-state recurrence).

Each chunk of 64 samples is one column of an FP32 GEMM with the channel's
[history | Toeplitz | state] matrix; states between chunks are carried in
FP64.  Error budget: every output is an FP32 sum of at most 96 products whose
terms decay with the impulse response, so the per-channel relative error is a
few FP32 ulps times the growth of the response (about 1e-6 here); the tests
hold it to 2e-5 on outputs and gradients, well inside the 1e-4 / 1e-3 bar and
far below the size of any indexing or carry mistake (which is O(1)).
"""
import numpy as np
import pytest
import torch

from paper_2511_14390_amd import filt as F
from paper_2511_14390_amd import workloads as W
from tests.helpers import chan_rel_err
from tests.test_parity_gpu import compare, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

TZ_TOL = 2e-5

TZ_CASES = [
    # (M, N, T, B): ragged tails, exact multiples of the chunk and of the
    # 64-chunk tile, a single partial chunk, M > N, the largest orders
    (0, 1, 1000, 3),
    (0, 2, 4096, 2),
    (0, 4, 64 * 64 * 2 + 37, 2),
    (2, 2, 777, 4),
    (4, 4, 64 * 5, 3),
    (3, 5, 999, 2),
    (6, 3, 1500, 2),
    (16, 16, 2000, 2),
    (0, 16, 64 * 64 + 64, 1),
    (1, 1, 40, 3),
    (5, 2, 63, 2),
    (0, 3, 65, 2),
]


def _lti(M, N, T, B, seed, with_b=True, with_xi=True, with_yi=True):
    return W.random_problem(seed, B=B, T=T, M=M, N=N, time_varying=False, layout="BT",
                            rho_max=0.95, with_b=with_b, with_xi=with_xi, with_yi=with_yi)


@pytest.mark.parametrize("M,N,T,B", TZ_CASES)
def test_toeplitz_matches_oracle(gpu_device, M, N, T, B):
    p = _lti(M, N, T, B, 5000 + 13 * M + 7 * N + T)
    yg, gg = run_gpu(p, gpu_device, toeplitz=True)
    yo, go = run_oracle(p)
    compare(p, yg, gg, yo, go, out_tol=TZ_TOL, grad_tol=TZ_TOL, label="toeplitz")


def test_toeplitz_no_b_no_initial_conditions(gpu_device):
    p = _lti(0, 4, 3000, 3, 5101, with_b=False, with_xi=False, with_yi=False)
    yg, gg = run_gpu(p, gpu_device, want=("x", "a", "yi"), toeplitz=True)
    yo, go = run_oracle(p)
    compare(p, yg, gg, yo, go, out_tol=TZ_TOL, grad_tol=TZ_TOL, label="toeplitz no-b")


@pytest.mark.parametrize("want", [("x",), ("a",), ("b",), ("yi",), ("xi",), ("a", "xi")])
def test_toeplitz_gradient_subsets(gpu_device, want):
    p = _lti(3, 4, 2500, 2, 5202)
    yg, gg = run_gpu(p, gpu_device, want=want, toeplitz=True)
    yo, go = run_oracle(p)
    assert set(gg) == set(want)
    compare(p, yg, gg, yo, {k: go[k] for k in gg}, out_tol=TZ_TOL, grad_tol=TZ_TOL,
            label=f"toeplitz want={want}")


def test_toeplitz_agrees_with_recurrence(gpu_device):
    p = _lti(2, 6, 20000, 4, 5303)
    y1, g1 = run_gpu(p, gpu_device, toeplitz=True)
    y2, g2 = run_gpu(p, gpu_device, recurrence=True)
    assert chan_rel_err(y1, y2, "BT") <= TZ_TOL
    for k in g1:
        ref = g2[k]
        err = np.abs(g1[k] - ref).max() / max(np.abs(ref).max(), 1e-30)
        assert err <= TZ_TOL, (k, err)


def test_auto_chunk_reports_the_tile_chunk():
    x = torch.zeros(2, 1000)
    a = torch.zeros(2, 4)
    assert F.auto_chunk(F.problem(x, a, None, "BT", toeplitz=True)) == 64
    assert F.auto_chunk(F.problem(x, a, None, "BT")) != 0


def test_toeplitz_long_signal_many_carry_groups(gpu_device):
    # more than 256 x 256 chunk steps: the tile pass of the time-invariant
    # carry walks two groups of tiles
    p = _lti(0, 4, (1 << 22) + 64 * 300 + 5, 1, 5404)
    yg, gg = run_gpu(p, gpu_device, want=("x", "a", "yi"), toeplitz=True)
    yo, go = run_oracle(p)
    compare(p, yg, gg, yo, go, out_tol=TZ_TOL, grad_tol=TZ_TOL, label="toeplitz long")


def test_long_narrow_domain_error_distribution(gpu_device):
    # config 4's domain (two pole pairs with radius U[0.9, 0.99]) over 12
    # seeds.  The default path (FP64-state recurrence) is held to the stated
    # 1e-4 (outputs) / 1e-3 (gradients) on every draw.  The opt-in matrix-core
    # path's per-draw errors are printed as a distribution: its FP32 sums let
    # the entering state's response cancel, and one draw in twelve exceeds
    # 1e-4 (4.7e-4 measured), which is why it is not the default; it is held
    # to 1e-3 here so that a regression still shows.
    dist = {"default": [], "toeplitz": []}
    for seed in range(12):
        p = W.config4(B=2, T=1 << 20, seed=9000 + seed)
        yo, go = run_oracle(p, nthreads=2)
        go = {k: go[k] for k in ("x", "a")}
        yg, gg = run_gpu(p, gpu_device, want=("x", "a"))
        dist["default"].append(compare(p, yg, gg, yo, go, label=f"config4-domain seed={9000 + seed}"))
        yt, gt = run_gpu(p, gpu_device, want=("x", "a"), toeplitz=True)
        dist["toeplitz"].append(compare(p, yt, gt, yo, go, out_tol=1e-3, grad_tol=1e-3,
                                        label=f"config4-domain toeplitz seed={9000 + seed}"))
    for path, errs in dist.items():
        for k in errs[0]:
            v = np.array([e[k] for e in errs])
            print(f"[tz-dist] {path} {k}: min {v.min():.2e} median {np.median(v):.2e} "
                  f"max {v.max():.2e} draws above 1e-4: {int((v > 1e-4).sum())}", flush=True)
