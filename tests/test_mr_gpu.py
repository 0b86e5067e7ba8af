"""GPU parity of the matrix recurrence v(n+1) = A v(n) + z(n) (the operator
of App. B: filt_mr_forward / filt_mr_backward and the autograd
MatrixRecurrence) against the oracle's mr_forward / mr_backward (pinned by
matrix powers, the first-order direct form, SciPy and finite differences).

Tolerance 2e-6 per channel (max |err| / max |ref|): the state and the gA
sums run in FP64, only FP32 input / output rounding separates the two.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2511_14390_amd import autograd as AG
from paper_2511_14390_amd import filt as F
from tests.helpers import chan_rel_err, vec_rel_err

pytestmark = pytest.mark.gpu

TOL = 2e-6


def _problem(seed, B, T, K, layout, rho=0.95, with_v0=True):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((B, K, K))
    for b in range(B):
        A[b] *= rho / max(np.abs(np.linalg.eigvals(A[b])).max(), 1e-3)
    shape = (B, T, K) if layout == "BT" else (T, B, K)
    v0 = rng.standard_normal((B, K)).astype(np.float32) if with_v0 else None
    return (A.astype(np.float32), v0, rng.standard_normal(shape).astype(np.float32),
            rng.standard_normal(shape).astype(np.float32))


def _t(v, dev):
    return None if v is None else torch.from_numpy(np.ascontiguousarray(v)).to(dev)


def _chan_err(got, ref, layout):
    # per channel over (time, state component)
    g = got if layout == "BT" else got.transpose(1, 0, 2)
    r = ref if layout == "BT" else ref.transpose(1, 0, 2)
    return chan_rel_err(g.reshape(g.shape[0], -1), r.reshape(r.shape[0], -1), "BT")


def _check(A, v0, z, gv, layout, chunk, dev, label):
    Ag, v0g, zg, gvg = (_t(x, dev) for x in (A, v0, z, gv))
    v = F.filt_mr_forward(Ag, zg, v0g, layout=layout, chunk=chunk)
    g = F.filt_mr_backward(gvg, Ag, v, v0g, layout=layout, chunk=chunk)
    torch.cuda.synchronize()
    vn = v.cpu().numpy()
    vo = oracle.mr_forward(A, v0, z, layout=layout)
    # the backward against the oracle's on the GPU's own forward output
    go = oracle.mr_backward(gv, A, v0, vn, layout=layout)
    e = {"v": _chan_err(vn, vo, layout), "z": _chan_err(g["z"].cpu().numpy(), go["z"], layout),
         "A": vec_rel_err(g["A"].cpu().numpy(), go["A"])}
    if v0 is not None:
        e["v0"] = vec_rel_err(g["v0"].cpu().numpy(), go["v0"])
    print(f"[mr] {label} errs={ {k: f'{x:.1e}' for k, x in e.items()} }", flush=True)
    assert max(e.values()) <= TOL, e


CASES = [
    # (K, layout, T, chunk)
    (1, "BT", 1000, 64),
    (3, "TB", 1500, 128),
    (4, "BT", 777, 32),
    (5, "TB", 2000, 0),
    (8, "BT", 1234, 96),
    (12, "TB", 900, 64),
    (16, "BT", 2100, 128),
    (16, "TB", 600, 0),
]


@pytest.mark.parametrize("K,layout,T,chunk", CASES)
def test_mr_matches_oracle(gpu_device, K, layout, T, chunk):
    seed = 9700 + 11 * K + T
    A, v0, z, gv = _problem(seed, 3, T, K, layout)
    _check(A, v0, z, gv, layout, chunk, gpu_device, f"seed={seed} K={K} {layout} T={T} "
                                                    f"chunk={chunk}")


def test_mr_zero_state_short_and_single_chunk(gpu_device):
    A, _, z, gv = _problem(9800, 2, 700, 6, "BT", with_v0=False)
    _check(A, None, z, gv, "BT", 64, gpu_device, "no v0")
    for T in (1, 2, 31, 33):
        A, v0, z, gv = _problem(9810 + T, 2, T, 5, "TB")
        _check(A, v0, z, gv, "TB", 32, gpu_device, f"T={T}")


def test_mr_empty_signal_zero_fills(gpu_device):
    dev = gpu_device
    A = torch.ones((2, 3, 3), device=dev)
    v0 = torch.ones((2, 3), device=dev)
    z = torch.zeros((2, 0, 3), device=dev)
    v = F.filt_mr_forward(A, z, v0)
    g = F.filt_mr_backward(z, A, v, v0)
    torch.cuda.synchronize()
    assert v.shape == (2, 0, 3)
    assert float(g["A"].abs().max()) == 0.0 and float(g["v0"].abs().max()) == 0.0


def test_mr_autograd_matches_oracle(gpu_device):
    A, v0, z, gv = _problem(9900, 4, 800, 7, "TB")
    dev = gpu_device
    Ag, v0g, zg = (_t(x, dev).requires_grad_(True) for x in (A, v0, z))
    v = AG.matrix_recurrence(Ag, zg, v0g, layout="TB")
    v.backward(_t(gv, dev))
    torch.cuda.synchronize()
    vn = v.detach().cpu().numpy()
    go = oracle.mr_backward(gv, A, v0, vn, layout="TB")
    assert _chan_err(vn, oracle.mr_forward(A, v0, z, layout="TB"), "TB") <= TOL
    assert _chan_err(zg.grad.cpu().numpy(), go["z"], "TB") <= TOL
    assert vec_rel_err(Ag.grad.cpu().numpy(), go["A"]) <= TOL
    assert vec_rel_err(v0g.grad.cpu().numpy(), go["v0"]) <= TOL


def test_mr_order16_long_signal(gpu_device):
    # 64 channels of 48000 steps with a 16-dimensional state (the LPC
    # workload's channel count and length); 3 channels against the oracle
    B, T, K = 64, 48000, 16
    A, v0, z, gv = _problem(9950, B, T, K, "BT", rho=0.98)
    dev = gpu_device
    Ag, v0g, zg, gvg = (_t(x, dev) for x in (A, v0, z, gv))
    v = F.filt_mr_forward(Ag, zg, v0g, layout="BT")
    g = F.filt_mr_backward(gvg, Ag, v, v0g, layout="BT")
    torch.cuda.synchronize()
    ch = [0, 31, 63]
    vn = v.cpu().numpy()[ch]
    vo = oracle.mr_forward(A[ch], v0[ch], z[ch])
    go = oracle.mr_backward(gv[ch], A[ch], v0[ch], vn)
    e = {"v": _chan_err(vn, vo, "BT"), "z": _chan_err(g["z"].cpu().numpy()[ch], go["z"], "BT"),
         "A": vec_rel_err(g["A"].cpu().numpy()[ch], go["A"]),
         "v0": vec_rel_err(g["v0"].cpu().numpy()[ch], go["v0"])}
    print(f"[mr] 64 x 48000 K=16: { {k: f'{x:.1e}' for k, x in e.items()} }", flush=True)
    assert max(e.values()) <= TOL, e
