"""GPU parity of cascades of second-order sections (filt_sos_forward /
filt_sos_backward, the autograd SOSFilter) against the oracle's cascade of
state-space transposed-form sections (oracle.sos_forward / sos_backward,
pinned against SciPy's sosfilt).

Tolerances as the other parity tests: outputs 1e-4, gradients 1e-3 (per
channel, max |err| / max |ref|).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2511_14390_amd import autograd as AG
from paper_2511_14390_amd import filt as F
from tests.helpers import chan_rel_err, vec_rel_err

pytestmark = pytest.mark.gpu

OUT_TOL = 1e-4
GRAD_TOL = 1e-3


def _problem(seed, S, B, T, layout, with_zi=True, rmax=0.97):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((S, B, 3)).astype(np.float32)
    r = rng.uniform(0.3, rmax, (S, B))
    th = rng.uniform(0.0, np.pi, (S, B))
    a = np.stack([-2 * r * np.cos(th), r * r], axis=-1).astype(np.float32)
    zi = rng.normal(0.0, 0.3, (S, B, 2)).astype(np.float32) if with_zi else None
    shape = (B, T) if layout == "BT" else (T, B)
    x = rng.standard_normal(shape).astype(np.float32)
    gy = rng.standard_normal(shape).astype(np.float32)
    return x, b, a, zi, gy


def _t(v, dev):
    return None if v is None else torch.from_numpy(np.ascontiguousarray(v)).to(dev)


def _errs(g, go, y, yo, layout):
    out = {"y": chan_rel_err(y, yo, layout), "x": chan_rel_err(g["x"], go["x"], layout)}
    for k in ("b", "a", "zi"):
        if k in g:
            # per section and channel
            out[k] = vec_rel_err(g[k].reshape(-1, g[k].shape[-1]),
                                 go[k].reshape(-1, go[k].shape[-1]))
    return out


@pytest.mark.parametrize("S,layout,T,chunk", [(1, "BT", 1000, 64), (2, "TB", 1500, 0),
                                              (4, "BT", 2500, 128), (6, "TB", 700, 64),
                                              (3, "BT", 5, 0)])
def test_sos_matches_oracle(gpu_device, S, layout, T, chunk):
    seed = 9950 + 10 * S + T
    x, b, a, zi, gy = _problem(seed, S, 3, T, layout)
    dev = gpu_device
    xg, bg, ag, zg, gg = (_t(v, dev) for v in (x, b, a, zi, gy))
    y = F.filt_sos_forward(xg, bg, ag, zg, layout=layout, chunk=chunk)
    g = F.filt_sos_backward(gg, xg, y, bg, ag, zg, layout=layout, chunk=chunk)
    torch.cuda.synchronize()
    yo = oracle.sos_forward(x, b, a, zi, layout)
    go = oracle.sos_backward(gy, x, b, a, zi, layout)
    e = _errs({k: v.cpu().numpy() for k, v in g.items()}, go, y.cpu().numpy(), yo, layout)
    print(f"[sos] seed={seed} S={S} {layout} T={T} chunk={chunk} "
          f"errs={ {k: f'{v:.2e}' for k, v in e.items()} }", flush=True)
    assert e["y"] <= OUT_TOL, e
    assert max(v for k, v in e.items() if k != "y") <= GRAD_TOL, e


def test_sos_zero_states_and_autograd(gpu_device):
    x, b, a, _, gy = _problem(9990, 3, 4, 900, "BT", with_zi=False)
    dev = gpu_device
    xg, bg, ag = (_t(v, dev).requires_grad_(True) for v in (x, b, a))
    y = AG.sosfilt(xg, bg, ag, None)
    y.backward(_t(gy, dev))
    torch.cuda.synchronize()
    go = oracle.sos_backward(gy, x, b, a, None, "BT")
    assert chan_rel_err(y.detach().cpu().numpy(), oracle.sos_forward(x, b, a, None, "BT"),
                        "BT") <= OUT_TOL
    assert chan_rel_err(xg.grad.cpu().numpy(), go["x"], "BT") <= GRAD_TOL
    for t, k in ((bg, "b"), (ag, "a")):
        assert vec_rel_err(t.grad.cpu().numpy().reshape(-1, t.shape[-1]),
                           go[k].reshape(-1, go[k].shape[-1])) <= GRAD_TOL, k


def test_sos_empty_signal(gpu_device):
    dev = gpu_device
    x = torch.zeros((2, 0), device=dev)
    b = torch.ones((3, 2, 3), device=dev)
    a = torch.zeros((3, 2, 2), device=dev)
    zi = torch.ones((3, 2, 2), device=dev)
    y = F.filt_sos_forward(x, b, a, zi)
    g = F.filt_sos_backward(torch.zeros_like(x), x, y, b, a, zi)
    torch.cuda.synchronize()
    assert y.shape == (2, 0)
    for k in ("b", "a", "zi"):
        assert float(g[k].abs().max()) == 0.0, k
