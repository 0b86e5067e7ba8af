"""GPU parity of the derivative of the backward pass (filt_backward2, and
double backward through autograd.LFilter) against the oracle's backward2
(pinned by central differences of the oracle's backward, Hessian-vector
products against gradient differences and Hessian symmetry).

y is an input of the backward: both sides get the GPU forward's y, so the
comparison covers filt_backward2 alone.  Tolerance: 2e-6 per channel
(max |err| / max |ref|): every pass it runs keeps FP64 state and sums, so
only FP32 input / output rounding separates it from the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2511_14390_amd import autograd as AG
from paper_2511_14390_amd import filt as F
from paper_2511_14390_amd import workloads as W
from tests.helpers import chan_rel_err, vec_rel_err

pytestmark = pytest.mark.gpu

TOL = 2e-6  # FP64 recursions and sums, FP32 I/O (as the other FP64-state parity tests)
NAMES = ("x", "a", "b", "xi", "yi")


def _case(seed, tv, layout, M, N, T, B=3, hop=1):
    frames = hop > 1
    p = W.random_problem(seed, B=B, T=T, M=0 if M is None else M, N=N, time_varying=tv,
                         layout=layout, hop=hop if frames else 16, rho_max=0.95,
                         with_b=M is not None, frames=frames)
    v = {"x": p.x, "a": p.a if N > 0 else None, "b": p.b if M is not None else None,
         "xi": p.xi if (M is not None and M > 0) else None, "yi": p.yi if N > 0 else None}
    rng = np.random.default_rng(seed + 7)
    cot = {k: (None if t is None else rng.standard_normal(t.shape).astype(np.float32))
           for k, t in v.items()}
    return p, v, cot


def _t(v, dev):
    return None if v is None else torch.from_numpy(np.ascontiguousarray(v)).to(dev)


def _errs(got, ref, tv, layout):
    e = {}
    for k in ("gy", "x", "y"):
        e[k] = chan_rel_err(got[k], ref[k], layout)
    for k in ("a", "b"):
        if k in ref:
            e[k] = (chan_rel_err(got[k], ref[k], layout) if tv
                    else vec_rel_err(got[k], ref[k]))
    for k in ("xi", "yi"):
        if k in ref and ref[k].size:
            e[k] = vec_rel_err(got[k], ref[k])
    return e


def _run(p, v, cot, dev, layout, chunk, hop, want=("gy", "x", "y", "a", "b", "xi", "yi")):
    g = {k: _t(t, dev) for k, t in v.items()}
    c = {k: _t(t, dev) for k, t in cot.items()}
    y = F.filt_forward(g["x"], g["a"], g["b"], g["xi"], g["yi"], layout=layout, chunk=chunk,
                       hop=hop)
    gy = _t(p.gy, dev)
    w = F.filt_backward2(gy, g["x"], y, g["a"], g["b"], g["xi"], g["yi"], vx=c["x"],
                         va=c["a"], vb=c["b"], vxi=c["xi"], vyi=c["yi"], layout=layout,
                         chunk=chunk, hop=hop, want=want)
    torch.cuda.synchronize()
    return y.cpu().numpy(), {k: t.cpu().numpy() for k, t in w.items()}


def _oracle(p, v, cot, y, layout, hop):
    kw = dict(vx=cot["x"], va=cot["a"], vb=cot["b"], vxi=cot["xi"], vyi=cot["yi"],
              layout=layout)
    if hop > 1:
        return oracle.backward2_frames(p.gy, v["x"], y, v["a"], v["b"], v["xi"], v["yi"],
                                       hop=hop, **kw)
    return oracle.backward2(p.gy, v["x"], y, v["a"], v["b"], v["xi"], v["yi"], **kw)


CASES = [
    # (tv, layout, M, N, T, chunk, hop); M None: b = [1]
    (False, "BT", 2, 3, 700, 64, 1),
    (False, "TB", 4, 4, 900, 128, 1),
    (True, "BT", 2, 5, 600, 64, 1),
    (True, "TB", 1, 12, 500, 64, 1),
    (False, "BT", None, 2, 800, 0, 1),
    (True, "TB", 3, 0, 400, 32, 1),
    (True, "BT", 2, 4, 1000, 64, 16),
    (True, "TB", 0, 16, 700, 96, 7),
]


@pytest.mark.parametrize("tv,layout,M,N,T,chunk,hop", CASES)
def test_backward2_matches_oracle(gpu_device, tv, layout, M, N, T, chunk, hop):
    seed = 9100 + 13 * (M or 0) + 5 * N + T + hop
    p, v, cot = _case(seed, tv, layout, M, N, T, hop=hop)
    y, w = _run(p, v, cot, gpu_device, layout, chunk, hop)
    ref = _oracle(p, v, cot, y, layout, hop)
    e = _errs(w, ref, tv, layout)
    print(f"[backward2] seed={seed} tv={tv} {layout} M={M} N={N} T={T} hop={hop} "
          f"errs={ {k: f'{x:.1e}' for k, x in e.items()} }", flush=True)
    assert max(e.values()) <= TOL, e


def test_backward2_cotangent_subsets_and_output_subsets(gpu_device):
    p, v, cot = _case(9300, True, "BT", 2, 3, 500)
    for drop in (("x", "xi"), ("a", "yi"), ("b",), ("a", "b", "yi")):
        c = dict(cot)
        for k in drop:
            c[k] = None
        y, w = _run(p, v, c, gpu_device, "BT", 64, 1)
        ref = _oracle(p, v, c, y, "BT", 1)
        e = _errs(w, ref, True, "BT")
        assert max(e.values()) <= TOL, (drop, e)
    # only some outputs: the others are not computed
    y, w = _run(p, v, cot, gpu_device, "BT", 64, 1, want=("a", "yi"))
    assert set(w) == {"a", "yi"}
    ref = _oracle(p, v, cot, y, "BT", 1)
    assert chan_rel_err(w["a"], ref["a"], "BT") <= TOL
    assert vec_rel_err(w["yi"], ref["yi"]) <= TOL


def test_backward2_empty_signal_zero_fills(gpu_device):
    dev = gpu_device
    x = torch.zeros((3, 0), device=dev)
    a = torch.ones((3, 2), device=dev)
    b = torch.ones((3, 3), device=dev)
    xi = torch.ones((3, 2), device=dev)
    yi = torch.ones((3, 2), device=dev)
    w = F.filt_backward2(x, x, x, a, b, xi, yi, va=a, vb=b, vxi=xi, vyi=yi)
    torch.cuda.synchronize()
    assert w["x"].shape == (3, 0) and w["gy"].shape == (3, 0)
    for k in ("a", "b", "xi", "yi"):
        assert float(w[k].abs().max()) == 0.0, k


@pytest.mark.parametrize("tv,layout", [(False, "BT"), (True, "TB")])
def test_double_backward_through_lfilter(gpu_device, tv, layout):
    # Hessian-vector product of L = <w, y(theta)> by reverse over reverse
    # (torch.autograd.grad with create_graph) against the oracle's: the
    # explicit part from backward2 plus its y part sent back through the
    # filter's backward
    p, v, t = _case(9400 + tv, tv, layout, 2, 4, 600)
    dev = gpu_device
    th = {k: _t(x, dev).requires_grad_(True) for k, x in v.items()}
    y = AG.lfilter(th["x"], th["a"], th["b"], th["xi"], th["yi"], layout=layout)
    wgt = _t(p.gy, dev)
    L = (y * wgt).sum()
    ins = [th[k] for k in NAMES]
    g = torch.autograd.grad(L, ins, create_graph=True)
    s = sum((gi * _t(t[k], dev)).sum() for gi, k in zip(g, NAMES))
    hv = torch.autograd.grad(s, ins)
    torch.cuda.synchronize()
    yv = y.detach().cpu().numpy()
    d = oracle.backward2(p.gy, v["x"], yv, v["a"], v["b"], v["xi"], v["yi"], vx=t["x"],
                         va=t["a"], vb=t["b"], vxi=t["xi"], vyi=t["yi"], layout=layout)
    back = oracle.backward(d["y"], v["x"], yv, v["a"], v["b"], v["xi"], v["yi"], layout=layout)
    for k, h in zip(NAMES, hv):
        ref = d[k] + back[k]
        got = h.cpu().numpy()
        err = (chan_rel_err(got, ref, layout) if k == "x" or (tv and k in ("a", "b"))
               else vec_rel_err(got, ref))
        print(f"[double backward] tv={tv} {layout} {k}: {err:.1e}", flush=True)
        assert err <= TOL, (k, err)


def test_backward2_full_size_df_m4n4_shape(gpu_device):
    # the M = N = 4 time-invariant workload's shape ([T, B] = [65536, 1024]);
    # 6 channels against the oracle
    T, B = 65536, 1024
    p = W.config3()
    rng = np.random.default_rng(9500)
    cot = {"x": rng.standard_normal((T, B)).astype(np.float32),
           "a": rng.standard_normal((B, 4)).astype(np.float32),
           "b": rng.standard_normal((B, 5)).astype(np.float32),
           "xi": rng.standard_normal((B, 4)).astype(np.float32),
           "yi": rng.standard_normal((B, 4)).astype(np.float32)}
    v = {"x": p.x, "a": p.a, "b": p.b, "xi": p.xi, "yi": p.yi}
    y, w = _run(p, v, cot, gpu_device, "TB", 0, 1)
    ch = np.array([0, 1, 333, 512, 900, 1023])
    sub = {k: (t[:, ch] if k == "x" else t[ch]) for k, t in v.items()}
    csub = {k: (t[:, ch] if k == "x" else t[ch]) for k, t in cot.items()}
    ref = oracle.backward2(p.gy[:, ch], sub["x"], y[:, ch], sub["a"], sub["b"], sub["xi"],
                           sub["yi"], vx=csub["x"], va=csub["a"], vb=csub["b"],
                           vxi=csub["xi"], vyi=csub["yi"], layout="TB")
    got = {k: (t[:, ch] if k in ("gy", "x", "y") else t[ch]) for k, t in w.items()}
    e = _errs(got, ref, False, "TB")
    print(f"[backward2] full size: { {k: f'{x:.1e}' for k, x in e.items()} }", flush=True)
    assert max(e.values()) <= TOL, e
