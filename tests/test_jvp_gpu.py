"""GPU tests of the forward-mode derivative (filt_jvp and forward-mode AD
through autograd.LFilter), against the FP64 oracle:

* the pairing identity <dy, gy> = sum over inputs of <grad, tangent>, with
  the oracle's (pinned) backward giving the gradients;
* the oracle's own directional derivative by central differences in FP64;
* forward-mode AD through LFilter gives filt_jvp's result exactly.
"""
import numpy as np
import pytest
import torch
import torch.autograd.forward_ad as fwAD

import oracle
from paper_2511_14390_amd import autograd as AG
from paper_2511_14390_amd import filt as F
from paper_2511_14390_amd import workloads as W
from tests.helpers import chan_rel_err

pytestmark = pytest.mark.gpu

NAMES = ("x", "a", "b", "xi", "yi")


def _case(seed, tv, layout, M=2, N=5, T=700, B=4):
    p = W.random_problem(seed, B=B, T=T, M=M, N=N, time_varying=tv, layout=layout, hop=16,
                         rho_max=0.95)
    rng = np.random.default_rng(seed + 1)
    vals = dict(zip(NAMES, (p.x, p.a, p.b, p.xi, p.yi)))
    tang = {k: (None if v is None else rng.standard_normal(v.shape).astype(np.float32))
            for k, v in vals.items()}
    return p, vals, tang


def _gpu_jvp(p, vals, tang, dev):
    t = lambda v: None if v is None else torch.from_numpy(np.ascontiguousarray(v)).to(dev)
    x, a, b, xi, yi = (t(vals[k]) for k in NAMES)
    y = F.filt_forward(x, a, b, xi, yi, layout=p.layout)
    dy = F.filt_jvp(x, y, a, b, xi, yi, dx=t(tang["x"]), db=t(tang["b"]), da=t(tang["a"]),
                    dxi=t(tang["xi"]), dyi=t(tang["yi"]), layout=p.layout)
    torch.cuda.synchronize()
    return dy.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("tv,layout", [(False, "BT"), (False, "TB"), (True, "BT"), (True, "TB")])
def test_jvp_pairs_with_oracle_gradients(gpu_device, tv, layout):
    p, vals, tang = _case(7600 + 2 * tv + (layout == "TB"), tv, layout)
    dy = _gpu_jvp(p, vals, tang, gpu_device)
    yo = oracle.forward(p.x, p.a, p.b, p.xi, p.yi, layout=layout)
    go = oracle.backward(p.gy, p.x, yo, p.a, p.b, p.xi, p.yi, layout=layout)
    lhs = float((dy * p.gy).sum())
    terms = [(go[k] * tang[k].astype(np.float64)).sum() for k in NAMES if tang[k] is not None]
    rhs = float(sum(terms))
    scale = float(np.abs(dy * p.gy).sum())
    print(f"[jvp] tv={tv} {layout}: <dy,gy>={lhs:.6e} pairing={rhs:.6e}", flush=True)
    assert abs(lhs - rhs) <= 1e-5 * scale


@pytest.mark.parametrize("tv,layout", [(False, "BT"), (True, "TB")])
def test_jvp_matches_oracle_central_differences(gpu_device, tv, layout):
    p, vals, tang = _case(7700 + tv, tv, layout, T=300, B=3)
    dy = _gpu_jvp(p, vals, tang, gpu_device)
    eps = 1e-6
    f64 = lambda v: None if v is None else v.astype(np.float64)

    def fwd(sign):
        v = {k: None if vals[k] is None else f64(vals[k]) + sign * eps * f64(tang[k])
             for k in NAMES}
        return oracle.forward(v["x"], v["a"], v["b"], v["xi"], v["yi"], layout=layout)

    fd = (fwd(+1) - fwd(-1)) / (2 * eps)
    err = chan_rel_err(dy, fd, layout)
    print(f"[jvp] central differences tv={tv} {layout}: rel err {err:.2e}", flush=True)
    assert err <= 1e-4


@pytest.mark.parametrize("tv,layout", [(False, "BT"), (True, "TB")])
def test_forward_mode_ad_through_lfilter(gpu_device, tv, layout):
    p, vals, tang = _case(7800 + tv, tv, layout, T=500)
    t = lambda v: None if v is None else torch.from_numpy(np.ascontiguousarray(v)).to(gpu_device)
    primals = [t(vals[k]) for k in NAMES]
    tangents = [t(tang[k]) for k in NAMES]
    with fwAD.dual_level():
        dual = [fwAD.make_dual(pv, tv_) for pv, tv_ in zip(primals, tangents)]
        out = AG.lfilter(*dual, layout=layout)
        dy = fwAD.unpack_dual(out).tangent
    torch.cuda.synchronize()
    ref = _gpu_jvp(p, vals, tang, gpu_device)
    assert np.array_equal(dy.cpu().numpy().astype(np.float64), ref)


def test_jvp_single_tangents_and_all_pole(gpu_device):
    # each tangent alone (the others NULL), on an all-pole per-sample filter
    p, vals, tang = _case(7900, True, "BT", M=0, N=4, T=400)
    vals["b"] = None
    tang["b"] = None
    tang["xi"] = None
    yo = oracle.forward(p.x, p.a, None, None, p.yi, layout="BT")
    go = oracle.backward(p.gy, p.x, yo, p.a, None, None, p.yi, layout="BT")
    for k in ("x", "a", "yi"):
        only = {n: (tang[n] if n == k else None) for n in NAMES}
        dy = _gpu_jvp(p, vals, only, gpu_device)
        lhs = float((dy * p.gy).sum())
        rhs = float((go[k] * only[k].astype(np.float64)).sum())
        assert abs(lhs - rhs) <= 1e-5 * float(np.abs(dy * p.gy).sum()), k
