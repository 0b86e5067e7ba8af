"""Pins of the oracle's forward-mode derivative (oracle.jvp) and of the
derivative of its backward pass (oracle.backward2, backward2_frames) -- the
second-order use the paper's closing remarks name.

* jvp against central differences of the (pinned) forward, and paired with
  the (pinned) backward: <gy, jvp(t)> = sum_k <backward(gy)_k, t_k>;
* backward2 against central differences of Q = sum_k <v_k, backward()_k>
  in every input, y taken as an input of its own, for time-invariant,
  per-sample and frame-held coefficients, with and without b and with N = 0;
* the Hessian-vector product of L = <w, forward(theta)> composed from
  backward2 and the backward (the y path) against differences of the
  gradient, and the symmetry <s, H t> = <t, H s>.
"""
import numpy as np
import pytest

import oracle

NAMES = ("x", "a", "b", "xi", "yi")


def _problem(seed, tv, layout, M=2, N=3, T=9, B=2, hop=None):
    rng = np.random.default_rng(seed)
    R = T if hop is None else -(-T // hop)

    def coef(K):
        if K is None:
            return None
        if not tv:
            return 0.3 * rng.standard_normal((B, K))
        return 0.3 * rng.standard_normal((R, B, K) if layout == "TB" else (B, R, K))

    sig = (B, T) if layout == "BT" else (T, B)
    v = {"x": rng.standard_normal(sig), "a": coef(N) if N > 0 else None,
         "b": coef(M + 1) if M is not None else None,
         "xi": rng.standard_normal((B, M)) if M is not None and M > 0 else None,
         "yi": rng.standard_normal((B, N)) if N > 0 else None}
    return v, rng.standard_normal(sig), rng


def _like(rng, v):
    return {k: (None if t is None else rng.standard_normal(t.shape)) for k, t in v.items()}


def _fwd(v, layout, hop=None):
    if hop is None:
        return oracle.forward(v["x"], v["a"], v["b"], v["xi"], v["yi"], layout=layout)
    return oracle.forward_frames(v["x"], v["a"], v["b"], v["xi"], v["yi"], hop=hop,
                                 layout=layout)


def _bwd(gy, y, v, layout, hop=None):
    if hop is None:
        return oracle.backward(gy, v["x"], y, v["a"], v["b"], v["xi"], v["yi"], layout=layout)
    return oracle.backward_frames(gy, v["x"], y, v["a"], v["b"], v["xi"], v["yi"], hop=hop,
                                  layout=layout)


CASES = [(False, "BT", 2, 3), (False, "TB", 2, 3), (True, "BT", 2, 3), (True, "TB", 1, 4),
         (False, "BT", None, 2), (True, "TB", None, 3), (True, "BT", 3, 0)]


@pytest.mark.parametrize("tv,layout,M,N", CASES)
def test_jvp_matches_central_differences_of_forward(tv, layout, M, N):
    v, _, rng = _problem(8100 + 10 * tv + 3 * (N or 0), tv, layout, M=M, N=N)
    t = _like(rng, v)
    y = _fwd(v, layout)
    dy = oracle.jvp(v["x"], y, v["a"], v["b"], v["xi"], v["yi"], dx=t["x"], da=t["a"],
                    db=t["b"], dxi=t["xi"], dyi=t["yi"], layout=layout)
    h = 1e-6
    step = lambda s: {k: (None if w is None else w + s * h * t[k]) for k, w in v.items()}
    fd = (_fwd(step(1), layout) - _fwd(step(-1), layout)) / (2 * h)
    np.testing.assert_allclose(dy, fd, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("tv,layout,M,N", CASES)
def test_jvp_pairs_with_backward(tv, layout, M, N):
    v, gy, rng = _problem(8200 + 10 * tv + 3 * (N or 0), tv, layout, M=M, N=N, T=40, B=3)
    t = _like(rng, v)
    y = _fwd(v, layout)
    dy = oracle.jvp(v["x"], y, v["a"], v["b"], v["xi"], v["yi"], dx=t["x"], da=t["a"],
                    db=t["b"], dxi=t["xi"], dyi=t["yi"], layout=layout)
    g = _bwd(gy, y, v, layout)
    lhs = float((gy * dy).sum())
    rhs = float(sum((g[k] * t[k]).sum() for k in NAMES if t[k] is not None and k in g))
    assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(lhs))


def _Q(gy, y, v, cot, layout, hop=None):
    g = _bwd(gy, y, v, layout, hop)
    return float(sum((g[k] * cot[k]).sum() for k in NAMES if cot[k] is not None and k in g))


def _b2(gy, y, v, cot, layout, hop=None):
    kw = dict(vx=cot["x"], va=cot["a"], vb=cot["b"], vxi=cot["xi"], vyi=cot["yi"],
              layout=layout)
    if hop is None:
        return oracle.backward2(gy, v["x"], y, v["a"], v["b"], v["xi"], v["yi"], **kw)
    return oracle.backward2_frames(gy, v["x"], y, v["a"], v["b"], v["xi"], v["yi"], hop=hop,
                                   **kw)


def _fd_check(gy, y, v, cot, layout, hop=None, h=1e-5):
    g2 = _b2(gy, y, v, cot, layout, hop)
    inputs = dict(v, gy=gy, y=y)
    for name in ("gy", "x", "y", "a", "b", "xi", "yi"):
        base = inputs[name]
        if base is None:
            assert name not in g2 or not np.any(g2[name]), name
            continue
        fd = np.zeros_like(base)
        for idx in np.ndindex(base.shape):
            vals = []
            for s in (1, -1):
                w = {k: (None if u is None else u.copy()) for k, u in inputs.items()}
                w[name][idx] += s * h
                vv = {k: w[k] for k in NAMES}
                vals.append(_Q(w["gy"], w["y"], vv, cot, layout, hop))
            fd[idx] = (vals[0] - vals[1]) / (2 * h)
        np.testing.assert_allclose(g2[name], fd, rtol=1e-6, atol=1e-8, err_msg=name)


@pytest.mark.parametrize("tv,layout,M,N", CASES)
def test_backward2_matches_central_differences(tv, layout, M, N):
    v, gy, rng = _problem(8300 + 10 * tv + 3 * (N or 0), tv, layout, M=M, N=N)
    cot = _like(rng, v)
    y = _fwd(v, layout)
    # y enters the backward as an input of its own: perturb it away from the
    # forward's output so that nothing relies on y = forward(x)
    y = y + 0.1 * rng.standard_normal(y.shape)
    _fd_check(gy, y, v, cot, layout)


def test_backward2_with_some_cotangents_zero():
    v, gy, rng = _problem(8400, True, "BT", M=2, N=3)
    y = _fwd(v, "BT")
    for drop in (("x", "xi"), ("a", "yi"), ("b",), ("x", "a", "b", "xi", "yi")):
        cot = _like(rng, v)
        for k in drop:
            cot[k] = None
        _fd_check(gy, y, v, cot, "BT")


@pytest.mark.parametrize("layout", ["BT", "TB"])
def test_backward2_frames_matches_central_differences(layout):
    v, gy, rng = _problem(8500 + (layout == "TB"), True, layout, M=1, N=2, T=11, hop=4)
    cot = _like(rng, v)
    y = _fwd(v, layout, hop=4)
    _fd_check(gy, y, v, cot, layout, hop=4)


def _hvp(w, v, t, layout):
    """H t for L = <w, forward(theta)>: backward2 gives the explicit part;
    its y output flows back through y = forward(theta) (the backward)."""
    y = _fwd(v, layout)
    g2 = _b2(w, y, v, t, layout)
    back = _bwd(g2["y"], y, v, layout)
    return {k: g2[k] + back[k] for k in NAMES if v[k] is not None}


@pytest.mark.parametrize("tv,layout", [(False, "BT"), (True, "TB")])
def test_hessian_vector_product_matches_gradient_differences(tv, layout):
    v, w, rng = _problem(8600 + tv, tv, layout, M=2, N=3, T=12)
    t = _like(rng, v)
    hv = _hvp(w, v, t, layout)
    h = 1e-6

    def grad(s):
        vv = {k: (None if u is None else u + s * h * t[k]) for k, u in v.items()}
        return _bwd(w, _fwd(vv, layout), vv, layout)

    gp, gm = grad(1), grad(-1)
    for k in hv:
        np.testing.assert_allclose(hv[k], (gp[k] - gm[k]) / (2 * h), rtol=1e-6, atol=1e-8,
                                   err_msg=k)


def test_hessian_is_symmetric():
    v, w, rng = _problem(8700, True, "BT", M=2, N=3, T=30, B=3)
    s, t = _like(rng, v), _like(rng, v)
    hs, ht = _hvp(w, v, s, "BT"), _hvp(w, v, t, "BT")
    a = sum(float((s[k] * ht[k]).sum()) for k in ht)
    b = sum(float((t[k] * hs[k]).sum()) for k in hs)
    assert abs(a - b) <= 1e-10 * max(1.0, abs(a))
