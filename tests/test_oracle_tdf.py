"""Pins of the oracle's state-space filter and transposed direct form II
(Sec. 2 Eqs. 4-5 with the backward of Sec. 3.1 Eqs. 6-9 and App. A).

* the transposed direct form with an initial state against SciPy's
  lfilter(b, a, x, zi) (a library routine), every order shape;
* with zero initial state it is the same transfer function as the direct
  form, whose oracle (oracle.c) is separate code;
* every gradient (x, b, a, zi; and A, B, C, D, v(0) of a general dense
  state-space filter) against central finite differences of the forward;
* y is linear in (x, zi) jointly, so <gy, y> = <gx, x> + <gzi, zi>.
"""
import numpy as np
import pytest
import scipy.signal

import oracle

SHAPES = [(0, 1), (0, 2), (2, 2), (3, 1), (1, 4), (4, 4), (5, 0), (0, 6)]


def _tdf_problem(seed, B, T, M, N, layout):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((B, M + 1))
    # stable denominators: a random real pole per order, radius <= 0.9
    a = np.zeros((B, N))
    for c in range(B):
        den = np.poly(rng.uniform(-0.9, 0.9, N)) if N else np.ones(1)
        a[c] = den[1:]
    K = max(M, N, 1)
    zi = rng.normal(0.0, 0.5, (B, K))
    x = rng.standard_normal((B, T) if layout == "BT" else (T, B))
    gy = rng.standard_normal(x.shape)
    return x, b, a, zi, gy


@pytest.mark.parametrize("M,N", SHAPES)
@pytest.mark.parametrize("layout", ["BT", "TB"])
def test_tdf_forward_matches_scipy_lfilter_with_zi(M, N, layout):
    x, b, a, zi, _ = _tdf_problem(700 + 10 * M + N, 3, 120, M, N, layout)
    y = oracle.tdf_forward(x, b, a, zi, layout=layout)
    xs = x if layout == "BT" else x.T
    ys = y if layout == "BT" else y.T
    for c in range(3):
        want, _ = scipy.signal.lfilter(b[c], np.r_[1.0, a[c]], xs[c], zi=zi[c])
        np.testing.assert_allclose(ys[c], want, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("M,N", SHAPES)
def test_tdf_with_zero_state_is_the_direct_form(M, N):
    x, b, a, _, _ = _tdf_problem(720 + 10 * M + N, 2, 90, M, N, "BT")
    y = oracle.tdf_forward(x, b, a, None)
    np.testing.assert_allclose(y, oracle.forward(x, a, b, layout="BT"), rtol=1e-12,
                               atol=1e-12)


def _fd(loss, base, h=1e-6):
    out = {}
    for name, v in base.items():
        g = np.zeros_like(v)
        for idx in np.ndindex(v.shape):
            args = {k: w.copy() for k, w in base.items()}
            args[name][idx] += h
            lp = loss(**args)
            args[name][idx] -= 2 * h
            lm = loss(**args)
            g[idx] = (lp - lm) / (2 * h)
        out[name] = g
    return out


@pytest.mark.parametrize("M,N", [(2, 3), (3, 1), (0, 2), (4, 0)])
@pytest.mark.parametrize("layout", ["BT", "TB"])
def test_tdf_gradients_match_central_finite_differences(M, N, layout):
    x, b, a, zi, gy = _tdf_problem(740 + 10 * M + N, 2, 11, M, N, layout)
    g = oracle.tdf_backward(gy, x, b, a, zi, layout=layout)

    def loss(x, b, a, zi):
        return float((gy * oracle.tdf_forward(x, b, a, zi, layout=layout)).sum())

    fd = _fd(loss, dict(x=x, b=b, a=a, zi=zi))
    for k in ("x", "b", "a", "zi"):
        np.testing.assert_allclose(g[k], fd[k], rtol=1e-6, atol=1e-7, err_msg=k)


def test_general_state_space_gradients_match_finite_differences():
    rng = np.random.default_rng(760)
    Bn, K, T = 2, 3, 9
    A = 0.4 * rng.standard_normal((Bn, K, K))
    Bv = rng.standard_normal((Bn, K))
    C = rng.standard_normal((Bn, K))
    D = rng.standard_normal(Bn)
    v0 = rng.standard_normal((Bn, K))
    x = rng.standard_normal((Bn, T))
    gy = rng.standard_normal((Bn, T))
    g = oracle.ss_backward(gy, x, A, Bv, C, D, v0)

    def loss(x, A, B, C, D, v0):
        return float((gy * oracle.ss_forward(x, A, B, C, D, v0)).sum())

    fd = _fd(loss, dict(x=x, A=A, B=Bv, C=C, D=D, v0=v0))
    for k in ("x", "A", "B", "C", "D", "v0"):
        np.testing.assert_allclose(g[k], fd[k], rtol=1e-6, atol=1e-7, err_msg=k)


@pytest.mark.parametrize("M,N", [(3, 2), (1, 4)])
def test_tdf_adjoint_identity(M, N):
    x, b, a, zi, gy = _tdf_problem(780 + M, 3, 50, M, N, "BT")
    y = oracle.tdf_forward(x, b, a, zi)
    g = oracle.tdf_backward(gy, x, b, a, zi)
    lhs = float((gy * y).sum())
    rhs = float((g["x"] * x).sum() + (g["zi"] * zi).sum())
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))
