"""Pins of the oracle's second-order-section cascade: the output against
SciPy's sosfilt with per-section initial states (a library routine), and
every gradient against central finite differences of the cascade."""
import numpy as np
import pytest
import scipy.signal

import oracle


def _sos_problem(seed, S, B, T, layout):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((S, B, 3))
    a = np.zeros((S, B, 2))
    for s in range(S):
        r = rng.uniform(0.3, 0.95, B)
        th = rng.uniform(0.0, np.pi, B)
        a[s, :, 0] = -2 * r * np.cos(th)
        a[s, :, 1] = r * r
    zi = rng.normal(0.0, 0.3, (S, B, 2))
    x = rng.standard_normal((B, T) if layout == "BT" else (T, B))
    gy = rng.standard_normal(x.shape)
    return x, b, a, zi, gy


@pytest.mark.parametrize("S", [1, 2, 4])
@pytest.mark.parametrize("layout", ["BT", "TB"])
def test_sos_forward_matches_scipy_sosfilt(S, layout):
    x, b, a, zi, _ = _sos_problem(800 + S, S, 3, 150, layout)
    y = oracle.sos_forward(x, b, a, zi, layout)
    xs = x if layout == "BT" else x.T
    ys = y if layout == "BT" else y.T
    for c in range(3):
        sos = np.concatenate([b[:, c], np.ones((S, 1)), a[:, c]], axis=1)
        want, _ = scipy.signal.sosfilt(sos, xs[c], zi=zi[:, c])
        np.testing.assert_allclose(ys[c], want, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("layout", ["BT", "TB"])
def test_sos_gradients_match_central_finite_differences(layout):
    x, b, a, zi, gy = _sos_problem(820, 3, 2, 10, layout)
    g = oracle.sos_backward(gy, x, b, a, zi, layout)
    h = 1e-6
    base = dict(x=x, b=b, a=a, zi=zi)
    for name, v in base.items():
        fd = np.zeros_like(v)
        for idx in np.ndindex(v.shape):
            args = {k: w.copy() for k, w in base.items()}
            args[name][idx] += h
            lp = float((gy * oracle.sos_forward(args["x"], args["b"], args["a"], args["zi"],
                                                layout)).sum())
            args[name][idx] -= 2 * h
            lm = float((gy * oracle.sos_forward(args["x"], args["b"], args["a"], args["zi"],
                                                layout)).sum())
            fd[idx] = (lp - lm) / (2 * h)
        np.testing.assert_allclose(g[name], fd, rtol=1e-6, atol=1e-7, err_msg=name)
