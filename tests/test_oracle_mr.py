"""Pins of the oracle's matrix recurrence v(n+1) = A v(n) + z(n) (the
state-space recursion of Sec. 2 Eq. 4 with the input in state space, the
operator of App. B) and its backward (Sec. 3.1 Eqs. 7 and 9).

* zero input: v(n) = A^n v0 (numpy matrix powers); impulse input: the
  columns of A^n;
* one state: the first-order all-pole direct form (oracle.forward, separate
  C code) and its backward;
* diagonal A: each component is SciPy's first-order lfilter with zi;
* the gradients against central finite differences (both layouts), and the
  adjoint identity <gv, v> = <gz, z> + <gv0, v0> (v is linear in z, v0).
"""
import numpy as np
import pytest
import scipy.signal

import oracle


def _problem(seed, B, T, K, layout, scale=0.4):
    rng = np.random.default_rng(seed)
    A = scale * rng.standard_normal((B, K, K)) / np.sqrt(K)
    v0 = rng.standard_normal((B, K))
    shape = (B, T, K) if layout == "BT" else (T, B, K)
    return A, v0, rng.standard_normal(shape), rng.standard_normal(shape)


@pytest.mark.parametrize("layout", ["BT", "TB"])
def test_zero_input_gives_matrix_powers(layout):
    A, v0, z, _ = _problem(9600, 2, 12, 5, layout)
    v = oracle.mr_forward(A, v0, np.zeros_like(z), layout=layout)
    vc = v if layout == "BT" else v.transpose(1, 0, 2)
    for b in range(2):
        for n in range(12):
            np.testing.assert_allclose(vc[b, n], np.linalg.matrix_power(A[b], n + 1) @ v0[b],
                                       rtol=1e-12, atol=1e-14)


def test_impulse_input_gives_columns_of_powers():
    A, _, z, _ = _problem(9601, 1, 9, 4, "BT")
    for j in range(4):
        z = np.zeros((1, 9, 4))
        z[0, 0, j] = 1.0
        v = oracle.mr_forward(A, None, z)
        for n in range(9):
            np.testing.assert_allclose(v[0, n], np.linalg.matrix_power(A[0], n)[:, j],
                                       rtol=1e-12, atol=1e-14)


def test_one_state_is_the_first_order_direct_form():
    rng = np.random.default_rng(9602)
    B, T = 3, 40
    a1 = rng.uniform(-0.9, 0.9, B)
    A = a1[:, None, None]
    v0 = rng.standard_normal((B, 1))
    z = rng.standard_normal((B, T, 1))
    gv = rng.standard_normal((B, T, 1))
    v = oracle.mr_forward(A, v0, z)
    # y[n] = z[n] - (-a1) y[n-1], y[-1] = v0: y[n] = v(n+1)
    y = oracle.forward(z[:, :, 0], -a1[:, None], None, None, v0, layout="BT")
    np.testing.assert_allclose(v[:, :, 0], y, rtol=1e-12, atol=1e-13)
    g = oracle.mr_backward(gv, A, v0, v)
    gd = oracle.backward(gv[:, :, 0], z[:, :, 0], y, -a1[:, None], None, None, v0, layout="BT")
    np.testing.assert_allclose(g["z"][:, :, 0], gd["x"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(g["A"][:, 0, 0], -gd["a"][:, 0], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(g["v0"][:, 0], gd["yi"][:, 0], rtol=1e-12, atol=1e-13)


def test_diagonal_A_is_scipy_first_order_lfilter():
    rng = np.random.default_rng(9603)
    K, T = 4, 50
    lam = rng.uniform(-0.95, 0.95, K)
    A = np.diag(lam)[None]
    v0 = rng.standard_normal((1, K))
    z = rng.standard_normal((1, T, K))
    v = oracle.mr_forward(A, v0, z)
    for i in range(K):
        want, _ = scipy.signal.lfilter([1.0], [1.0, -lam[i]], z[0, :, i], zi=[lam[i] * v0[0, i]])
        np.testing.assert_allclose(v[0, :, i], want, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("layout", ["BT", "TB"])
@pytest.mark.parametrize("K", [1, 3, 5])
def test_gradients_match_central_differences(layout, K):
    A, v0, z, gv = _problem(9610 + K, 2, 8, K, layout)
    v = oracle.mr_forward(A, v0, z, layout=layout)
    g = oracle.mr_backward(gv, A, v0, v, layout=layout)
    base = {"A": A, "v0": v0, "z": z}

    def loss(A, v0, z):
        return float((gv * oracle.mr_forward(A, v0, z, layout=layout)).sum())

    h = 1e-6
    for name, val in base.items():
        fd = np.zeros_like(val)
        for idx in np.ndindex(val.shape):
            args = {k: w.copy() for k, w in base.items()}
            args[name][idx] += h
            lp = loss(**args)
            args[name][idx] -= 2 * h
            fd[idx] = (lp - loss(**args)) / (2 * h)
        np.testing.assert_allclose(g[name], fd, rtol=1e-6, atol=1e-8, err_msg=name)


def test_adjoint_identity():
    A, v0, z, gv = _problem(9620, 3, 60, 6, "TB")
    v = oracle.mr_forward(A, v0, z, layout="TB")
    g = oracle.mr_backward(gv, A, v0, v, layout="TB")
    lhs = float((gv * v).sum())
    rhs = float((g["z"] * z).sum() + (g["v0"] * v0).sum())
    assert abs(lhs - rhs) <= 1e-11 * max(1.0, abs(lhs))


def test_empty_signal():
    A, v0, z, gv = _problem(9630, 2, 0, 3, "BT")
    v = oracle.mr_forward(A, v0, z)
    g = oracle.mr_backward(gv, A, v0, v)
    assert v.shape == (2, 0, 3)
    assert not g["A"].any() and not g["v0"].any()
