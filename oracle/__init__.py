"""FP64 CPU oracle for the direct-form filter and its closed-form backward.

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
benchmark's CPU-baseline leg call this; the product path never does.  It
shares no code with the HIP library (``oracle.c`` is plain C compiled with
gcc).  See ``oracle.c`` for the equations (paper Sec. 2 Eq. 1, Sec. 3.1
Eqs. 6-9, Appendix A) and the reading of each.

Array conventions (numpy, any real dtype; converted to float64 here):

* layout ``"TB"``: signals ``[T, B]``; layout ``"BT"``: signals ``[B, T]``.
* ``a``: ``[B, N]`` (time-invariant) or ``[T, B, N]`` / ``[B, T, N]``
  (per-sample, following the signal layout), holding ``a_1..a_N``.
* ``b``: same with ``M + 1`` taps ``b_0..b_M``; ``None`` means ``b = [1]``.
* ``xi``: ``[B, M]`` with ``xi[:, j-1] = x[-j]``; ``yi``: ``[B, N]``.

Parity status: every function here is pinned by tests under ``tests/``
(``test_oracle_pins.py``, ``test_oracle_frames.py``, ``test_oracle_tdf.py``,
``test_oracle_sos.py``, ``test_oracle_backward2.py``, ``test_oracle_mr.py``:
closed forms, SciPy,
dense solves, finite differences, adjoint and pairing identities, Hessian
symmetry); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (in place)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC,
                               "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64, I = ctypes.c_int64, ctypes.c_int
        lib.oracle_forward.argtypes = [I64, I64, I, I, I, I, P, P, P, P, P, P, I]
        lib.oracle_forward.restype = I
        lib.oracle_backward.argtypes = [I64, I64, I, I, I, I] + [P] * 12 + [I]
        lib.oracle_backward.restype = I
        _lib = lib
    return _lib


def _f64(a):
    if a is None:
        return None
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dims(x, a, b, layout):
    if layout not in ("TB", "BT"):
        raise ValueError("layout must be 'TB' or 'BT'")
    if x.ndim != 2:
        raise ValueError("x must be 2-D")
    T, B = x.shape if layout == "TB" else x.shape[::-1]
    N = 0 if a is None else a.shape[-1]
    M = 0 if b is None else b.shape[-1] - 1
    tv = int((a is not None and a.ndim == 3) or (b is not None and b.ndim == 3))
    for c, K in ((a, N), (b, M + 1)):
        if c is None:
            continue
        want = (B, K) if not tv else ((T, B, K) if layout == "TB" else (B, T, K))
        if c.shape != want:
            raise ValueError(f"coefficient shape {c.shape} != {want}")
    return int(B), int(T), int(M), int(N), tv


def forward(x, a, b=None, xi=None, yi=None, layout="BT", nthreads=1):
    """y = direct-form filter of x (FP64)."""
    x, a, b, xi, yi = map(_f64, (x, a, b, xi, yi))
    B, T, M, N, tv = _dims(x, a, b, layout)
    if a is None:
        a = np.zeros((B, 0) if not tv else x.shape + (0,))
    y = np.zeros_like(x)
    rc = _load().oracle_forward(B, T, M, N, tv, 0 if layout == "TB" else 1, _ptr(x), _ptr(b),
                                _ptr(a), _ptr(xi), _ptr(yi), _ptr(y), int(nthreads))
    if rc:
        raise ValueError("oracle_forward rejected its arguments")
    return y


def backward(gy, x, y, a, b=None, xi=None, yi=None, layout="BT", nthreads=1,
             want=("x", "a", "b", "xi", "yi")):
    """Closed-form gradients.  Returns a dict with the requested keys among
    x, a, b, xi, yi (b only if b was given)."""
    gy, x, y, a, b, xi, yi = map(_f64, (gy, x, y, a, b, xi, yi))
    B, T, M, N, tv = _dims(x, a, b, layout)
    if a is None:
        a = np.zeros((B, 0) if not tv else x.shape + (0,))
    out = {}
    gx = np.zeros_like(x) if "x" in want else None
    ga = np.zeros_like(a) if "a" in want else None
    gb = np.zeros_like(b) if ("b" in want and b is not None) else None
    gxi = np.zeros((B, M)) if "xi" in want else None
    gyi = np.zeros((B, N)) if "yi" in want else None
    rc = _load().oracle_backward(B, T, M, N, tv, 0 if layout == "TB" else 1, _ptr(gy), _ptr(x),
                                 _ptr(y), _ptr(b), _ptr(a), _ptr(xi), _ptr(yi), _ptr(gx),
                                 _ptr(gb), _ptr(ga), _ptr(gxi), _ptr(gyi), int(nthreads))
    if rc:
        raise ValueError("oracle_backward rejected its arguments")
    for k, v in (("x", gx), ("a", ga), ("b", gb), ("xi", gxi), ("yi", gyi)):
        if v is not None:
            out[k] = v
    return out


# ---------------------------------------------------------------------------
# Frame-held coefficients (parameter-varying filters whose coefficients change
# once per frame of `hop` samples; the paper's closing remarks on
# parameter-varying cases, with the gradients of Sec. 3.1 Eqs. 6-9).
#
# A frame-held row set has F = ceil(T / hop) rows per channel: [F, B, K]
# (layout "TB") or [B, F, K] ("BT").  Sample t uses the row of frame t // hop,
# so the filter is the per-sample one on the expanded rows, and by the chain
# rule the gradient of a frame's row is the sum of the per-sample gradient
# rows over the frame's samples.


def _frame_axis(layout):
    if layout not in ("TB", "BT"):
        raise ValueError("layout must be 'TB' or 'BT'")
    return 0 if layout == "TB" else 1


def frame_expand(c, T, hop, layout="BT"):
    """Per-sample rows (the layout of a per-sample coefficient array) from
    frame-held rows: row t is the row of frame t // hop."""
    c = _f64(c)
    hop = int(hop)
    if hop < 1:
        raise ValueError("hop must be >= 1")
    ax = _frame_axis(layout)
    F = -(-int(T) // hop)
    if c.ndim != 3 or c.shape[ax] != F:
        raise ValueError(f"frame rows must have {F} frames on axis {ax}, got {c.shape}")
    return np.take(c, np.arange(int(T)) // hop, axis=ax)


def frame_reduce(g, hop, layout="BT"):
    """Gradient of frame-held rows from per-sample gradient rows: the sum of
    the rows of each frame's samples (the last frame may be shorter)."""
    g = _f64(g)
    hop = int(hop)
    ax = _frame_axis(layout)
    T = g.shape[ax]
    if T == 0:
        return np.zeros(g.shape[:ax] + (0,) + g.shape[ax + 1:])
    return np.add.reduceat(g, np.arange(0, T, hop), axis=ax)


def forward_frames(x, a, b=None, xi=None, yi=None, hop=1, layout="BT", nthreads=1):
    """Forward with frame-held a (and b, if given)."""
    x = _f64(x)
    T = x.shape[0] if layout == "TB" else x.shape[1]
    ae = None if a is None else frame_expand(a, T, hop, layout)
    be = None if b is None else frame_expand(b, T, hop, layout)
    return forward(x, ae, be, xi, yi, layout=layout, nthreads=nthreads)


def backward_frames(gy, x, y, a, b=None, xi=None, yi=None, hop=1, layout="BT", nthreads=1,
                    want=("x", "a", "b", "xi", "yi")):
    """Closed-form gradients with frame-held a (and b): the per-sample
    backward on the expanded rows, its a / b rows reduced per frame."""
    x = _f64(x)
    T = x.shape[0] if layout == "TB" else x.shape[1]
    ae = None if a is None else frame_expand(a, T, hop, layout)
    be = None if b is None else frame_expand(b, T, hop, layout)
    g = backward(gy, x, y, ae, be, xi, yi, layout=layout, nthreads=nthreads, want=want)
    for k in ("a", "b"):
        if k in g:
            g[k] = frame_reduce(g[k], hop, layout)
    return g


# ---------------------------------------------------------------------------
# State-space filter and the transposed direct form (Sec. 2 Eqs. 4-5; the
# backward of Sec. 3.1 Eqs. 6-9 and App. A), time-invariant.
#
# State-space filter, per channel: v(n+1) = A v(n) + B x(n),
# y(n) = C . v(n) + D x(n), with the initial state v(0).  Shapes: x [B, T]
# ("BT") or [T, B] ("TB"); A [B, K, K]; Bv, C [B, K]; D [B]; v0 [B, K].
#
# Transposed direct form II (SciPy's lfilter with its zi state): with
# K = max(M, N), b_j = 0 past M and a_j = 0 past N, the state after sample n
# is z(n), y(n) = b_0 x(n) + z_0(n-1) and
# z_i(n) = b_{i+1} x(n) - a_{i+1} y(n) + z_{i+1}(n-1).  As a state-space
# filter with v(n) = z(n-1) (so v(0) = zi): A[i][0] = -a_{i+1},
# A[i][i+1] = 1, B_i = b_{i+1} - a_{i+1} b_0, C = e_0, D = b_0 -- the
# transpose of the direct form's companion realisation with B and C swapped
# (Sec. 2).


def _chan_first(v, layout):
    return v if layout == "BT" else v.T


def ss_forward(x, A, Bv, C, D, v0=None, layout="BT"):
    """y of the state-space filter (FP64), every channel at once."""
    x = _chan_first(_f64(x), layout)
    A, Bv, C, D = map(_f64, (A, Bv, C, D))
    Bn, T = x.shape
    K = A.shape[-1]
    v = np.zeros((Bn, K)) if v0 is None else _f64(v0).copy()
    y = np.zeros((Bn, T))
    for n in range(T):
        y[:, n] = np.einsum("bk,bk->b", C, v) + D * x[:, n]
        v = np.einsum("bij,bj->bi", A, v) + Bv * x[:, n, None]
    return y if layout == "BT" else y.T


def ss_backward(gy, x, A, Bv, C, D, v0=None, layout="BT"):
    """Gradients of L = <gy, y> for the state-space filter by the paper's
    reverse recursion: gz(n) = A^T gz(n+1) + C gy(n+1) from gz(T-1) = 0
    (Eq. 7 with dL/dv(n) = gy(n) C, Eq. 6), gx(n) = B . gz(n) + D gy(n)
    (Eq. 8), gv0 = gz(-1), gB = sum_n gz(n) x(n), gA_ij = sum_n gz_i(n) v_j(n)
    (Eq. 9, the chain-rule orientation), gC = sum_n gy(n) v(n),
    gD = sum_n gy(n) x(n) (Eq. 6).  Returns a dict x, A, B, C, D, v0."""
    x = _chan_first(_f64(x), layout)
    gy = _chan_first(_f64(gy), layout)
    A, Bv, C, D = map(_f64, (A, Bv, C, D))
    Bn, T = x.shape
    K = A.shape[-1]
    # the states v(0) .. v(T-1) of the forward
    vs = np.zeros((T, Bn, K))
    v = np.zeros((Bn, K)) if v0 is None else _f64(v0).copy()
    for n in range(T):
        vs[n] = v
        v = np.einsum("bij,bj->bi", A, v) + Bv * x[:, n, None]
    gx = np.zeros((Bn, T))
    gA = np.zeros_like(A)
    gB = np.zeros_like(Bv)
    gC = np.zeros_like(C)
    gD = np.zeros(Bn)
    gz = np.zeros((Bn, K))  # gz(T-1)
    for n in range(T - 1, -1, -1):
        if n < T - 1:
            gz = np.einsum("bji,bj->bi", A, gz) + C * gy[:, n + 1, None]
        gx[:, n] = np.einsum("bk,bk->b", Bv, gz) + D * gy[:, n]
        gB += gz * x[:, n, None]
        gA += gz[:, :, None] * vs[n][:, None, :]
        gC += gy[:, n, None] * vs[n]
        gD += gy[:, n] * x[:, n]
    gv0 = np.einsum("bji,bj->bi", A, gz) + C * gy[:, 0, None] if T > 0 else np.zeros((Bn, K))
    return {"x": gx if layout == "BT" else gx.T, "A": gA, "B": gB, "C": gC, "D": gD,
            "v0": gv0}


def tdf_matrices(b, a):
    """(A, B, C, D) of the transposed direct form II for b [B, M+1], a [B, N]
    (a_0 = 1 implicit), K = max(M, N) (at least 1)."""
    b, a = _f64(b), _f64(a)
    Bn = b.shape[0]
    M, N = b.shape[1] - 1, a.shape[1]
    K = max(M, N, 1)
    bb = np.zeros((Bn, K + 1))
    bb[:, :M + 1] = b
    aa = np.zeros((Bn, K + 1))
    aa[:, 1:N + 1] = a
    A = np.zeros((Bn, K, K))
    A[:, :, 0] = -aa[:, 1:]
    for i in range(K - 1):
        A[:, i, i + 1] = 1.0
    Bv = bb[:, 1:] - aa[:, 1:] * bb[:, :1]
    C = np.zeros((Bn, K))
    C[:, 0] = 1.0
    return A, Bv, C, bb[:, 0].copy()


def tdf_forward(x, b, a, zi=None, layout="BT"):
    """Transposed direct form II with initial state zi [B, max(M, N)]
    (SciPy's lfilter semantics), time-invariant."""
    A, Bv, C, D = tdf_matrices(b, a)
    return ss_forward(x, A, Bv, C, D, zi, layout)


def tdf_backward(gy, x, b, a, zi=None, layout="BT"):
    """Gradients of the transposed direct form with respect to x, b, a and
    zi: the state-space gradients mapped through tdf_matrices by the chain
    rule (B_i = b_{i+1} - a_{i+1} b_0, A[i][0] = -a_{i+1}, D = b_0)."""
    b, a = _f64(b), _f64(a)
    M, N = b.shape[1] - 1, a.shape[1]
    A, Bv, C, D = tdf_matrices(b, a)
    K = A.shape[-1]
    g = ss_backward(gy, x, A, Bv, C, D, zi, layout)
    aa = np.zeros((b.shape[0], K))
    aa[:, :N] = a
    gb = np.zeros_like(b)
    gb[:, 0] = g["D"] - (g["B"] * aa).sum(axis=1)
    gb[:, 1:] = g["B"][:, :M]
    ga = -g["A"][:, :N, 0] - b[:, :1] * g["B"][:, :N]
    return {"x": g["x"], "b": gb, "a": ga, "zi": g["v0"]}


# ---------------------------------------------------------------------------
# Second-order sections (the cascade of biquads the paper's experiments
# motivate for higher orders, Sec. 4; SciPy's sosfilt): section s filters the
# previous section's output with b [S, B, 3], a [S, B, 2] (a_0 = 1 implied)
# in the transposed direct form with its own initial state zi [S, B, 2].


def sos_forward(x, b, a, zi=None, layout="BT"):
    """Cascade output: every section's transposed-form filter in turn."""
    y = _f64(x)
    for s in range(b.shape[0]):
        y = tdf_forward(y, b[s], a[s], None if zi is None else zi[s], layout)
    return y


def sos_backward(gy, x, b, a, zi=None, layout="BT"):
    """Gradients of the cascade: the sections' inputs from a forward pass,
    then each section's transposed-form gradients from the last section to
    the first, the input gradient of one section being the output gradient
    of the one before it (chain rule)."""
    S = b.shape[0]
    ins = [_f64(x)]
    for s in range(S - 1):
        ins.append(tdf_forward(ins[-1], b[s], a[s], None if zi is None else zi[s], layout))
    g = _f64(gy)
    gb = np.zeros(b.shape)
    ga = np.zeros(a.shape)
    gzi = np.zeros((S,) + a.shape[1:])
    for s in range(S - 1, -1, -1):
        r = tdf_backward(g, ins[s], b[s], a[s], None if zi is None else zi[s], layout)
        gb[s], ga[s], gzi[s] = r["b"], r["a"], r["zi"]
        g = r["x"]
    return {"x": g, "b": gb, "a": ga, "zi": gzi}


# ---------------------------------------------------------------------------
# Forward-mode derivative and the derivative of the backward pass (the
# paper's closing remarks: forward-mode differentiation follows the same way
# and serves second-order optimisation).  Plain FP64 loops over time,
# channels vectorised; coefficients are taken as per-sample rows (time-
# invariant ones repeated over time, their gradients summed over time).


def _chan(v, layout):
    """Signal as [B, T] (channel first)."""
    return None if v is None else _chan_first(_f64(v), layout)


def _rows(c, B, T, layout):
    """Coefficients as per-sample rows [B, T, K] (channel first)."""
    if c is None:
        return None
    c = _f64(c)
    if c.ndim == 2:
        return np.broadcast_to(c[:, None, :], (B, T, c.shape[1]))
    return c if layout == "BT" else c.transpose(1, 0, 2)


def _back(v, vi, n):
    """v[:, n] for n >= 0, else the history vi[:, -n - 1] (zero past its end
    or when vi is None)."""
    if n >= 0:
        return v[:, n]
    j = -n
    if vi is None or j > vi.shape[1]:
        return 0.0
    return vi[:, j - 1]


def _out_sig(v, layout):
    return v if layout == "BT" else v.T.copy()


def _out_rows(g, tv, layout):
    """Per-sample gradient rows [B, T, K] to the coefficient layout; summed
    over time for time-invariant coefficients."""
    if not tv:
        return g.sum(axis=1)
    return g if layout == "BT" else g.transpose(1, 0, 2).copy()


def jvp(x, y, a, b=None, xi=None, yi=None, dx=None, da=None, db=None, dxi=None, dyi=None,
        layout="BT"):
    """Tangent of y = forward(x, a, b, xi, yi) along (dx, da, db, dxi, dyi)
    (None = zero).  Eq. 1 differentiated term by term:
        dy[n] = sum_k b_k[n] dx[n-k] + sum_k db_k[n] x[n-k]
                - sum_k da_k[n] y[n-k] - sum_k a_k[n] dy[n-k],
    with the histories xi, yi, dxi, dyi before time 0.  y is the forward's
    output."""
    xc, yc = _chan(x, layout), _chan(y, layout)
    B, T = xc.shape
    M = 0 if b is None else _f64(b).shape[-1] - 1
    N = 0 if a is None else _f64(a).shape[-1]
    ar, br = _rows(a, B, T, layout), _rows(b, B, T, layout)
    dar, dbr = _rows(da, B, T, layout), _rows(db, B, T, layout)
    dxc = _chan(dx, layout)
    xi, yi, dxi, dyi = map(_f64, (xi, yi, dxi, dyi))
    dy = np.zeros((B, T))
    for n in range(T):
        acc = np.zeros(B)
        if dxc is not None or dxi is not None:
            src = dxc if dxc is not None else np.zeros((B, T))
            for k in range(M + 1):
                bk = br[:, n, k] if br is not None else 1.0
                acc += bk * _back(src, dxi, n - k)
        if dbr is not None:
            for k in range(M + 1):
                acc += dbr[:, n, k] * _back(xc, xi, n - k)
        if dar is not None:
            for k in range(1, N + 1):
                acc -= dar[:, n, k - 1] * _back(yc, yi, n - k)
        for k in range(1, N + 1):
            acc -= ar[:, n, k - 1] * _back(dy, dyi, n - k)
        dy[:, n] = acc
    return _out_sig(dy, layout)


def backward2(gy, x, y, a, b=None, xi=None, yi=None, vx=None, va=None, vb=None, vxi=None,
              vyi=None, layout="BT"):
    """Derivative of the backward pass.  backward() maps (gy, x, y, a, b, xi,
    yi) -- y taken as an input of its own -- to the gradients (gx, ga, gb,
    gxi, gyi); for cotangents (vx, va, vb, vxi, vyi) of those (None = zero)
    this returns the gradient of
        Q = <vx, gx> + <va, ga> + <vb, gb> + <vxi, gxi> + <vyi, gyi>
    with respect to every input, keys gy, x, y, a, b, xi, yi (b, xi only
    when b is given, a / yi only when N > 0).

    The gradients are the transposed Jacobian of the forward applied to gy,
    so Q = <gy, dy> with dy the tangent jvp() gives along the cotangents, and
    (ybar the adjoint, ybar[n] = gy[n] - sum_k a_k[n+k] ybar[n+k]) Q is the
    pairing of ybar with dy's input terms plus the initial-condition terms.
    Term by term:
        d/dgy       = dy
        d/dx[m]     = sum_{k=0..M} vb_k[m+k] ybar[m+k]
        d/dxi_j     = sum_{k=j..M} vb_k[k-j] ybar[k-j]
        d/dy[m]     = -sum_{k=1..N} va_k[m+k] ybar[m+k]
        d/dyi_j     = -sum_{k=j..N} va_k[k-j] ybar[k-j]
        d/db_k[n]   = ybar[n] vx[n-k]       (vx's history vxi)
        d/da_k[n]   = -ybar[n] dy[n-k]      (dy's history vyi)
    (time-invariant coefficients: the last two summed over n)."""
    gyc, xc, yc = _chan(gy, layout), _chan(x, layout), _chan(y, layout)
    B, T = gyc.shape
    M = 0 if b is None else _f64(b).shape[-1] - 1
    N = 0 if a is None else _f64(a).shape[-1]
    tv = int((a is not None and _f64(a).ndim == 3) or (b is not None and _f64(b).ndim == 3))
    ar = _rows(a, B, T, layout)
    var, vbr = _rows(va, B, T, layout), _rows(vb, B, T, layout)
    vxc = _chan(vx, layout)
    vxi, vyi = _f64(vxi), _f64(vyi)
    # adjoint of gy (the all-pole part of the backward)
    yb = np.zeros((B, T))
    for n in range(T - 1, -1, -1):
        acc = gyc[:, n].copy()
        for k in range(1, N + 1):
            if n + k < T:
                acc -= ar[:, n + k, k - 1] * yb[:, n + k]
        yb[:, n] = acc
    dy = _chan(jvp(x, y, a, b, xi, yi, dx=vx, da=va, db=vb, dxi=vxi, dyi=vyi,
                   layout=layout), layout)
    out = {"gy": _out_sig(dy, layout)}
    gx = np.zeros((B, T))
    gyo = np.zeros((B, T))
    for m in range(T):
        for k in range(M + 1):
            if vbr is not None and m + k < T:
                gx[:, m] += vbr[:, m + k, k] * yb[:, m + k]
        for k in range(1, N + 1):
            if var is not None and m + k < T:
                gyo[:, m] -= var[:, m + k, k - 1] * yb[:, m + k]
    out["x"] = _out_sig(gx, layout)
    out["y"] = _out_sig(gyo, layout)
    if b is not None:
        gxi = np.zeros((B, M))
        gb = np.zeros((B, T, M + 1))
        for j in range(1, M + 1):
            for k in range(j, M + 1):
                if vbr is not None and k - j < T:
                    gxi[:, j - 1] += vbr[:, k - j, k] * yb[:, k - j]
        zeros = np.zeros((B, T))
        for n in range(T):
            for k in range(M + 1):
                gb[:, n, k] = yb[:, n] * _back(vxc if vxc is not None else zeros, vxi, n - k)
        out["b"] = _out_rows(gb, tv, layout)
        out["xi"] = gxi
    if N > 0:
        gyi = np.zeros((B, N))
        ga = np.zeros((B, T, N))
        for j in range(1, N + 1):
            for k in range(j, N + 1):
                if var is not None and k - j < T:
                    gyi[:, j - 1] -= var[:, k - j, k - 1] * yb[:, k - j]
        for n in range(T):
            for k in range(1, N + 1):
                ga[:, n, k - 1] = -yb[:, n] * _back(dy, vyi, n - k)
        out["a"] = _out_rows(ga, tv, layout)
        out["yi"] = gyi
    return out


def backward2_frames(gy, x, y, a, b=None, xi=None, yi=None, vx=None, va=None, vb=None,
                     vxi=None, vyi=None, hop=1, layout="BT"):
    """backward2 with frame-held a, b (and their cotangents va, vb, one row
    per frame): a frame's gradient row is the sum of its samples' rows, so
    its cotangent applies to every sample of the frame; the a / b outputs
    are summed per frame."""
    x = _f64(x)
    T = x.shape[0] if layout == "TB" else x.shape[1]
    ex = lambda c: None if c is None else frame_expand(c, T, hop, layout)
    g = backward2(gy, x, y, ex(a), ex(b), xi, yi, vx=vx, va=ex(va), vb=ex(vb), vxi=vxi, vyi=vyi,
                  layout=layout)
    for k in ("a", "b"):
        if k in g:
            g[k] = frame_reduce(g[k], hop, layout)
    return g


# ---------------------------------------------------------------------------
# Matrix recurrence: the state-space recursion of Sec. 2 Eq. 4 with the input
# already in state space, the operator of App. B, batched over channels:
#   v(n+1) = A v(n) + z(n),  n = 0 .. T-1,  v(0) = v0,
# output v(1) .. v(T).  Backward (Sec. 3.1 Eqs. 7 and 9 for this operator):
# the adjoint of the input runs the same recursion with A transposed in
# reverse time, gz(n) = gv(n) + A^T gz(n+1) with gz(T) = 0; then
# gv0 = A^T gz(0) and gA = sum_n gz(n) v(n)^T (v(0) = v0).
#
# Shapes: A [B, K, K] (v_i(n+1) = sum_j A[b, i, j] v_j(n) + z_i(n)); v0 [B, K]
# or None (zero); z, v, gv, gz [B, T, K] (layout "BT") or [T, B, K] ("TB").


def _mr_chan(s, layout):
    return s if layout == "BT" else s.transpose(1, 0, 2)


def mr_forward(A, v0, z, layout="BT"):
    """v(1..T) of the matrix recurrence (FP64)."""
    A, z = _f64(A), _mr_chan(_f64(z), layout)
    B, T, K = z.shape
    v = np.zeros((B, T, K))
    cur = np.zeros((B, K)) if v0 is None else _f64(v0).copy()
    for n in range(T):
        cur = np.einsum("bij,bj->bi", A, cur) + z[:, n]
        v[:, n] = cur
    return np.ascontiguousarray(_mr_chan(v, layout))


def mr_backward(gv, A, v0, v, layout="BT"):
    """Gradients {z, A, v0} of <gv, v> for the matrix recurrence; v is the
    forward's output."""
    A, gv, v = _f64(A), _mr_chan(_f64(gv), layout), _mr_chan(_f64(v), layout)
    B, T, K = gv.shape
    v0 = np.zeros((B, K)) if v0 is None else _f64(v0)
    gz = np.zeros((B, T, K))
    acc = np.zeros((B, K))
    for n in range(T - 1, -1, -1):
        acc = gv[:, n] + np.einsum("bji,bj->bi", A, acc)
        gz[:, n] = acc
    gA = np.zeros((B, K, K))
    for n in range(T):
        prev = v0 if n == 0 else v[:, n - 1]
        gA += gz[:, n, :, None] * prev[:, None, :]
    gv0 = np.einsum("bji,bj->bi", A, gz[:, 0]) if T > 0 else np.zeros((B, K))
    return {"z": np.ascontiguousarray(_mr_chan(gz, layout)), "A": gA, "v0": gv0}
