"""Thin ctypes binding of libfilt.so (``include/filt.h``).

Argument marshalling only: every step of the filter runs in the HIP library.
Tensors must live on the GPU; PyTorch provides the memory, the workspace and
the current HIP stream.  If the library has not been built the first call
raises -- there is no CPU fallback.

Shapes (same as the C ABI): layout ``"TB"`` signals ``[T, B]``, ``"BT"``
signals ``[B, T]``; ``a`` is ``[B, N]`` or per-sample ``[T, B, N]`` /
``[B, T, N]``; ``b`` likewise with ``M + 1`` taps (``None`` means ``b = [1]``);
``xi`` ``[B, M]``, ``yi`` ``[B, N]`` (``None`` means zero).
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfilt.so")

FILT_OK, FILT_EINVAL, FILT_EUNSUPPORTED, FILT_EWORKSPACE, FILT_EHIP = range(5)
FILT_LAYOUT_TB, FILT_LAYOUT_BT = 0, 1
FILT_F32_STATE = 0x2
FILT_RECURRENCE = 0x4
FILT_TOEPLITZ = 0x8


class FiltProblem(ctypes.Structure):
    _fields_ = [("B", ctypes.c_int64), ("T", ctypes.c_int64), ("M", ctypes.c_int32),
                ("N", ctypes.c_int32), ("time_varying", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("flags", ctypes.c_int32), ("chunk", ctypes.c_int32)]


class FiltError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                               "(python -m paper_2511_14390_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P, S, I64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64
        PP = ctypes.POINTER(FiltProblem)
        L.filt_workspace_bytes.argtypes = [PP, ctypes.POINTER(ctypes.c_size_t)]
        L.filt_workspace_bytes.restype = ctypes.c_int
        L.filt_auto_chunk.argtypes = [PP]
        L.filt_auto_chunk.restype = I64
        for name in ("filt_forward", "filt_forward_f64"):
            f = getattr(L, name)
            f.argtypes = [PP] + [P] * 6 + [P, S, P]
            f.restype = ctypes.c_int
        for name in ("filt_backward", "filt_backward_f64"):
            f = getattr(L, name)
            f.argtypes = [PP] + [P] * 12 + [P, S, P]
            f.restype = ctypes.c_int
        L.filt_strerror.argtypes = [ctypes.c_int]
        L.filt_strerror.restype = ctypes.c_char_p
        L.filt_last_error.argtypes = []
        L.filt_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status):
    if status != FILT_OK:
        L = lib()
        raise FiltError(status, f"{L.filt_strerror(status).decode()}: "
                                f"{L.filt_last_error().decode()}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _layout_code(layout):
    if layout == "TB":
        return FILT_LAYOUT_TB
    if layout == "BT":
        return FILT_LAYOUT_BT
    raise ValueError("layout must be 'TB' or 'BT'")


def problem(x, a, b=None, layout="BT", chunk=0, f32_state=False, recurrence=False,
            toeplitz=False, hop=1):
    """Build the filt_problem for these tensors (shapes checked here).
    Coefficients with a time axis are per sample (hop = 1) or frame-held:
    hop >= 2 samples per row, ceil(T / hop) rows per channel."""
    if x.dim() != 2:
        raise ValueError("x must be 2-D")
    hop = int(hop)
    if hop < 1:
        raise ValueError("hop must be >= 1")
    T, B = (x.shape[0], x.shape[1]) if layout == "TB" else (x.shape[1], x.shape[0])
    N = 0 if a is None else a.shape[-1]
    M = 0 if b is None else b.shape[-1] - 1
    tv = (a is not None and a.dim() == 3) or (b is not None and b.dim() == 3)
    if hop > 1 and not tv:
        raise ValueError("hop > 1 needs coefficients with a time axis")
    R = -(-T // hop)
    for c, K in ((a, N), (b, M + 1)):
        if c is None:
            continue
        want = (B, K) if not tv else ((R, B, K) if layout == "TB" else (B, R, K))
        if tuple(c.shape) != want:
            raise ValueError(f"coefficient shape {tuple(c.shape)} != {want}")
    flags = ((FILT_F32_STATE if f32_state else 0) | (FILT_RECURRENCE if recurrence else 0)
             | (FILT_TOEPLITZ if toeplitz else 0))
    p = FiltProblem(B, T, M, N, hop if tv else 0, _layout_code(layout), flags, int(chunk))
    return p


def _prep(t, dtype, device, name):
    if t is None:
        return None
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return t.contiguous()


def workspace_bytes(p):
    n = ctypes.c_size_t(0)
    _check(lib().filt_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    return n.value


def auto_chunk(p):
    return int(lib().filt_auto_chunk(ctypes.byref(p)))


def _workspace(p, device, ws):
    need = workspace_bytes(p)
    if ws is not None and ws.numel() >= need:
        return ws, need
    return torch.empty(max(need, 1), dtype=torch.uint8, device=device), need


def _stream(device, stream):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def filt_forward(x, a, b=None, xi=None, yi=None, *, layout="BT", chunk=0, f32_state=False,
                 recurrence=False, toeplitz=False, hop=1, out=None, ws=None, stream=None):
    """y = direct-form filter of x (see include/filt.h).  Returns y.
    hop >= 2: a and b hold one row per frame of hop samples."""
    dev, dt = x.device, x.dtype
    if dt not in (torch.float32, torch.float64):
        raise ValueError("x must be float32 or float64")
    if dev.type != "cuda":
        raise ValueError("filt_forward runs on the GPU only")
    x = x.contiguous()
    a, b, xi, yi = (_prep(t, dt, dev, n) for t, n in ((a, "a"), (b, "b"), (xi, "xi"), (yi, "yi")))
    p = problem(x, a, b, layout, chunk, f32_state, recurrence, toeplitz, hop)
    y = out if out is not None else torch.empty_like(x)
    ws, need = _workspace(p, dev, ws)
    fn = lib().filt_forward_f64 if dt == torch.float64 else lib().filt_forward
    _check(fn(ctypes.byref(p), _ptr(x), _ptr(b), _ptr(a), _ptr(xi), _ptr(yi), _ptr(y), _ptr(ws),
              ctypes.c_size_t(ws.numel()), _stream(dev, stream)))
    return y


def filt_backward(gy, x, y, a, b=None, xi=None, yi=None, *, layout="BT", chunk=0,
                  f32_state=False, recurrence=False, toeplitz=False, hop=1,
                  want=("x", "a", "b", "xi", "yi"), ws=None, stream=None):
    """Closed-form gradients (see include/filt.h).  Returns a dict with the
    requested keys among x, a, b, xi, yi (b only if b was given; xi / yi
    always have shapes [B, M] / [B, N]; with hop >= 2 the a / b gradients
    have one row per frame, like a and b)."""
    dev, dt = gy.device, gy.dtype
    if dev.type != "cuda":
        raise ValueError("filt_backward runs on the GPU only")
    gy = gy.contiguous()
    x, y, a, b, xi, yi = (_prep(t, dt, dev, n) for t, n in
                          ((x, "x"), (y, "y"), (a, "a"), (b, "b"), (xi, "xi"), (yi, "yi")))
    p = problem(gy, a, b, layout, chunk, f32_state, recurrence, toeplitz, hop)
    B, M, N = p.B, p.M, p.N
    gx = torch.empty_like(gy) if "x" in want else None
    ga = torch.empty_like(a) if ("a" in want and a is not None and N > 0) else None
    gb = torch.empty_like(b) if ("b" in want and b is not None) else None
    gxi = torch.empty((B, M), dtype=dt, device=dev) if "xi" in want else None
    gyi = torch.empty((B, N), dtype=dt, device=dev) if "yi" in want else None
    ws, need = _workspace(p, dev, ws)
    fn = lib().filt_backward_f64 if dt == torch.float64 else lib().filt_backward
    _check(fn(ctypes.byref(p), _ptr(gy), _ptr(x), _ptr(y), _ptr(b), _ptr(a), _ptr(xi), _ptr(yi),
              _ptr(gx), _ptr(gb), _ptr(ga), _ptr(gxi if M > 0 else None),
              _ptr(gyi if N > 0 else None), _ptr(ws), ctypes.c_size_t(ws.numel()),
              _stream(dev, stream)))
    out = {}
    for k, v in (("x", gx), ("a", ga), ("b", gb), ("xi", gxi), ("yi", gyi)):
        if v is not None:
            out[k] = v
    return out


def filt_jvp(x, y, a, b=None, xi=None, yi=None, *, dx=None, db=None, da=None, dxi=None,
             dyi=None, layout="BT", chunk=0, hop=1, ws=None, stream=None):
    """Forward-mode derivative: the tangent of y = filt_forward(x, a, b, xi,
    yi) along the given input tangents (None = zero).  y is the forward's
    output.  See filt_jvp in include/filt.h."""
    dev = x.device
    if dev.type != "cuda":
        raise ValueError("filt_jvp runs on the GPU only")
    if x.dtype != torch.float32:
        raise ValueError("filt_jvp takes float32 tensors")
    L = lib()
    if not getattr(L, "_jvp_ready", False):
        PP, P = ctypes.POINTER(FiltProblem), ctypes.c_void_p
        L.filt_jvp_workspace_bytes.argtypes = [PP, ctypes.POINTER(ctypes.c_size_t)]
        L.filt_jvp_workspace_bytes.restype = ctypes.c_int
        L.filt_jvp.argtypes = [PP] + [P] * 12 + [P, ctypes.c_size_t, P]
        L.filt_jvp.restype = ctypes.c_int
        L._jvp_ready = True
    x = x.contiguous()
    y, a, b, xi, yi, dx, db, da, dxi, dyi = (
        _prep(t, torch.float32, dev, n) for t, n in
        ((y, "y"), (a, "a"), (b, "b"), (xi, "xi"), (yi, "yi"), (dx, "dx"), (db, "db"),
         (da, "da"), (dxi, "dxi"), (dyi, "dyi")))
    p = problem(x, a, b, layout, chunk, hop=hop)
    n = ctypes.c_size_t(0)
    _check(L.filt_jvp_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    if ws is None or ws.numel() < n.value:
        ws = torch.empty(max(n.value, 1), dtype=torch.uint8, device=dev)
    dy = torch.empty_like(x)
    _check(L.filt_jvp(ctypes.byref(p), _ptr(x), _ptr(y), _ptr(b), _ptr(a), _ptr(xi), _ptr(yi),
                      _ptr(dx), _ptr(db), _ptr(da), _ptr(dxi), _ptr(dyi), _ptr(dy), _ptr(ws),
                      ctypes.c_size_t(ws.numel()), _stream(dev, stream)))
    return dy


def filt_backward2(gy, x, y, a, b=None, xi=None, yi=None, *, vx=None, va=None, vb=None,
                   vxi=None, vyi=None, layout="BT", chunk=0, f32_state=False, toeplitz=False,
                   hop=1, want=("gy", "x", "y", "a", "b", "xi", "yi"), ws=None, stream=None):
    """Derivative of filt_backward (see filt_backward2 in include/filt.h):
    the gradients of sum_k <v_k, filt_backward(...)_k> for the cotangents
    vx, va, vb, vxi, vyi (None = zero).  Returns a dict with the requested
    keys among gy, x, y, a, b, xi, yi (b, xi only with b; a, yi only with
    N > 0)."""
    dev = gy.device
    if dev.type != "cuda":
        raise ValueError("filt_backward2 runs on the GPU only")
    if gy.dtype != torch.float32:
        raise ValueError("filt_backward2 takes float32 tensors")
    L = lib()
    if not getattr(L, "_b2_ready", False):
        PP, P = ctypes.POINTER(FiltProblem), ctypes.c_void_p
        L.filt_backward2_workspace_bytes.argtypes = [PP, ctypes.POINTER(ctypes.c_size_t)]
        L.filt_backward2_workspace_bytes.restype = ctypes.c_int
        L.filt_backward2.argtypes = [PP] + [P] * 19 + [P, ctypes.c_size_t, P]
        L.filt_backward2.restype = ctypes.c_int
        L._b2_ready = True
    gy = gy.contiguous()
    x, y, a, b, xi, yi, vx, va, vb, vxi, vyi = (
        _prep(t, torch.float32, dev, n) for t, n in
        ((x, "x"), (y, "y"), (a, "a"), (b, "b"), (xi, "xi"), (yi, "yi"), (vx, "vx"),
         (va, "va"), (vb, "vb"), (vxi, "vxi"), (vyi, "vyi")))
    p = problem(gy, a, b, layout, chunk, f32_state, False, toeplitz, hop)
    B, M, N = p.B, p.M, p.N
    out = {}
    if "gy" in want:
        out["gy"] = torch.empty_like(gy)
    if "x" in want:
        out["x"] = torch.empty_like(gy)
    if "y" in want:
        out["y"] = torch.empty_like(gy)
    if "b" in want and b is not None:
        out["b"] = torch.empty_like(b)
    if "a" in want and a is not None and N > 0:
        out["a"] = torch.empty_like(a)
    if "xi" in want and b is not None:
        out["xi"] = torch.empty((B, M), dtype=gy.dtype, device=dev)
    if "yi" in want and N > 0:
        out["yi"] = torch.empty((B, N), dtype=gy.dtype, device=dev)
    n = ctypes.c_size_t(0)
    _check(L.filt_backward2_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    if ws is None or ws.numel() < n.value:
        ws = torch.empty(max(n.value, 1), dtype=torch.uint8, device=dev)
    g = out.get
    _check(L.filt_backward2(ctypes.byref(p), _ptr(gy), _ptr(x), _ptr(y), _ptr(b), _ptr(a),
                            _ptr(xi), _ptr(yi), _ptr(vx), _ptr(vb), _ptr(va), _ptr(vxi),
                            _ptr(vyi), _ptr(g("gy")), _ptr(g("x")), _ptr(g("y")), _ptr(g("b")),
                            _ptr(g("a")), _ptr(g("xi") if M > 0 else None),
                            _ptr(g("yi") if N > 0 else None), _ptr(ws),
                            ctypes.c_size_t(ws.numel()), _stream(dev, stream)))
    return out


def _mr_lib():
    L = lib()
    if not getattr(L, "_mr_ready", False):
        PP, P = ctypes.POINTER(FiltProblem), ctypes.c_void_p
        L.filt_mr_workspace_bytes.argtypes = [PP, ctypes.POINTER(ctypes.c_size_t)]
        L.filt_mr_workspace_bytes.restype = ctypes.c_int
        L.filt_mr_forward.argtypes = [PP] + [P] * 4 + [P, ctypes.c_size_t, P]
        L.filt_mr_forward.restype = ctypes.c_int
        L.filt_mr_backward.argtypes = [PP] + [P] * 7 + [P, ctypes.c_size_t, P]
        L.filt_mr_backward.restype = ctypes.c_int
        L._mr_ready = True
    return L


def _mr_prep(A, z, layout, chunk):
    if z.dim() != 3:
        raise ValueError("z must be [B, T, K] or [T, B, K]")
    T, B = (z.shape[0], z.shape[1]) if layout == "TB" else (z.shape[1], z.shape[0])
    K = z.shape[2]
    if tuple(A.shape) != (B, K, K):
        raise ValueError(f"A must be {(B, K, K)}, got {tuple(A.shape)}")
    p = FiltProblem(B, T, 0, K, 0, _layout_code(layout), 0, int(chunk))
    L = _mr_lib()
    n = ctypes.c_size_t(0)
    _check(L.filt_mr_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    return p, L, n.value


def filt_mr_forward(A, z, v0=None, *, layout="BT", chunk=0, ws=None, stream=None):
    """Matrix recurrence v(n+1) = A v(n) + z(n) per channel (see
    filt_mr_forward in include/filt.h).  A [B, K, K]; z [B, T, K] ("BT") or
    [T, B, K] ("TB"); v0 [B, K] or None.  Returns v (the shape of z)."""
    dev = z.device
    if dev.type != "cuda" or z.dtype != torch.float32:
        raise ValueError("filt_mr_forward takes float32 tensors on the GPU")
    z = z.contiguous()
    A, v0 = (_prep(t, torch.float32, dev, n) for t, n in ((A, "A"), (v0, "v0")))
    p, L, need = _mr_prep(A, z, layout, chunk)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    v = torch.empty_like(z)
    _check(L.filt_mr_forward(ctypes.byref(p), _ptr(A), _ptr(v0), _ptr(z), _ptr(v), _ptr(ws),
                             ctypes.c_size_t(ws.numel()), _stream(dev, stream)))
    return v


def filt_mr_backward(gv, A, v, v0=None, *, layout="BT", chunk=0, want=("z", "A", "v0"),
                     ws=None, stream=None):
    """Gradients of the matrix recurrence for dL/dv = gv; v is the forward's
    output.  Returns a dict with z (always), and A / v0 if requested (v0
    only when v0 was given)."""
    dev = gv.device
    if dev.type != "cuda" or gv.dtype != torch.float32:
        raise ValueError("filt_mr_backward takes float32 tensors on the GPU")
    gv = gv.contiguous()
    A, v, v0 = (_prep(t, torch.float32, dev, n) for t, n in ((A, "A"), (v, "v"), (v0, "v0")))
    p, L, need = _mr_prep(A, gv, layout, chunk)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    gz = torch.empty_like(gv)
    gA = torch.empty_like(A) if "A" in want else None
    gv0 = torch.empty((p.B, p.N), dtype=gv.dtype, device=dev) \
        if ("v0" in want and v0 is not None) else None
    _check(L.filt_mr_backward(ctypes.byref(p), _ptr(A), _ptr(v0), _ptr(v), _ptr(gv), _ptr(gz),
                              _ptr(gA), _ptr(gv0), _ptr(ws), ctypes.c_size_t(ws.numel()),
                              _stream(dev, stream)))
    out = {"z": gz}
    if gA is not None:
        out["A"] = gA
    if gv0 is not None:
        out["v0"] = gv0
    return out


def _tdf_lib():
    L = lib()
    if not getattr(L, "_tdf_ready", False):
        PP, P = ctypes.POINTER(FiltProblem), ctypes.c_void_p
        L.filt_tdf_workspace_bytes.argtypes = [PP, ctypes.POINTER(ctypes.c_size_t)]
        L.filt_tdf_workspace_bytes.restype = ctypes.c_int
        L.filt_tdf_forward.argtypes = [PP] + [P] * 6 + [ctypes.c_size_t, P]
        L.filt_tdf_forward.restype = ctypes.c_int
        L.filt_tdf_backward.argtypes = [PP] + [P] * 11 + [ctypes.c_size_t, P]
        L.filt_tdf_backward.restype = ctypes.c_int
        L._tdf_ready = True
    return L


def _tdf_prep(x, b, a, zi, layout, chunk):
    dev = x.device
    if dev.type != "cuda":
        raise ValueError("the transposed form runs on the GPU only")
    if x.dtype != torch.float32:
        raise ValueError("the transposed form takes float32 tensors")
    if b is None or b.dim() != 2:
        raise ValueError("b must be [B, M+1] (time-invariant)")
    if a is not None and a.dim() != 2:
        raise ValueError("a must be [B, N] (time-invariant)")
    b, a, zi = (_prep(t, torch.float32, dev, n) for t, n in ((b, "b"), (a, "a"), (zi, "zi")))
    p = problem(x, a, b, layout, chunk)
    K = max(p.M, p.N, 1)
    if zi is not None and tuple(zi.shape) != (p.B, K):
        raise ValueError(f"zi must be [{p.B}, {K}], got {tuple(zi.shape)}")
    n = ctypes.c_size_t(0)
    _check(_tdf_lib().filt_tdf_workspace_bytes(ctypes.byref(p), ctypes.byref(n)))
    return p, b, a, zi, K, n.value


def filt_tdf_forward(x, b, a, zi=None, *, layout="BT", chunk=0, ws=None, stream=None):
    """Transposed direct form II with initial state zi [B, max(M, N)]
    (SciPy's lfilter(b, a, x, zi) semantics; see filt_tdf_forward in
    include/filt.h).  Returns y."""
    x = x.contiguous()
    p, b, a, zi, K, need = _tdf_prep(x, b, a, zi, layout, chunk)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
    y = torch.empty_like(x)
    _check(_tdf_lib().filt_tdf_forward(ctypes.byref(p), _ptr(x), _ptr(b), _ptr(a), _ptr(zi),
                                       _ptr(y), _ptr(ws), ctypes.c_size_t(ws.numel()),
                                       _stream(x.device, stream)))
    return y


def filt_tdf_backward(gy, x, y, b, a, zi=None, *, layout="BT", chunk=0,
                      want=("x", "b", "a", "zi"), ws=None, stream=None):
    """Gradients of the transposed direct form with respect to x, b, a, zi
    (the requested keys; a only with N > 0)."""
    gy = gy.contiguous()
    x = _prep(x, torch.float32, gy.device, "x")
    y = _prep(y, torch.float32, gy.device, "y")
    p, b, a, zi, K, need = _tdf_prep(gy, b, a, zi, layout, chunk)
    dev = gy.device
    gx = torch.empty_like(gy) if "x" in want else None
    gb = torch.empty_like(b) if "b" in want else None
    ga = torch.empty_like(a) if ("a" in want and a is not None and p.N > 0) else None
    gzi = torch.empty((p.B, K), dtype=torch.float32, device=dev) if "zi" in want else None
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _check(_tdf_lib().filt_tdf_backward(ctypes.byref(p), _ptr(gy), _ptr(x), _ptr(y), _ptr(b),
                                        _ptr(a), _ptr(zi), _ptr(gx), _ptr(gb), _ptr(ga),
                                        _ptr(gzi), _ptr(ws), ctypes.c_size_t(ws.numel()),
                                        _stream(dev, stream)))
    return {k: v for k, v in (("x", gx), ("b", gb), ("a", ga), ("zi", gzi)) if v is not None}


def _sos_lib():
    L = lib()
    if not getattr(L, "_sos_ready", False):
        PP, P, I = ctypes.POINTER(FiltProblem), ctypes.c_void_p, ctypes.c_int32
        L.filt_sos_workspace_bytes.argtypes = [PP, I, ctypes.POINTER(ctypes.c_size_t)]
        L.filt_sos_workspace_bytes.restype = ctypes.c_int
        L.filt_sos_forward.argtypes = [PP, I] + [P] * 6 + [ctypes.c_size_t, P]
        L.filt_sos_forward.restype = ctypes.c_int
        L.filt_sos_backward.argtypes = [PP, I] + [P] * 11 + [ctypes.c_size_t, P]
        L.filt_sos_backward.restype = ctypes.c_int
        L._sos_ready = True
    return L


def _sos_prep(x, b, a, zi, layout, chunk):
    dev = x.device
    if dev.type != "cuda":
        raise ValueError("the section cascade runs on the GPU only")
    if x.dtype != torch.float32:
        raise ValueError("the section cascade takes float32 tensors")
    if b.dim() != 3 or b.shape[-1] != 3 or a.dim() != 3 or a.shape[-1] != 2:
        raise ValueError("b must be [S, B, 3] and a [S, B, 2]")
    b, a, zi = (_prep(t, torch.float32, dev, n) for t, n in ((b, "b"), (a, "a"), (zi, "zi")))
    S = b.shape[0]
    p = problem(x, a[0], b[0], layout, chunk)
    if tuple(a.shape) != (S, p.B, 2) or (zi is not None and tuple(zi.shape) != (S, p.B, 2)):
        raise ValueError("a and zi must be [S, B, 2]")
    n = ctypes.c_size_t(0)
    _check(_sos_lib().filt_sos_workspace_bytes(ctypes.byref(p), S, ctypes.byref(n)))
    return p, S, b, a, zi, n.value


def filt_sos_forward(x, b, a, zi=None, *, layout="BT", chunk=0, ws=None, stream=None):
    """Cascade of second-order sections (SciPy's sosfilt per channel):
    b [S, B, 3], a [S, B, 2], zi [S, B, 2] or None.  Returns y."""
    x = x.contiguous()
    p, S, b, a, zi, need = _sos_prep(x, b, a, zi, layout, chunk)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
    y = torch.empty_like(x)
    _check(_sos_lib().filt_sos_forward(ctypes.byref(p), S, _ptr(x), _ptr(b), _ptr(a), _ptr(zi),
                                       _ptr(y), _ptr(ws), ctypes.c_size_t(ws.numel()),
                                       _stream(x.device, stream)))
    return y


def filt_sos_backward(gy, x, y, b, a, zi=None, *, layout="BT", chunk=0,
                      want=("x", "b", "a", "zi"), ws=None, stream=None):
    """Gradients of the section cascade with respect to x, b, a, zi."""
    gy = gy.contiguous()
    x = _prep(x, torch.float32, gy.device, "x")
    y = _prep(y, torch.float32, gy.device, "y")
    p, S, b, a, zi, need = _sos_prep(gy, b, a, zi, layout, chunk)
    dev = gy.device
    gx = torch.empty_like(gy) if "x" in want else None
    gb = torch.empty_like(b) if "b" in want else None
    ga = torch.empty_like(a) if "a" in want else None
    gzi = torch.empty((S, p.B, 2), dtype=torch.float32, device=dev) if "zi" in want else None
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    _check(_sos_lib().filt_sos_backward(ctypes.byref(p), S, _ptr(gy), _ptr(x), _ptr(y), _ptr(b),
                                        _ptr(a), _ptr(zi), _ptr(gx), _ptr(gb), _ptr(ga),
                                        _ptr(gzi), _ptr(ws), ctypes.c_size_t(ws.numel()),
                                        _stream(dev, stream)))
    return {k: v for k, v in (("x", gx), ("b", gb), ("a", ga), ("zi", gzi)) if v is not None}


def profile_enable(on: bool):
    """Start (True) or stop (False) per-kernel event timing inside the library."""
    L = lib()
    L.filt_profile_enable.argtypes = [ctypes.c_int]
    L.filt_profile_enable.restype = ctypes.c_int
    _check(L.filt_profile_enable(1 if on else 0))


def profile_only(name):
    """Record only launches of kernel `name` (None: every launch)."""
    L = lib()
    L.filt_profile_only.argtypes = [ctypes.c_char_p]
    L.filt_profile_only.restype = ctypes.c_int
    _check(L.filt_profile_only(None if name is None else name.encode()))


def profile_read(max_entries: int = 64):
    """{kernel name: (launches, total ms)} of the recorded launches (synchronises)."""
    L = lib()
    L.filt_profile_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    L.filt_profile_read.restype = ctypes.c_int
    names = ctypes.create_string_buffer(64 * max_entries)
    counts = (ctypes.c_int32 * max_entries)()
    ms = (ctypes.c_double * max_entries)()
    n = L.filt_profile_read(names, counts, ms, max_entries)
    out = {}
    for i in range(n):
        nm = names.raw[64 * i:64 * (i + 1)].split(b"\0", 1)[0].decode()
        out[nm] = (int(counts[i]), float(ms[i]))
    return out


# ------------------------------------------------------------------ batched


class FiltSegment(ctypes.Structure):
    _fields_ = [("x_off", ctypes.c_int64), ("T", ctypes.c_int64), ("a_off", ctypes.c_int64),
                ("ic_off", ctypes.c_int64), ("N", ctypes.c_int32), ("hop", ctypes.c_int32)]


def _plan_lib():
    L = lib()
    if not getattr(L, "_plan_ready", False):
        P, VP = ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)
        L.filt_plan_create.argtypes = [ctypes.POINTER(FiltSegment), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32), VP]
        L.filt_plan_create.restype = ctypes.c_int
        L.filt_plan_destroy.argtypes = [P]
        L.filt_plan_destroy.restype = None
        L.filt_plan_forward.argtypes = [P] * 5 + [P]
        L.filt_plan_forward.restype = ctypes.c_int
        L.filt_plan_backward.argtypes = [P] * 8 + [P]
        L.filt_plan_backward.restype = ctypes.c_int
        L.filt_plan_tune.argtypes = [P] * 9 + [P]
        L.filt_plan_tune.restype = ctypes.c_int
        L.filt_plan_capture.argtypes = [P] * 9 + [P]
        L.filt_plan_capture.restype = ctypes.c_int
        L.filt_plan_replay.argtypes = [P, P]
        L.filt_plan_replay.restype = ctypes.c_int
        L.filt_plan_get_chunks.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
        L.filt_plan_get_chunks.restype = ctypes.c_int
        L._plan_ready = True
    return L


class BatchedFilter:
    """Many independent all-pole filters with per-sample or frame-held
    coefficients, packed into flat tensors (see filt_segment in
    include/filt.h): segment i covers x[x_off[i] : x_off[i] + T[i]], its rows
    a[a_off[i] : a_off[i] + R_i*N[i]] ([R_i, N_i] row-major, R_i = T[i], or
    ceil(T[i] / hop) with hop >= 2) and yi[ic_off[i] : ic_off[i] + N[i]].
    hop is one value for every segment or a sequence of one per segment."""

    def __init__(self, T, N, x_off, a_off, ic_off, chunks=None, hop=1):
        L = _plan_lib()
        n = len(T)
        hops = [int(hop)] * n if not hasattr(hop, "__len__") else [int(h) for h in hop]
        segs = (FiltSegment * max(n, 1))()
        for i in range(n):
            segs[i] = FiltSegment(int(x_off[i]), int(T[i]), int(a_off[i]), int(ic_off[i]),
                                  int(N[i]), hops[i])
        ch = None
        if chunks is not None:
            ch = (ctypes.c_int32 * 5)(*[int(c) for c in chunks])
        h = ctypes.c_void_p(0)
        _check(L.filt_plan_create(segs, n, ch, ctypes.byref(h)))
        self._h = h
        self.nseg = n

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _plan_lib().filt_plan_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def chunks(self):
        out = (ctypes.c_int32 * 5)()
        _check(_plan_lib().filt_plan_get_chunks(self._h, out))
        return list(out)

    def forward(self, x, a, yi=None, out=None, stream=None):
        y = out if out is not None else torch.empty_like(x)
        _check(_plan_lib().filt_plan_forward(self._h, _ptr(x), _ptr(a), _ptr(yi), _ptr(y),
                                             _stream(x.device, stream)))
        return y

    def backward(self, gy, y, a, yi=None, want=("x", "a", "yi"), out=None, stream=None):
        o = out or {}
        gx = o.get("x", torch.empty_like(gy)) if "x" in want else None
        ga = o.get("a", torch.zeros_like(a)) if "a" in want else None
        gyi = (o.get("yi", torch.zeros_like(yi)) if ("yi" in want and yi is not None) else None)
        _check(_plan_lib().filt_plan_backward(self._h, _ptr(gy), _ptr(y), _ptr(a), _ptr(yi),
                                              _ptr(gx), _ptr(ga), _ptr(gyi),
                                              _stream(gy.device, stream)))
        return {k: v for k, v in (("x", gx), ("a", ga), ("yi", gyi)) if v is not None}

    def tune(self, x, a, yi, gy, stream=None):
        y = torch.empty_like(x)
        gx = torch.empty_like(x)
        ga = torch.zeros_like(a)
        gyi = torch.zeros_like(yi) if yi is not None else None
        _check(_plan_lib().filt_plan_tune(self._h, _ptr(x), _ptr(a), _ptr(yi), _ptr(gy),
                                          _ptr(y), _ptr(gx), _ptr(ga), _ptr(gyi),
                                          _stream(x.device, stream)))
        return self.chunks

    def capture(self, x, a, yi, gy, y, gx, ga, gyi, stream=None):
        """Capture forward + backward on these tensors into a HIP graph."""
        s = stream if stream is not None else torch.cuda.Stream(x.device)
        torch.cuda.current_stream(x.device).synchronize()
        _check(_plan_lib().filt_plan_capture(self._h, _ptr(x), _ptr(a), _ptr(yi), _ptr(gy),
                                             _ptr(y), _ptr(gx), _ptr(ga), _ptr(gyi),
                                             ctypes.c_void_p(s.cuda_stream)))
        s.synchronize()

    def replay(self, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(_plan_lib().filt_plan_replay(self._h, ctypes.c_void_p(s.cuda_stream)))
