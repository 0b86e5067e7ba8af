"""``torch.autograd.Function`` over the C ABI: differentiable direct-form filter.

Forward calls ``filt_forward``; forward-mode AD (dual tensors of
``torch.autograd.forward_ad``) calls ``filt_jvp``; backward calls
``filt_backward`` (the closed-form adjoint of Sec. 3.1 Eqs. 7-9 run in
reverse time, fused with the gradient reductions).  Only the inputs and the output ``y`` are saved: in the
direct form the filter state at any chunk boundary is a slice of ``y``
(the last N outputs) and of ``x``, so nothing else needs to be stored and the
backward recomputes everything else from them.  Gradients are requested only
for the inputs that need them (``ctx.needs_input_grad``).  The backward is
itself differentiable (``LFilterGrad``, FP32): its backward is
``filt_backward2``, so ``create_graph=True`` gives Hessian-vector products
by reverse over reverse.
"""
from __future__ import annotations

import torch
from torch.autograd.function import once_differentiable

from . import filt as _f


class LFilter(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, a, b, xi, yi, layout, chunk, f32_state, toeplitz, hop):
        y = _f.filt_forward(x, a, b, xi, yi, layout=layout, chunk=chunk, f32_state=f32_state,
                            toeplitz=toeplitz, hop=hop)
        ctx.save_for_backward(x, a, b, xi, yi, y)
        ctx.save_for_forward(x, a, b, xi, yi, y)
        ctx.cfg = (layout, chunk, f32_state, toeplitz, hop)
        return y

    @staticmethod
    def jvp(ctx, dx, da, db, dxi, dyi, *_):
        # forward mode: the tangent of y is the same recursion run on the
        # tangent input (filt_jvp)
        x, a, b, xi, yi, y = ctx.saved_tensors
        layout, chunk, _, _, hop = ctx.cfg
        return _f.filt_jvp(x, y, a, b, xi, yi, dx=dx, db=db, da=da, dxi=dxi, dyi=dyi,
                           layout=layout, chunk=chunk, hop=hop)

    @staticmethod
    def backward(ctx, gy):
        x, a, b, xi, yi, y = ctx.saved_tensors
        need = ctx.needs_input_grad
        want = tuple(k for k, n in zip(("x", "a", "b", "xi", "yi"), need[:5]) if n)
        if not want:
            return (None,) * 10
        if torch.is_grad_enabled():
            # create_graph: a differentiable call whose backward is
            # filt_backward2 (y's gradient flows on through this filter)
            gx, ga, gb, gxi, gyi = LFilterGrad.apply(gy, x, y, a, b, xi, yi, ctx.cfg, want)
        else:
            layout, chunk, f32_state, toeplitz, hop = ctx.cfg
            g = _f.filt_backward(gy, x, y, a, b, xi, yi, layout=layout, chunk=chunk,
                                 f32_state=f32_state, toeplitz=toeplitz, hop=hop, want=want)
            gx, ga, gb, gxi, gyi = (g.get(k) for k in ("x", "a", "b", "xi", "yi"))
        return (gx, ga, gb if b is not None else None, gxi if xi is not None else None,
                gyi if yi is not None else None, None, None, None, None, None)


class LFilterGrad(torch.autograd.Function):
    """The backward of LFilter as a function of (gy, x, y, a, b, xi, yi):
    forward filt_backward, backward filt_backward2 (FP32)."""

    @staticmethod
    def forward(ctx, gy, x, y, a, b, xi, yi, cfg, want):
        layout, chunk, f32_state, toeplitz, hop = cfg
        g = _f.filt_backward(gy, x, y, a, b, xi, yi, layout=layout, chunk=chunk,
                             f32_state=f32_state, toeplitz=toeplitz, hop=hop, want=want)
        ctx.save_for_backward(gy, x, y, a, b, xi, yi)
        ctx.cfg = cfg
        ctx.set_materialize_grads(False)
        return tuple(g.get(k) for k in ("x", "a", "b", "xi", "yi"))

    @staticmethod
    @once_differentiable
    def backward(ctx, vx, va, vb, vxi, vyi):
        gy, x, y, a, b, xi, yi = ctx.saved_tensors
        layout, chunk, f32_state, toeplitz, hop = ctx.cfg
        names = ("gy", "x", "y", "a", "b", "xi", "yi")
        want = tuple(k for k, n in zip(names, ctx.needs_input_grad[:7]) if n)
        if not want or all(v is None for v in (vx, va, vb, vxi, vyi)):
            return (None,) * 9
        if gy.dtype != torch.float32:
            raise NotImplementedError("second derivatives run in FP32 only")
        N = 0 if a is None else a.shape[-1]
        M = 0 if b is None else b.shape[-1] - 1
        # cotangents of outputs that are empty carry nothing
        vxi = vxi if (vxi is not None and M > 0) else None
        vyi = vyi if (vyi is not None and N > 0) else None
        w = _f.filt_backward2(gy, x, y, a, b, xi, yi, vx=vx, va=va, vb=vb, vxi=vxi, vyi=vyi,
                              layout=layout, chunk=chunk, f32_state=f32_state,
                              toeplitz=toeplitz, hop=hop, want=want)
        out = [w.get(k) for k in names]
        # inputs that were not given (None) get no gradient
        for i, t in enumerate((gy, x, y, a, b, xi, yi)):
            if t is None:
                out[i] = None
        return tuple(out) + (None, None)


def lfilter(x, a, b=None, xi=None, yi=None, layout="BT", chunk=0, f32_state=False,
            toeplitz=False, hop=1):
    """Differentiable y[n] = sum_k b_k[n] x[n-k] - sum_k a_k[n] y[n-k].

    ``a`` / ``b`` may be per-channel ``[B, K]``, per-sample (the signal
    layout plus a trailing tap axis) or, with ``hop >= 2``, frame-held: one
    row per frame of ``hop`` samples in place of the time axis
    (``ceil(T / hop)`` rows), whose gradients are summed over each frame.
    Coefficients shared across channels can be passed as ``c.expand(B, K)``;
    autograd sums the per-channel gradients.
    """
    if a is not None:
        a = a.contiguous()
    if b is not None:
        b = b.contiguous()
    if xi is not None:
        xi = xi.contiguous()
    if yi is not None:
        yi = yi.contiguous()
    return LFilter.apply(x.contiguous(), a, b, xi, yi, layout, int(chunk), bool(f32_state),
                         bool(toeplitz), int(hop))


class TDFilter(torch.autograd.Function):
    """Transposed direct form II with an initial state (SciPy's lfilter with
    zi), time-invariant: forward filt_tdf_forward, backward filt_tdf_backward
    for the inputs that need gradients.  Saves the inputs and y."""

    @staticmethod
    def forward(ctx, x, b, a, zi, layout, chunk):
        y = _f.filt_tdf_forward(x, b, a, zi, layout=layout, chunk=chunk)
        ctx.save_for_backward(x, b, a, zi, y)
        ctx.cfg = (layout, chunk)
        return y

    @staticmethod
    @once_differentiable
    def backward(ctx, gy):
        x, b, a, zi, y = ctx.saved_tensors
        layout, chunk = ctx.cfg
        need = ctx.needs_input_grad
        want = [k for k, n in zip(("x", "b", "a", "zi"), need[:4]) if n]
        if not want:
            return (None,) * 6
        g = _f.filt_tdf_backward(gy, x, y, b, a, zi, layout=layout, chunk=chunk,
                                 want=tuple(want))
        return (g.get("x"), g.get("b"), g.get("a") if a is not None else None,
                g.get("zi") if zi is not None else None, None, None)


def lfilter_tdf(x, b, a, zi=None, layout="BT", chunk=0):
    """Differentiable transposed direct form II: SciPy's
    ``lfilter(b, a, x, zi=zi)`` per channel, b ``[B, M+1]``, a ``[B, N]``
    (a_0 = 1 implied), zi ``[B, max(M, N)]`` or None."""
    return TDFilter.apply(x.contiguous(), b.contiguous(), None if a is None else a.contiguous(),
                          None if zi is None else zi.contiguous(), layout, int(chunk))


class SOSFilter(torch.autograd.Function):
    """Cascade of second-order sections (SciPy's sosfilt with per-section
    initial states), time-invariant: forward filt_sos_forward, backward
    filt_sos_backward.  Saves the inputs and y."""

    @staticmethod
    def forward(ctx, x, b, a, zi, layout, chunk):
        y = _f.filt_sos_forward(x, b, a, zi, layout=layout, chunk=chunk)
        ctx.save_for_backward(x, b, a, zi, y)
        ctx.cfg = (layout, chunk)
        return y

    @staticmethod
    @once_differentiable
    def backward(ctx, gy):
        x, b, a, zi, y = ctx.saved_tensors
        layout, chunk = ctx.cfg
        need = ctx.needs_input_grad
        want = [k for k, n in zip(("x", "b", "a", "zi"), need[:4]) if n]
        if not want:
            return (None,) * 6
        g = _f.filt_sos_backward(gy, x, y, b, a, zi, layout=layout, chunk=chunk,
                                 want=tuple(want))
        return (g.get("x"), g.get("b"), g.get("a"), g.get("zi") if zi is not None else None,
                None, None)


def sosfilt(x, b, a, zi=None, layout="BT", chunk=0):
    """Differentiable cascade of second-order sections: b ``[S, B, 3]``,
    a ``[S, B, 2]`` (a_0 = 1 implied), zi ``[S, B, 2]`` or None; per
    channel SciPy's ``sosfilt``."""
    return SOSFilter.apply(x.contiguous(), b.contiguous(), a.contiguous(),
                           None if zi is None else zi.contiguous(), layout, int(chunk))


class MatrixRecurrence(torch.autograd.Function):
    """v(n+1) = A v(n) + z(n) per channel (the operator of App. B): forward
    filt_mr_forward, backward filt_mr_backward (the same recursion with A
    transposed in reverse time, then gA and gv0).  Saves A, v0 and v."""

    @staticmethod
    def forward(ctx, A, v0, z, layout, chunk):
        v = _f.filt_mr_forward(A, z, v0, layout=layout, chunk=chunk)
        ctx.save_for_backward(A, v0, v)
        ctx.cfg = (layout, chunk)
        return v

    @staticmethod
    @once_differentiable
    def backward(ctx, gv):
        A, v0, v = ctx.saved_tensors
        layout, chunk = ctx.cfg
        need = ctx.needs_input_grad
        if not any(need[:3]):
            return (None,) * 5
        want = tuple(k for k, n in zip(("A", "v0"), need[:2]) if n)
        g = _f.filt_mr_backward(gv, A, v, v0, layout=layout, chunk=chunk, want=want)
        return (g.get("A"), g.get("v0") if v0 is not None else None,
                g["z"] if need[2] else None, None, None)


def matrix_recurrence(A, z, v0=None, layout="BT", chunk=0):
    """Differentiable v(1..T) of v(n+1) = A v(n) + z(n), v(0) = v0, per
    channel: A [B, K, K], z [B, T, K] ("BT") or [T, B, K] ("TB"),
    v0 [B, K] or None; 1 <= K <= 16."""
    return MatrixRecurrence.apply(A.contiguous(), None if v0 is None else v0.contiguous(),
                                  z.contiguous(), layout, int(chunk))
