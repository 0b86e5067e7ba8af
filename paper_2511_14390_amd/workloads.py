"""Seeded synthetic inputs shaped like the paper's filtering workloads.

This module only draws inputs: it holds none of the filtering arithmetic and
is shared by the FP64 oracle side and the HIP side of every test and of the
benchmark.  All draws use ``numpy.random.default_rng(seed)`` in FP64 and are
rounded to FP32 at the end; the oracle consumes the same FP32-rounded values.

Recipes (sign convention ``A(z) = 1 + sum_k a_k z^-k``, paper Eq. 1):

* ``pole_pair_section(r, theta)`` gives ``[1, -2 r cos(theta), r^2]``.
* ``reflection_to_direct(k)``: the step-up recursion
  ``a^(m)_i = a^(m-1)_i + k_m a^(m-1)_{m-i}``, ``a^(m)_m = k_m``.
* ``bandwidth_expand(a, rho_max)``: ``a_k <- gamma^k a_k`` with
  ``gamma = min(1, rho_max / rho)``, ``rho`` the largest pole radius of the
  frame, so every frame's poles lie within ``rho_max``.
* Per-sample coefficients are frame-held: one draw per frame of ``hop``
  samples, repeated over the frame (the last frame truncated).  With
  ``frames=True`` the generators return the frame rows themselves
  (``ceil(T / hop)`` rows per channel) from the same draws instead.
* Initial conditions ``N(0, 0.1)`` use 0.1 as the standard deviation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

F32 = np.float32


def pole_pair_section(r, theta):
    """Second-order denominator [1, a1, a2] for the conjugate pole pair r*exp(+-i theta)."""
    r = np.asarray(r, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    return np.stack([np.ones_like(r), -2.0 * r * np.cos(theta), r * r], axis=-1)


def poly_mul(p, q):
    """Product of polynomials in z^-1 given as [..., deg+1] coefficient arrays."""
    out = np.zeros(p.shape[:-1] + (p.shape[-1] + q.shape[-1] - 1,))
    for i in range(p.shape[-1]):
        for j in range(q.shape[-1]):
            out[..., i + j] += p[..., i] * q[..., j]
    return out


def reflection_to_direct(k):
    """Step-up recursion: reflection coefficients [..., N] -> a_1..a_N [..., N]."""
    k = np.asarray(k, dtype=np.float64)
    N = k.shape[-1]
    a = np.zeros(k.shape)
    for m in range(1, N + 1):
        prev = a[..., : m - 1].copy()
        km = k[..., m - 1]
        for i in range(1, m):
            a[..., i - 1] = prev[..., i - 1] + km * prev[..., m - i - 1]
        a[..., m - 1] = km
    return a


def max_pole_radius(a):
    """Largest |root| of z^N + a_1 z^(N-1) + ... + a_N for a [..., N] (batched)."""
    a = np.asarray(a, dtype=np.float64)
    N = a.shape[-1]
    if N == 0:
        return np.zeros(a.shape[:-1])
    flat = a.reshape(-1, N)
    comp = np.zeros((flat.shape[0], N, N))
    comp[:, 0, :] = -flat
    if N > 1:
        idx = np.arange(N - 1)
        comp[:, idx + 1, idx] = 1.0
    ev = np.linalg.eigvals(comp)
    return np.abs(ev).max(axis=-1).reshape(a.shape[:-1])


def bandwidth_expand(a, rho_max=0.99):
    """Scale every pole radius of each frame so that it is at most rho_max."""
    a = np.asarray(a, dtype=np.float64)
    rho = max_pole_radius(a)
    gamma = np.minimum(1.0, rho_max / np.maximum(rho, 1e-300))
    powers = gamma[..., None] ** np.arange(1, a.shape[-1] + 1)
    return a * powers


def frame_held(frames, T, hop, axis):
    """Repeat frame values hop times along `axis` and cut to length T."""
    return np.repeat(frames, hop, axis=axis).take(np.arange(T), axis=axis)


@dataclass
class Problem:
    """One filtering problem: FP32 numpy inputs plus their description."""

    name: str
    layout: str                 # "TB" or "BT"
    x: np.ndarray
    a: np.ndarray
    b: np.ndarray | None = None
    xi: np.ndarray | None = None
    yi: np.ndarray | None = None
    gy: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def B(self):
        return self.x.shape[1] if self.layout == "TB" else self.x.shape[0]

    @property
    def T(self):
        return self.x.shape[0] if self.layout == "TB" else self.x.shape[1]

    @property
    def N(self):
        return self.a.shape[-1]

    @property
    def M(self):
        return 0 if self.b is None else self.b.shape[-1] - 1

    @property
    def time_varying(self):
        return self.a.ndim == 3


def _f32(v):
    return None if v is None else np.ascontiguousarray(np.asarray(v, dtype=F32))


def _reflection_frames(rng, lead_shape, F, N, hop, T, axis, rho_max=0.99, expand=True):
    k = rng.uniform(-0.9, 0.9, lead_shape[:axis] + (F,) + lead_shape[axis:] + (N,))
    a = bandwidth_expand(reflection_to_direct(k), rho_max)
    return frame_held(a, T, hop, axis) if expand else a


def config1(B=4, T=4096, seed=1001):
    """Time-invariant order-2 all-pole, b=[1]; poles r~U[.5,.95], theta~U[0,pi];
    x~N(0,1); y[-1], y[-2] ~ N(0, 0.1); layout [B, T]."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.5, 0.95, B)
    th = rng.uniform(0.0, math.pi, B)
    a = pole_pair_section(r, th)[:, 1:]
    x = rng.standard_normal((B, T))
    yi = rng.normal(0.0, 0.1, (B, 2))
    gy = rng.standard_normal((B, T))
    return Problem("lti-allpole-n2", "BT", _f32(x), _f32(a), None, None, _f32(yi), _f32(gy),
                   {"seed": seed})


def config2(B=64, T=48000, N=16, hop=240, seed=1002, frames=False):
    """Per-sample all-pole (LPC-like): per channel and frame of `hop` samples,
    reflection coefficients U(-0.9, 0.9) -> step-up -> bandwidth expansion to
    radius 0.99, held over the frame; x~N(0,1); zero initial state; [B, T].
    frames=True: a holds the [B, ceil(T / hop), N] frame rows."""
    rng = np.random.default_rng(seed)
    F = -(-T // hop)
    a = _reflection_frames(rng, (B,), F, N, hop, T, axis=1, expand=not frames)
    x = rng.standard_normal((B, T))
    gy = rng.standard_normal((B, T))
    return Problem("ltv-allpole-n16", "BT", _f32(x), _f32(a), None, None, None, _f32(gy),
                   {"seed": seed, "hop": hop, "frames": frames})


def config3(B=1024, T=65536, seed=1003):
    """Time-invariant M=N=4: two conjugate pole pairs per channel, r~U[.3,.98],
    theta~U[0,pi]; b_k~N(0,1); x~N(0,1); x and y initial conditions ~N(0,0.1);
    channel-interleaved layout [T, B]."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.3, 0.98, (B, 2))
    th = rng.uniform(0.0, math.pi, (B, 2))
    den = poly_mul(pole_pair_section(r[:, 0], th[:, 0]), pole_pair_section(r[:, 1], th[:, 1]))
    a = den[:, 1:]
    b = rng.standard_normal((B, 5))
    x = rng.standard_normal((T, B))
    xi = rng.normal(0.0, 0.1, (B, 4))
    yi = rng.normal(0.0, 0.1, (B, 4))
    gy = rng.standard_normal((T, B))
    return Problem("lti-df-m4n4", "TB", _f32(x), _f32(a), _f32(b), _f32(xi), _f32(yi), _f32(gy),
                   {"seed": seed})


def config4(B=2, T=1 << 22, seed=1004):
    """Long narrow signals: time-invariant all-pole N=4, two pole pairs with
    r~U[.9,.99], theta~U[0,pi]; x~N(0,1); zero initial conditions; [B, T]."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.9, 0.99, (B, 2))
    th = rng.uniform(0.0, math.pi, (B, 2))
    den = poly_mul(pole_pair_section(r[:, 0], th[:, 0]), pole_pair_section(r[:, 1], th[:, 1]))
    a = den[:, 1:]
    x = rng.standard_normal((B, T))
    gy = rng.standard_normal((B, T))
    return Problem("lti-allpole-n4-long", "BT", _f32(x), _f32(a), None, None, None, _f32(gy),
                   {"seed": seed})


@dataclass
class Segments:
    """Packed variable-length batch of independent all-pole filters (M = 0)."""

    T: np.ndarray            # [S] int64 lengths
    N: np.ndarray            # [S] int32 orders
    x_off: np.ndarray        # [S] int64 offsets into x / y / gy
    a_off: np.ndarray        # [S] int64 offsets into the packed per-sample a
    ic_off: np.ndarray       # [S] int64 offsets into yi
    x: np.ndarray            # [sum T] f32
    a: np.ndarray            # packed f32, per segment [T_i, N_i] row-major at a_off
    yi: np.ndarray           # [sum N] f32
    gy: np.ndarray           # [sum T] f32
    meta: dict = field(default_factory=dict)

    @property
    def rows(self):
        """Coefficient rows per segment: T_i, or ceil(T_i / hop) frames."""
        if self.meta.get("frames"):
            h = int(self.meta["hop"])
            return (self.T + h - 1) // h
        return self.T

    def segment(self, i):
        t, n, r = int(self.T[i]), int(self.N[i]), int(self.rows[i])
        xo, ao, io = int(self.x_off[i]), int(self.a_off[i]), int(self.ic_off[i])
        return (self.x[xo:xo + t], self.a[ao:ao + r * n].reshape(r, n), self.yi[io:io + n],
                self.gy[xo:xo + t])


def config5(nseg=512, Tmin=1000, Tmax=200000, orders=(1, 2, 4, 8, 16), hop=128, seed=1005,
            frames=False):
    """Batched uneven filters: T_i ~ U{Tmin..Tmax}, N_i uniform over `orders`,
    per-sample coefficients from frame-held reflection coefficients
    U(-0.9, 0.9) with `hop`, bandwidth-expanded to radius 0.99; x~N(0,1);
    y initial conditions ~N(0, 0.1).  frames=True: each segment's block holds
    its ceil(T_i / hop) frame rows instead of T_i sample rows."""
    rng = np.random.default_rng(seed)
    T = rng.integers(Tmin, Tmax + 1, nseg).astype(np.int64)
    N = rng.choice(np.asarray(orders), nseg).astype(np.int32)
    x_off = np.concatenate([[0], np.cumsum(T)[:-1]]).astype(np.int64)
    R = (T + hop - 1) // hop if frames else T
    # coefficient blocks start on 16-byte boundaries (multiples of 4 floats)
    a_len = (R * N + 3) // 4 * 4
    a_off = np.concatenate([[0], np.cumsum(a_len)[:-1]]).astype(np.int64)
    ic_off = np.concatenate([[0], np.cumsum(N)[:-1]]).astype(np.int64)
    x = np.empty(int(T.sum()), dtype=F32)
    gy = np.empty(int(T.sum()), dtype=F32)
    a = np.zeros(int(a_len.sum()), dtype=F32)
    yi = np.empty(int(N.sum()), dtype=F32)
    for i in range(nseg):
        t, n = int(T[i]), int(N[i])
        F = -(-t // hop)
        ai = _reflection_frames(rng, (), F, n, hop, t, axis=0, expand=not frames)
        a[a_off[i]:a_off[i] + ai.size] = ai.reshape(-1)
        x[x_off[i]:x_off[i] + t] = rng.standard_normal(t)
        yi[ic_off[i]:ic_off[i] + n] = rng.normal(0.0, 0.1, n)
        gy[x_off[i]:x_off[i] + t] = rng.standard_normal(t)
    return Segments(T, N, x_off, a_off, ic_off, x, a, yi, gy,
                    {"seed": seed, "hop": hop, "nseg": nseg, "frames": frames})


def random_problem(seed, B, T, M, N, time_varying, layout, rho_max=0.95, hop=8,
                   with_xi=True, with_yi=True, with_b=True, frames=False):
    """Small random stable problem for parity tests.  Time-invariant
    denominators come from random pole pairs (plus one real pole for odd N);
    per-sample ones from frame-held reflection coefficients (frames=True:
    the frame rows themselves, ceil(T / hop) per channel)."""
    rng = np.random.default_rng(seed)
    if time_varying:
        axis = 0 if layout == "TB" else 1
        F = -(-T // hop)
        R = F if frames else T
        held = (lambda v: v) if frames else (lambda v: frame_held(v, T, hop, axis))
        if N > 0:
            k = rng.uniform(-0.9, 0.9, ((F, B) if axis == 0 else (B, F)) + (N,))
            a = held(bandwidth_expand(reflection_to_direct(k), rho_max))
        else:
            a = np.zeros(((R, B) if axis == 0 else (B, R)) + (0,))
        bf = rng.standard_normal(((F, B) if axis == 0 else (B, F)) + (M + 1,))
        b = held(bf)
    else:
        den = np.ones((B, 1))
        for _ in range(N // 2):
            r = rng.uniform(0.2, rho_max, B)
            th = rng.uniform(0.0, math.pi, B)
            den = poly_mul(den, pole_pair_section(r, th))
        if N % 2:
            p = rng.uniform(-rho_max, rho_max, B)
            den = poly_mul(den, np.stack([np.ones(B), -p], -1))
        a = den[:, 1:]
        b = rng.standard_normal((B, M + 1))
    x = rng.standard_normal((T, B) if layout == "TB" else (B, T))
    gy = rng.standard_normal(x.shape)
    if not with_b:
        if M != 0:
            raise ValueError("with_b=False needs M == 0")
        b = None
    xi = rng.normal(0.0, 0.1, (B, M)) if (with_xi and M > 0) else None
    yi = rng.normal(0.0, 0.1, (B, N)) if (with_yi and N > 0) else None
    return Problem(f"rand-s{seed}", layout, _f32(x), _f32(a), _f32(b), _f32(xi), _f32(yi),
                   _f32(gy), {"seed": seed, "hop": hop if frames else 1, "frames": frames})
