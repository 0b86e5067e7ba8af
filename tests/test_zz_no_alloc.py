"""GPU test of filt_forward_noalloc: the forward with its workspace in the
library's static device scratch instead of a caller buffer, called through
the C ABI and checked against filt_forward (same kernels, so equal bit for
bit) on two calls in a row, the second on a smaller problem."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2511_14390_amd import filt as F
from paper_2511_14390_amd import workloads as W

pytestmark = pytest.mark.gpu


def _noalloc():
    L = F.lib()
    fn = L.filt_forward_noalloc
    fn.argtypes = [ctypes.POINTER(F.FiltProblem)] + [ctypes.c_void_p] * 7
    fn.restype = ctypes.c_int
    return fn


def _run(fn, p, dev, chunk):
    t = lambda v: None if v is None else torch.from_numpy(np.ascontiguousarray(v)).to(dev)
    x, a, b, xi, yi = map(t, (p.x, p.a, p.b, p.xi, p.yi))
    prob = F.problem(x, a, b, p.layout, chunk)
    y = torch.full_like(x, float("nan"))
    s = torch.cuda.current_stream(dev)
    rc = fn(ctypes.byref(prob), *(F._ptr(v) for v in (x, b, a, xi, yi, y)),
            ctypes.c_void_p(s.cuda_stream))
    assert rc == F.FILT_OK, F.lib().filt_last_error().decode()
    ref = F.filt_forward(x, a, b, xi, yi, layout=p.layout, chunk=chunk)
    torch.cuda.synchronize()
    return y, ref


def test_noalloc_forward_matches_workspace_forward(gpu_device):
    fn = _noalloc()
    # per-sample order 16 (summaries, carry and applies all use the scratch)
    big = W.random_problem(8100, B=16, T=20000, M=0, N=16, time_varying=True, layout="BT",
                           hop=128, rho_max=0.99, with_b=False)
    y, ref = _run(fn, big, gpu_device, chunk=192)
    assert torch.equal(y, ref)
    # a smaller problem of another shape on the same scratch right after
    small = W.random_problem(8101, B=3, T=1500, M=2, N=5, time_varying=True, layout="TB",
                             hop=16, rho_max=0.99)
    y, ref = _run(fn, small, gpu_device, chunk=64)
    assert torch.equal(y, ref)


def test_noalloc_rejects_problems_beyond_the_scratch(gpu_device):
    fn = _noalloc()
    prob = F.FiltProblem(64, 1 << 22, 0, 16, 1, F.FILT_LAYOUT_BT, 0, 32)
    fake = ctypes.c_void_p(0x1000)  # rejected on the host, never dereferenced
    rc = fn(ctypes.byref(prob), fake, None, fake, None, None, fake, None)
    assert rc == F.FILT_EWORKSPACE
    assert b"static scratch" in F.lib().filt_last_error()
