"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/filt.h, and rejects bad arguments on the host (before any
GPU work is queued)."""
import ctypes

import numpy as np
import os
import re

import pytest

from paper_2511_14390_amd import filt as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "filt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(filt_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(F.LIB_PATH):
        pytest.skip("libfilt.so not built")
    return F.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("filt_forward", "filt_backward", "filt_workspace_bytes", "filt_forward_f64",
              "filt_backward_f64", "filt_strerror", "filt_last_error", "filt_auto_chunk"):
        assert n in names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def _prob(**kw):
    d = dict(B=4, T=100, M=0, N=2, time_varying=0, layout=1, flags=0, chunk=0)
    d.update(kw)
    return F.FiltProblem(d["B"], d["T"], d["M"], d["N"], d["time_varying"], d["layout"],
                         d["flags"], d["chunk"])


def _ws(L, p):
    n = ctypes.c_size_t(0)
    rc = L.filt_workspace_bytes(ctypes.byref(p), ctypes.byref(n))
    return rc, n.value


def test_workspace_query(L):
    rc, n = _ws(L, _prob())
    assert rc == F.FILT_OK and n > 0
    rc, n = _ws(L, _prob(B=0))
    assert rc == F.FILT_OK and n == 0
    # grows with the problem
    _, small = _ws(L, _prob(T=1000, time_varying=1, N=16))
    _, big = _ws(L, _prob(T=100000, time_varying=1, N=16))
    assert big > small


@pytest.mark.parametrize("kw,code", [
    (dict(B=-1), F.FILT_EINVAL),
    (dict(T=-5), F.FILT_EINVAL),
    (dict(N=-1), F.FILT_EINVAL),
    (dict(N=17), F.FILT_EUNSUPPORTED),
    (dict(M=20), F.FILT_EUNSUPPORTED),
    (dict(layout=7), F.FILT_EINVAL),
    (dict(time_varying=-1), F.FILT_EINVAL),
    (dict(time_varying=3, T=1 << 31), F.FILT_EUNSUPPORTED),
    (dict(chunk=48), F.FILT_EINVAL),
    (dict(flags=0x80), F.FILT_EINVAL),
])
def test_invalid_problems_rejected(L, kw, code):
    rc, _ = _ws(L, _prob(**kw))
    assert rc == code
    assert L.filt_last_error().decode() != ""


def test_forward_argument_errors_on_host(L):
    p = _prob()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: rejected before any launch
    # NULL x
    rc = L.filt_forward(ctypes.byref(p), None, None, fake, None, None, fake, fake,
                        ctypes.c_size_t(1 << 20), None)
    assert rc == F.FILT_EINVAL
    # b NULL with M > 0
    p2 = _prob(M=2)
    rc = L.filt_forward(ctypes.byref(p2), fake, None, fake, None, None, fake, fake,
                        ctypes.c_size_t(1 << 20), None)
    assert rc == F.FILT_EINVAL
    # a NULL with N > 0
    rc = L.filt_forward(ctypes.byref(p), fake, None, None, None, None, fake, fake,
                        ctypes.c_size_t(1 << 20), None)
    assert rc == F.FILT_EINVAL
    # y NULL
    rc = L.filt_forward(ctypes.byref(p), fake, None, fake, None, None, None, fake,
                        ctypes.c_size_t(1 << 20), None)
    assert rc == F.FILT_EINVAL
    # workspace too small / missing
    rc = L.filt_forward(ctypes.byref(p), fake, None, fake, None, None, fake, fake,
                        ctypes.c_size_t(8), None)
    assert rc == F.FILT_EWORKSPACE
    rc = L.filt_forward(ctypes.byref(p), fake, None, fake, None, None, fake, None,
                        ctypes.c_size_t(1 << 20), None)
    assert rc == F.FILT_EWORKSPACE
    # empty problems are no-ops even with NULL buffers
    p0 = _prob(T=0)
    assert L.filt_forward(ctypes.byref(p0), None, None, None, None, None, None, None,
                          ctypes.c_size_t(0), None) == F.FILT_OK


def test_backward_argument_errors_on_host(L):
    p = _prob(M=1)
    fake = ctypes.c_void_p(0x1000)
    args = [fake] * 12
    # gb requested but b NULL
    a = list(args)
    a[3] = None  # b
    rc = L.filt_backward(ctypes.byref(p), *a, fake, ctypes.c_size_t(1 << 20), None)
    assert rc == F.FILT_EINVAL
    # ga requested but y NULL
    a = list(args)
    a[2] = None  # y
    rc = L.filt_backward(ctypes.byref(p), *a, fake, ctypes.c_size_t(1 << 20), None)
    assert rc == F.FILT_EINVAL
    # NULL gy
    a = list(args)
    a[0] = None
    rc = L.filt_backward(ctypes.byref(p), *a, fake, ctypes.c_size_t(1 << 20), None)
    assert rc == F.FILT_EINVAL


def test_strerror(L):
    assert L.filt_strerror(F.FILT_OK).decode() == "ok"
    assert "workspace" in L.filt_strerror(F.FILT_EWORKSPACE).decode()


def test_auto_chunk_multiple_of_32(L):
    for B, T in ((1, 10), (4, 4096), (64, 48000), (1024, 65536), (2, 1 << 22)):
        c = L.filt_auto_chunk(ctypes.byref(_prob(B=B, T=T)))
        assert c >= 32 and c % 32 == 0


def test_auto_chunk_order16_per_sample_by_layout(L):
    # [T, B]: chunks of at least 16 N; [B, T]: 12 N (16 N = 256 rows of 64
    # bytes would be a power-of-two stride between a wavefront's chains)
    p = dict(B=64, T=48000, N=16, time_varying=1)
    tb = L.filt_auto_chunk(ctypes.byref(_prob(layout=F.FILT_LAYOUT_TB, **p)))
    bt = L.filt_auto_chunk(ctypes.byref(_prob(layout=F.FILT_LAYOUT_BT, **p)))
    assert (tb, bt) == (256, 192)
    # orders up to 8 keep 12 N in both layouts
    p8 = dict(B=64, T=48000, N=8, time_varying=1)
    assert L.filt_auto_chunk(ctypes.byref(_prob(layout=F.FILT_LAYOUT_TB, **p8))) == 96


def test_profile_filter_is_host_only_and_bounds_the_name(L):
    L.filt_profile_only.argtypes = [ctypes.c_char_p]
    L.filt_profile_only.restype = ctypes.c_int
    try:
        assert L.filt_profile_only(b"fwd_summary") == F.FILT_OK
        assert L.filt_profile_only(b"x" * 63) == F.FILT_OK
        assert L.filt_profile_only(b"x" * 64) == F.FILT_EINVAL
        assert b"63" in L.filt_last_error()
    finally:
        assert L.filt_profile_only(None) == F.FILT_OK


def test_python_binding_refuses_cpu_tensors():
    import torch

    x = torch.zeros(2, 10)
    a = torch.zeros(2, 2)
    with pytest.raises(ValueError):
        F.filt_forward(x, a)


def test_plan_create_rejects_bad_segments_on_host(L):
    F._plan_lib()
    h = ctypes.c_void_p(0)
    bad_order = (F.FiltSegment * 1)(F.FiltSegment(0, 100, 0, 0, 17, 0))
    assert L.filt_plan_create(bad_order, 1, None, ctypes.byref(h)) == F.FILT_EUNSUPPORTED
    bad_len = (F.FiltSegment * 1)(F.FiltSegment(0, -1, 0, 0, 2, 0))
    assert L.filt_plan_create(bad_len, 1, None, ctypes.byref(h)) == F.FILT_EINVAL
    bad_hop = (F.FiltSegment * 1)(F.FiltSegment(0, 100, 0, 0, 2, -3))
    assert L.filt_plan_create(bad_hop, 1, None, ctypes.byref(h)) == F.FILT_EINVAL
    bad_chunk = (ctypes.c_int32 * 5)(48, 64, 64, 64, 64)
    ok = (F.FiltSegment * 1)(F.FiltSegment(0, 100, 0, 0, 2, 0))
    assert L.filt_plan_create(ok, 1, (ctypes.c_int32 * 5)(-2, 64, 64, 64, 64),
                              ctypes.byref(h)) == F.FILT_EINVAL
    ok = (F.FiltSegment * 1)(F.FiltSegment(0, 100, 0, 0, 2, 0))
    assert L.filt_plan_create(ok, 1, bad_chunk, ctypes.byref(h)) == F.FILT_EINVAL
    assert L.filt_plan_create(ok, 1, None, None) == F.FILT_EINVAL


def test_frame_held_workspace_query(L):
    # time_varying = h >= 2: rows at frame rate; same workspace rules as per
    # sample (the adjoint is staged for the per-frame gradient reduction)
    for h in (2, 128, 240, 100000):
        rc, n = _ws(L, _prob(T=48000, N=16, time_varying=h))
        assert rc == F.FILT_OK and n > 0, h


def test_frame_division_is_exact():
    # the kernels find a sample's frame as (t * m) >> (31 + l) with
    # l = ceil(log2 h), m = ceil(2^(31+l) / h); exact for every t < 2^31
    rng = np.random.default_rng(4)
    hops = [2, 3, 5, 7, 100, 128, 240, 1000, 4095, 65537, (1 << 30) + 3, (1 << 31) - 1]
    ts = np.concatenate([np.arange(0, 5000), rng.integers(0, 1 << 31, 200000),
                         [(1 << 31) - 1, (1 << 31) - 2]]).astype(np.uint64)
    for h in hops:
        l = max(int(h - 1).bit_length(), 1)
        m = ((1 << (31 + l)) + h - 1) // h
        assert m < (1 << 32)
        q = ((ts * np.uint64(m)) >> np.uint64(32)) >> np.uint64(l - 1)
        assert np.array_equal(q, ts // np.uint64(h)), h


def test_empty_backward_is_ok_on_host(L):
    # B == 0, or T == 0 with no per-channel gradient requested: nothing to
    # write and nothing launched (T == 0 with gxi / gyi / ga / gb zero-fills
    # them on the stream; that case runs in the GPU tests)
    for kw in (dict(B=0), dict(T=0)):
        p = _prob(M=1, **kw)
        rc = L.filt_backward(ctypes.byref(p), *([None] * 12), None, ctypes.c_size_t(0), None)
        assert rc == F.FILT_OK, kw
    p = _prob(B=0, T=0, M=1)
    fake = ctypes.c_void_p(0x1000)  # B == 0: never touched
    rc = L.filt_backward(ctypes.byref(p), *([fake] * 12), None, ctypes.c_size_t(0), None)
    assert rc == F.FILT_OK


def test_plan_api_is_all_pole(L):
    # the batched plan covers filters with b = [1] (M = 0) and per-sample or
    # frame-held coefficients: its segment descriptor has no FIR order and the
    # plan calls take no b / xi / gb / gxi
    F._plan_lib()
    fields = [f[0] for f in F.FiltSegment._fields_]
    assert fields == ["x_off", "T", "a_off", "ic_off", "N", "hop"]
    assert len(L.filt_plan_forward.argtypes) == 6
    assert len(L.filt_plan_backward.argtypes) == 9


def test_backward2_checks_arguments_on_host(L):
    L.filt_backward2_workspace_bytes.argtypes = [ctypes.POINTER(F.FiltProblem),
                                                 ctypes.POINTER(ctypes.c_size_t)]
    L.filt_backward2.argtypes = ([ctypes.POINTER(F.FiltProblem)] + [ctypes.c_void_p] * 19
                                 + [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p])
    n = ctypes.c_size_t(7)
    assert L.filt_backward2_workspace_bytes(ctypes.byref(_prob(T=0)), ctypes.byref(n)) == 0
    assert n.value == 0
    # the workspace holds the passes' own workspaces and three signals
    p = _prob(B=4, T=1000, M=2, N=3)
    assert L.filt_backward2_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == 0
    wf = ctypes.c_size_t(0)
    assert L.filt_workspace_bytes(ctypes.byref(p), ctypes.byref(wf)) == 0
    assert n.value >= 3 * 4 * 1000 * 4
    fake = ctypes.c_void_p(0x1000)  # rejected before any access

    def call(p, **given):
        names = ("gy", "x", "y", "b", "a", "xi", "yi", "vx", "vb", "va", "vxi", "vyi", "wgy",
                 "wx", "wy", "wb", "wa", "wxi", "wyi")
        args = [given.get(k) for k in names]
        return L.filt_backward2(ctypes.byref(p), *args, None, ctypes.c_size_t(0), None)

    # b = [1] (NULL) with a cotangent or gradient for b
    q = _prob(M=0, N=2)
    assert call(q, gy=fake, a=fake, vb=fake) == F.FILT_EINVAL
    assert call(q, gy=fake, a=fake, wb=fake) == F.FILT_EINVAL
    # no feedback part but va / wa given
    q = _prob(M=1, N=0)
    assert call(q, gy=fake, b=fake, va=fake) == F.FILT_EINVAL
    # a missing with N > 0
    assert call(_prob(M=0, N=2), gy=fake) == F.FILT_EINVAL
    # B == 0: nothing to do
    assert call(_prob(B=0, M=0, N=2), gy=fake, a=fake, wgy=fake) == F.FILT_OK
    # workspace too small
    assert call(_prob(M=0, N=2), gy=fake, a=fake, wgy=fake) == F.FILT_EWORKSPACE
