"""Build libfilt.so (gfx950) in place from csrc/*.hip.

Each translation unit is compiled by hipcc in parallel, then linked into
``paper_2511_14390_amd/libfilt.so``.  Object files go to ``_build/`` next to
the package (not tracked).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import re
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libfilt.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


BUCKETS = (1, 2, 4, 8, 16, 32)
TYPES = (("float", "float"), ("float", "double"), ("double", "double"))


def _unit(name, header, body):
    path = os.path.join(BUILD, name)
    text = f"#define FILT_INSTANTIATING 1\n#include \"{header}\"\nnamespace filt_detail {{ {body} }}\n"
    if not os.path.exists(path) or open(path).read() != text:
        with open(path, "w") as f:
            f.write(text)
    return path


def _instantiation_units():
    """Generated translation units, one per (bucket, types, direction): the
    fully unrolled kernels of the large buckets dominate compile time, so they
    are spread over as many parallel hipcc processes as possible."""
    out = []
    for w in BUCKETS:
        for io in ("float", "double"):
            out.append(_unit(f"summary_w{w}_{io}_fwd.hip", "summary.h",
                             f"template filt_status fwd_summary_w<{w}, {io}>(const Dims &, "
                             f"const {io} *, const {io} *, const {io} *, const {io} *, double *, "
                             f"double *, hipStream_t);"))
            out.append(_unit(f"summary_w{w}_{io}_bwd.hip", "summary.h",
                             f"template filt_status bwd_summary_w<{w}, {io}>(const Dims &, "
                             f"const {io} *, const {io} *, const {io} *, double *, double *, "
                             f"hipStream_t);"))
        for io, acc in TYPES:
            out.append(_unit(f"apply_w{w}_{io}_{acc}_fwd.hip", "apply.h",
                             f"FILT_DECLARE_FWD({w}, {io}, {acc}, )"))
            out.append(_unit(f"apply_w{w}_{io}_{acc}_bwd.hip", "apply.h",
                             f"FILT_DECLARE_BWD({w}, {io}, {acc}, )"))
    for w in (1, 2, 4, 8, 16):
        out.append(_unit(f"batched_w{w}.hip", "batched.h", f"FILT_DECLARE_BATCHED({w}, )"))
    return out


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip"))) + _instantiation_units()


def _headers():
    return glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(INCLUDE, "*.h"))


def _compile(src, incremental=False):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj):
        newest = max(os.path.getmtime(p) for p in [src] + _headers())
        if os.path.getmtime(obj) >= newest:
            return obj, 0.0
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{msg}")
    return obj, time.time() - t0


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every translation unit (incremental=True skips objects newer
    than their sources and all headers -- a development shortcut)."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), os.cpu_count() or 1, 16)
    # longest units first so the pool stays busy
    def cost(p):
        m = re.search(r"_w(\d+)", os.path.basename(p))
        return -int(m.group(1)) if m else 0

    srcs.sort(key=cost)
    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda p: _compile(p, incremental), srcs))
    if verbose:
        for (obj, dt) in results:
            print(f"  {os.path.basename(obj)}: {dt:.1f}s", flush=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    t = time.time()
    build(verbose=True, incremental="--incremental" in sys.argv)
    print(f"built {LIB} in {time.time() - t:.1f}s", file=sys.stderr)
