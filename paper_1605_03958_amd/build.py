"""Build libsscn.so (gfx950 HIP kernels + C-ABI runtime) in-tree with hipcc.

Every source compiles to an object under _build/ in parallel and the objects
link into paper_1605_03958_amd/libsscn.so.  Packed-FP32 instruction
selection is disabled for all device code.

``build_host_sanitized(out)`` links a copy whose host runtime (the C-ABI
sources) is built with AddressSanitizer and UndefinedBehaviorSanitizer on
the host pass only, beside the regular kernel objects, for the CPU
sanitizer test; it loads only under the sanitizer runtime (LD_PRELOAD).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libsscn.so")
ARCH = os.environ.get("SSCN_OFFLOAD_ARCH", "gfx950")

SOURCES = ["sscn_kernels.hip", "sscn_sym.hip", "sscn_batch.hip", "sscn_api.cpp", "sscn_batch_api.cpp"]
HOST_SOURCES = ["sscn_api.cpp", "sscn_batch_api.cpp"]
# host pass only: each sanitizer flag follows its own -Xarch_host
HOST_SANITIZE = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined".split() + \
    ["-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall"]


def _compile(src: str, verbose: bool, extra=(), build_dir: str = BUILD) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = ["hipcc", "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + list(extra)
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the packed-FP32 feature flag: drop that note
    noise = "is not a recognized feature for this target"
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
    if msg.strip() and verbose:
        print(msg, flush=True)
    return obj


def build(verbose: bool = False, jobs: int = 4) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build_host_sanitized(out: str, verbose: bool = False) -> str:
    """Kernel objects as built by build() (compiled here if absent) plus the
    host runtime compiled with the host-pass sanitizers, linked to `out`."""
    san_dir = os.path.join(BUILD, "host_sanitized")
    os.makedirs(san_dir, exist_ok=True)
    kern = [s for s in SOURCES if s not in HOST_SOURCES]
    objs = [os.path.join(BUILD, s + ".o") for s in kern]
    missing = [s for s, o in zip(kern, objs) if not os.path.exists(o)]
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(lambda s: _compile(s, verbose), missing))
        objs += list(ex.map(lambda s: _compile(s, verbose, HOST_SANITIZE, san_dir), HOST_SOURCES))
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-shared-libasan"] + HOST_SANITIZE + \
        ["-o", out] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
