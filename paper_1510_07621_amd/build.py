"""Build libp3m.so (the HIP force library) in-tree for gfx950.

Each ``csrc/*.hip`` file is compiled with hipcc to a position-independent
object and the objects are linked into ``paper_1510_07621_amd/libp3m.so``.
Packed FP32 instructions are disabled (``-packed-fp32-ops``); float atomics
use the hardware instructions (``-munsafe-fp-atomics``: every buffer the
library atomically updates is its own coarse-grained ``hipMalloc`` memory).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libp3m.so")
ARCH = os.environ.get("P3M_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found (ROCm is required to build libp3m.so)")
    return path


def _compile(src: str, obj: str, extra: list[str]) -> None:
    cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")


def build(verbose: bool = False, extra_flags: list[str] | None = None) -> str:
    """Compile every HIP source and link libp3m.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    extra = list(extra_flags or [])
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    objs = [os.path.join(BUILD, os.path.basename(s)[:-4] + ".o") for s in srcs]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        futs = [ex.submit(_compile, s, o, extra) for s, o in zip(srcs, objs)]
        for f in futs:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


SAN_DIR = os.path.join(BUILD, "san")
SAN_LIB = os.path.join(SAN_DIR, "libp3m_san.so")
# AddressSanitizer and UndefinedBehaviorSanitizer on the host code only (the
# ABI's validation, plan set-up and host helpers); the device code is built
# as usual.
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-g",
             "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    """The shared AddressSanitizer runtime of ROCm's clang (to preload into
    the process that loads the sanitized library)."""
    found = sorted(glob.glob(os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..",
                                          "llvm", "lib", "clang", "*", "lib", "linux",
                                          "libclang_rt.asan-x86_64.so")))
    if not found:
        found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise RuntimeError("libclang_rt.asan-x86_64.so not found")
    return os.path.realpath(found[-1])


def _sources_digest(flags: list[str]) -> str:
    import hashlib
    h = hashlib.sha256(" ".join(flags).encode())
    for pat in (os.path.join(CSRC, "*"), os.path.join(INCLUDE, "*.h")):
        for p in sorted(glob.glob(pat)):
            with open(p, "rb") as f:
                h.update(os.path.basename(p).encode())
                h.update(f.read())
    return h.hexdigest()


def build_host_sanitized(verbose: bool = False) -> str:
    """Build ``_build/san/libp3m_san.so``: the same sources with the host code
    under ASan + UBSan (host optimisation -O1). Skipped when a build of the
    same sources and flags is there. Returns the library path."""
    flags = [f for f in HIPCC_FLAGS if f != "-O3"] + ["-O1"] + SAN_FLAGS
    digest = _sources_digest(flags)
    stamp = os.path.join(SAN_DIR, "sources.sha256")
    if os.path.exists(SAN_LIB) and os.path.exists(stamp):
        with open(stamp) as f:
            if f.read().strip() == digest:
                return SAN_LIB
    os.makedirs(SAN_DIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    objs = [os.path.join(SAN_DIR, os.path.basename(s)[:-4] + ".o") for s in srcs]

    def one(src, obj):
        cmd = [hipcc(), *flags, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")

    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        for f in [ex.submit(one, s, o) for s, o in zip(srcs, objs)]:
            f.result()
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *SAN_FLAGS[:4],
           "-shared-libsan", *objs, "-o", SAN_LIB]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    with open(stamp, "w") as f:
        f.write(digest + "\n")
    if verbose:
        print(f"built {SAN_LIB}")
    return SAN_LIB


if __name__ == "__main__":
    build(verbose=True, extra_flags=sys.argv[1:])
