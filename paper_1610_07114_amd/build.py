"""Build libtclbm.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "libtclbm.so")
SOURCES = ["tclbm_kernels.hip", "tclbm_api.hip"]
HEADERS = ["tclbm_internal.h", "tclbm_node.h"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
    # multiply-adds fused only within one source expression: every kernel path
    # (march, single-row strips, batch) rounds a node's arithmetic identically
    "-ffp-contract=on",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False, out: str = None, defines=()) -> str:
    """Compile every HIP source into paper_1610_07114_amd/_lib/libtclbm.so (or
    `out`, with extra -D definitions, for kernel-variant comparisons)."""
    os.makedirs(LIBDIR, exist_ok=True)
    target = out or LIB
    tmp = target + ".tmp"
    cmd = [_hipcc(), *HIPCC_FLAGS, *[f"-D{d}" for d in defines], "-I", os.path.join(HERE, "..", "include"),
           "-o", tmp, *[os.path.join(CSRC, s) for s in SOURCES]]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(" ".join(cmd))
    os.replace(tmp, target)
    return target


def source_digest() -> str:
    """SHA-256 over the kernel sources, headers and flags: identifies the
    kernel build that a stored profile or counter measurement belongs to."""
    import hashlib
    h = hashlib.sha256(" ".join(HIPCC_FLAGS).encode())
    for name in SOURCES + HEADERS:
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(HERE, "..", "include", "tclbm.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, s) for s in SOURCES + HEADERS]
    deps.append(os.path.join(HERE, "..", "include", "tclbm.h"))
    return any(os.path.getmtime(d) > t for d in deps)


if __name__ == "__main__":
    print(build(verbose=True))
