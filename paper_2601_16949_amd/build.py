"""Build the gfx950 shared library librttda.so in-tree with hipcc.

    python -m paper_2601_16949_amd.build [--jobs N]

Each HIP source under csrc/ is compiled to an object (in parallel), then linked into
paper_2601_16949_amd/librttda.so.  Always rebuilds.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "librttda.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


# host-side AddressSanitizer + UndefinedBehaviorSanitizer for the runtime's host code (the device
# code is built as usual); the instrumented library expects the sanitizer runtime to be preloaded
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                  "-Xarch_host", "-g"]
SAN_BUILD = os.path.join(BUILD, "sanitize")
SAN_OUT = os.path.join(SAN_BUILD, "librttda_san.so")


def compile_one(src: str, sanitize: bool = False) -> str:
    obj = os.path.join(SAN_BUILD if sanitize else BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *(SANITIZE_FLAGS if sanitize else []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    if r.stderr.strip():
        lines = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")
    return obj


def build(jobs: int = 4, verbose: bool = True, sanitize: bool = False) -> str:
    """Compile every source and link the library: paper_2601_16949_amd/librttda.so, or with
    sanitize the host-instrumented _build/sanitize/librttda_san.so (for the CPU-side ABI tests)."""
    os.makedirs(SAN_BUILD if sanitize else BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda f: compile_one(f, sanitize), srcs))
    out = SAN_OUT if sanitize else OUT
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out} from {len(srcs)} sources")
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("--sanitize", action="store_true", help="host-side ASan + UBSan build for the CPU tests")
    a = ap.parse_args()
    build(a.jobs, sanitize=a.sanitize)
