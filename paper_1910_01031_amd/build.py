"""Build libiewpf.so for gfx950 with hipcc (in-tree, next to this file).

Every HIP source is compiled with packed-FP32 instruction generation disabled and linked
into one shared library that exports the C ABI of include/iewpf.h.
"""
from __future__ import annotations

import os
import shlex
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libiewpf.so")
SOURCES = ["api.cpp", "host_precompute.cpp", "surrogate_api.cpp", "swe_kernels.hip",
           "noise_kernels.hip", "analysis_kernels.hip", "surrogate_kernels.hip", "noalloc.hip"]
ARCH = os.environ.get("IEWPF_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=on: a*b+c is fused only inside one source expression, so every inlined copy
# of a formula (halo rows and interior rows of a strip, single and batched launches) rounds
# identically and results do not depend on the strip height or the launch form.
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
          "-ffp-contract=on",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(shlex.quote(c) for c in cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose: bool = False, jobs: int = 5, defines=(), out: str = LIB) -> str:
    """Compile every source and link `out`; `defines` adds -D flags (variants for tuning)."""
    build_dir = BUILD if out == LIB else out + ".objs"
    os.makedirs(build_dir, exist_ok=True)
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmds.append([HIPCC] + COMMON + [f"-D{d}" for d in defines] + lang +
                    ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        outs = list(ex.map(_run, cmds))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    tmp = out + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
