"""Build libmessi.so (HIP for gfx950) next to this file.

Usage: python -m paper_2009_00786_amd.build   (or call build()).
Each source is compiled to an object in _build/ in parallel, then linked.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build", "messi")
LIB = os.path.join(HERE, "libmessi.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("MESSI_ARCH", "gfx950")

SOURCES = ["api.cpp", "breakpoints.cpp", "scan.hip", "build.hip", "query.hip", "bf16.hip", "server.cpp", "noalloc.hip"]
HEADERS = ["common.h", "scan.h", "query.h"]

# -packed-fp32-ops: keep the compiler from emitting packed fp32 ALU instructions.
COMMON_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC,
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-Wall", "-Wno-unused-function", "-Wno-pass-failed"]


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJDIR, src + ".o")
    cmd = [HIPCC, "--offload-arch=" + ARCH] + COMMON_FLAGS + ["-c", path, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "hip", "--offload-arch=" + ARCH] + COMMON_FLAGS + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), out))
    if out.strip():
        sys.stderr.write(out + "\n")
    return obj


def build(force: bool = True, jobs: int = 8) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    deps = [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(INCLUDE, "messi.h")]
    newest_dep = max(os.path.getmtime(d) for d in deps)
    todo = []
    for s in SOURCES:
        obj = os.path.join(OBJDIR, s + ".o")
        src = os.path.join(CSRC, s)
        if force or not os.path.exists(obj) or os.path.getmtime(obj) < max(os.path.getmtime(src), newest_dep):
            todo.append(s)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, todo))
    del objs
    all_objs = [os.path.join(OBJDIR, s + ".o") for s in SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + all_objs + ["-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
