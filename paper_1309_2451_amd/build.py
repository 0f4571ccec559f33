"""Build libssf.so (HIP, gfx950) in-tree.

The pass-kernel translation unit is compiled once per supported transform
length (the SSF_LENGTHS list in csrc/ssf_internal.hpp), in parallel, then
linked with the runtime into paper_1309_2451_amd/libssf.so.

    python -m paper_1309_2451_amd.build [--jobs N]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libssf.so")
ARCH = os.environ.get("SSF_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# -packed-fp32-ops: no packed FP32 instructions in generated code.
FLAGS = ["-O3", "--offload-arch=" + ARCH, "-fPIC", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def lengths():
    src = open(os.path.join(CSRC, "ssf_internal.hpp")).read()
    m = re.search(r"#define SSF_LENGTHS\(X\)(.*?)\n\n", src, re.S)
    return [int(v) for v in re.findall(r"X\((\d+)\)", m.group(1))]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError("command failed: %s\n%s" % (" ".join(cmd), out))
    return out


def _stale(obj, deps):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def build(jobs: int | None = None, verbose: bool = False, force: bool = True, defines=(), out: str | None = None,
          build_dir: str | None = None) -> str:
    """Compile every translation unit (force=True) or only those older than
    their sources (force=False), then link libssf.so."""
    bdir = build_dir or BUILD
    lib = out or LIB
    os.makedirs(bdir, exist_ok=True)
    extra = ["-D" + d for d in defines]
    hdrs = [os.path.join(CSRC, f) for f in ("ssf_internal.hpp", "ssf_pass.hpp")]
    hdrs.append(os.path.join(os.path.dirname(HERE), "include", "ssf.h"))
    jobs = jobs or int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))
    jobs = max(1, min(jobs, 16))
    tasks = []
    for n in lengths():
        obj = os.path.join(bdir, "ssf_kernels_%d.o" % n)
        tasks.append([HIPCC] + FLAGS + extra + ["-DSSF_N=%d" % n, "-c",
                                        os.path.join(CSRC, "ssf_kernels.hip"), "-o", obj])
    rt_obj = os.path.join(bdir, "ssf_runtime.o")
    tasks.append([HIPCC] + FLAGS + extra + ["-c", os.path.join(CSRC, "ssf_runtime.hip"), "-o", rt_obj])
    todo = [t for t in tasks if force or _stale(t[-1], hdrs + [t[-3]])]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for out in ex.map(_run, todo):
            if verbose and out.strip():
                print(out)
    objs = [t[-1] for t in tasks]
    tmp = lib + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    ap.add_argument("--incremental", action="store_true", help="only recompile stale objects")
    ap.add_argument("-D", dest="defines", action="append", default=[], help="extra preprocessor define")
    ap.add_argument("--out", default=None, help="output library path (default: in the package)")
    ap.add_argument("--build-dir", default=None)
    a = ap.parse_args()
    print(build(a.jobs, a.v, force=not a.incremental, defines=a.defines, out=a.out, build_dir=a.build_dir))
    sys.exit(0)
