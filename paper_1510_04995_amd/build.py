"""Build ``libgirih.so`` (HIP, gfx950) in-tree.

Every ``csrc/*.hip`` file is compiled to an object in parallel, then linked
into ``paper_1510_04995_amd/libgirih.so``.  Flags that matter for results:

* ``-ffp-contract=off``: no multiply-add fusion, so every kernel evaluates the
  listings' left-to-right order exactly (blocked == naive bit for bit);
* ``-Xclang -target-feature -Xclang -packed-fp32-ops``: no packed FP32 math.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgirih.so")
ARCH = os.environ.get("GIRIH_OFFLOAD_ARCH", "gfx950")

CFLAGS = ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(os.path.dirname(HERE), "include")]


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _headers():
    inc = os.path.join(os.path.dirname(HERE), "include")
    return [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")] + \
        [os.path.join(inc, f) for f in os.listdir(inc) if f.endswith(".h")]


def build(jobs=None, verbose=False, incremental=False):
    """Compile all HIP sources and link the shared library; returns its path.

    incremental: keep an object that is newer than its source and every
    header (a development shortcut; the default recompiles everything)."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    srcs = sources()
    jobs = jobs or min(8, os.cpu_count() or 4)
    newest_header = max(os.path.getmtime(h) for h in _headers())

    def compile_one(src):
        obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
        if incremental and os.path.exists(obj) and \
                os.path.getmtime(obj) > max(newest_header, os.path.getmtime(src)):
            return obj
        cmd = [hipcc] + CFLAGS + ["-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), r.stderr[-4000:]))
        if verbose:
            print("compiled", os.path.basename(src), flush=True)
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr[-4000:]))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
