"""Build libnopcs.so (HIP, gfx950) in-tree with hipcc.

Flags: -O3, -ffp-contract=off (no FMA contraction: the FP64 path reproduces its
operation order exactly), and the packed-FP32 target feature switched off.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnopcs.so")
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = ["api.hip", "sweep.hip", "march.hip", "dmarch.hip", "visc.hip", "cvisc.hip", "diag.hip", "plan.cpp"]
OPTIONAL_SOURCES = ["mixed.hip", "batch.hip", "solver.cpp"]
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]


def hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def sources():
    out = [os.path.join(CSRC, s) for s in SOURCES]
    out += [os.path.join(CSRC, s) for s in OPTIONAL_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    return out


def _newest_header():
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    hdrs.append(os.path.join(os.path.dirname(HERE), "include", "nopcs.h"))
    return max(os.path.getmtime(h) for h in hdrs if os.path.exists(h))


def _compile(src, verbose, incremental=False):
    os.makedirs(BUILD_DIR, exist_ok=True)
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj) and \
            os.path.getmtime(obj) > max(os.path.getmtime(src), _newest_header()):
        return obj
    cmd = [hipcc()] + HIP_FLAGS + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    before = _snapshot(src)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
    if _snapshot(src) != before:
        # hipcc reads the sources once for the device pass and once for the host
        # pass: an edit in between gives host code that launches kernels the
        # device code object does not hold
        os.remove(obj)
        raise RuntimeError("%s or a header changed while it was compiled; build again" % src)
    return obj


def _snapshot(src):
    """Contents of a source and of every header it may include."""
    files = [src] + sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h")))
    files.append(os.path.join(os.path.dirname(HERE), "include", "nopcs.h"))
    out = []
    for f in files:
        with open(f, "rb") as fh:
            out.append(fh.read())
    return out


def build(verbose=False, jobs=None, incremental=False):
    """Compile every source and link libnopcs.so (incremental=True reuses up-to-date objects)."""
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)), 8)
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, incremental), srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
