"""Build step for libpdhg.so (gfx950) -- run by __graft_entry__.build().

Each source is compiled to an object by its own hipcc process (in parallel),
then the objects are linked into the shared library."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpdhg.so")
SOURCES = [os.path.join(CSRC, f) for f in ("kernels.hip", "fishnet.hip", "noalloc.hip", "capi.cpp")]
HEADERS = [os.path.join(CSRC, f) for f in ("pdhg_internal.h", "sweep.h", "kernels.h")] + \
    [os.path.join(ROOT, "include", "pdhg.h")]
OBJDIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compiles every source (incremental: only those whose object is older
    than the source or any header) and links libpdhg.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    objs, procs = [], []
    newest_header = max(os.path.getmtime(h) for h in HEADERS)
    for src in SOURCES:
        obj = os.path.join(OBJDIR, os.path.splitext(os.path.basename(src))[0] + ".o")
        objs.append(obj)
        if incremental and os.path.exists(obj) and \
                os.path.getmtime(obj) > max(os.path.getmtime(src), newest_header):
            continue
        lang = [] if src.endswith(".hip") else ["-x", "hip"]
        cmd = [HIPCC] + FLAGS + inc + ["-c"] + lang + [src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = False
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out)
            failed = True
    if failed:
        raise RuntimeError("hipcc failed compiling libpdhg sources")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libpdhg.so")
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))
