"""Build the HIP library libecc_mi.so (gfx950) in-tree.

    python -m paper_2501_03245_amd.build            # compile every source
    python -m paper_2501_03245_amd.build --changed  # reuse objects whose inputs are unchanged

The translation units compile in parallel; the library is linked from them.
"""

from __future__ import annotations

import glob
import hashlib
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libecc_mi.so")
OBJDIR = os.path.join(ROOT, "_build")
SOURCES = ["ecc_mi.hip", "ecdsa.hip", "tests.hip", "server.hip", "probe.hip", "noalloc.hip", "ablate.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    "-pthread",
    # packed fp32 instructions stay off in every HIP build of this project
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _inputs_digest(src: str) -> str:
    """Digest of a source, every header it may include, and the flags."""
    h = hashlib.sha256()
    h.update(" ".join(HIPCC_FLAGS).encode())
    paths = [os.path.join(CSRC, src)] + sorted(glob.glob(os.path.join(CSRC, "*.h"))) + \
        sorted(glob.glob(os.path.join(INCLUDE, "*.h")))
    for p in paths:
        with open(p, "rb") as f:
            h.update(p.encode())
            h.update(f.read())
    return h.hexdigest()[:20]


def build(verbose: bool = True, changed_only: bool = False) -> str:
    """Compile every HIP source into one shared library.  With changed_only,
    objects from an earlier build whose inputs are unchanged are reused."""
    t0 = time.time()
    os.makedirs(OBJDIR, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, f"{os.path.splitext(src)[0]}-{_inputs_digest(src)}.o")
        objs.append(obj)
        if changed_only and os.path.exists(obj):
            continue
        cmd = [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj + ".tmp"]
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), src, obj))
    failed = []
    for p, src, obj in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if p.returncode != 0:
            failed.append((src, "\n".join(lines)))
            continue
        os.replace(obj + ".tmp", obj)
        if verbose and lines:
            print("\n".join(lines[-20:]), file=sys.stderr)
    if failed:
        raise RuntimeError("HIP build failed:\n" + "\n".join(f"== {s}\n{t}" for s, t in failed))
    tmp = LIB + ".tmp"
    subprocess.check_call([hipcc(), "--offload-arch=gfx950", "-shared", "-pthread", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    # drop objects of earlier inputs
    keep = set(objs)
    for o in glob.glob(os.path.join(OBJDIR, "*.o")):
        if o not in keep:
            os.remove(o)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.0f}s", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(changed_only="--changed" in sys.argv[1:])
