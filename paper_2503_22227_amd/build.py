"""Build the HIP library ``librnsfhe.so`` in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "librnsfhe.so")
SOURCES = ["context.hip", "ntt.hip", "keyswitch.hip", "capi.hip", "profile.hip", "batch.hip", "noalloc.hip",
           "client.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # keep the compiler from forming packed fp32 operations
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]

# the host pass does not know the device feature flag; that note is harmless
_NOISE = ("is not a recognized feature for this target", "--hip-link")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    text = "\n".join(l for l in res.stdout.splitlines() if not any(n in l for n in _NOISE))
    if text.strip():
        print(text, flush=True)
    if res.returncode != 0:
        raise subprocess.CalledProcessError(res.returncode, cmd)


def build(verbose: bool = False, out: str = LIB, defines=(), jobs: int = 0) -> str:
    """Compile every source (in parallel, one object each) and link one shared
    library (next to this file by default); returns its path.  ``defines`` are
    extra -D flags (kernel variants for tuning)."""
    tag = "%d" % os.getpid()
    objs, cmds = [], []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        if not os.path.exists(src):
            continue
        obj = out + "." + s + ".o" + tag
        objs.append(obj)
        cmds.append([HIPCC] + FLAGS + ["-D" + d for d in defines] + ["-c", src, "-o", obj])
    workers = jobs or min(len(cmds), max(1, (os.cpu_count() or 2)))
    try:
        with ThreadPoolExecutor(max_workers=workers) as pool:
            for f in [pool.submit(_run, c, verbose) for c in cmds]:
                f.result()
        tmp = out + ".tmp" + tag
        _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp], verbose)
        os.replace(tmp, out)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
