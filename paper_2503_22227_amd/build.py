"""Build the HIP library ``librnsfhe.so`` in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "librnsfhe.so")
SOURCES = ["context.hip", "ntt.hip", "keyswitch.hip", "capi.hip", "profile.hip", "batch.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-function",
    # keep the compiler from forming packed fp32 operations
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile every source into one shared library (next to this file by default);
    returns its path.  ``defines`` are extra -D flags (kernel variants for tuning)."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-D" + d for d in defines] + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # the host pass does not know the device feature flag; that note is harmless
    noise = "is not a recognized feature for this target"
    text = "\n".join(l for l in res.stdout.splitlines() if noise not in l and "--hip-link" not in l)
    if text.strip():
        print(text, flush=True)
    if res.returncode != 0:
        raise subprocess.CalledProcessError(res.returncode, cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
