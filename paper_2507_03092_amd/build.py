"""Build libstab.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "stab_api.hip")
DEPS = [os.path.join(PKG, "csrc", f) for f in ("stab_api.hip", "stab_kernels.hip", "stab_device.h",
                                                    "stab_batch.hip", "stab_batch_api.hip", "stab_commute.hip",
                                                    "stab_server_api.hip")]
HDR = os.path.join(ROOT, "include", "stab.h")
LIB = os.path.join(PKG, "libstab.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         # packed-FP32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function"]


def command(out: str = LIB) -> list:
    return [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", out, SRC]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile libstab.so; with force=False only when a source is newer than the library."""
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(p) for p in DEPS + [HDR])
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp"
    res = subprocess.run(command(tmp), capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr[-4000:])
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
