"""Compile the HIP library (gfx950) in-tree: paper_1603_08114_amd/librsvhmc.so."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("rsv_kernels.hip", "rsv_capi.hip", "rsv_mlp.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("rsv_device.h", "rsv_exp.h", "rsv_internal.h")] + \
          [os.path.join(ROOT, "include", f) for f in ("rsv_hmc.h", "rsv_mlp.h")]
LIB = os.path.join(PKG, "librsvhmc.so")
ARCH = "gfx950"


def hipcc_cmd(out=LIB, extra=()):
    return (["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
             "-o", out] + list(extra) + SOURCES)


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = hipcc_cmd(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def up_to_date() -> bool:
    if not os.path.exists(LIB):
        return False
    t = os.path.getmtime(LIB)
    return all(os.path.getmtime(f) <= t for f in SOURCES + HEADERS)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
