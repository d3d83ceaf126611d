"""Compile the HIP library (gfx950) in-tree: paper_1603_08114_amd/librsvhmc.so.

Each translation unit compiles in its own hipcc process (in parallel), then
one hipcc call links the shared library.
"""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
SOURCES = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
HEADERS = sorted(glob.glob(os.path.join(CSRC, "*.h"))) + \
          [os.path.join(ROOT, "include", f) for f in ("rsv_hmc.h", "rsv_mlp.h")]
LIB = os.path.join(PKG, "librsvhmc.so")
OBJ_DIR = os.path.join(PKG, "_build")
ARCH = "gfx950"
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def hipcc_cmd(out=LIB, extra=()):
    """One-step build of the whole library (used by tools that pass extra flags)."""
    return ["hipcc"] + FLAGS + ["-shared", "-o", out] + list(extra) + SOURCES


def _obj(src):
    return os.path.join(OBJ_DIR, os.path.basename(src).replace(".hip", ".o"))


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4, 8)

    def compile_one(src):
        cmd = ["hipcc"] + FLAGS + ["-c", "-o", _obj(src), src]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        noise = "'-packed-fp32-ops' is not a recognized feature"
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if noise not in l)
        if msg.strip():
            print(msg, flush=True)
        return r.returncode, src

    with ThreadPoolExecutor(jobs) as ex:
        for rc, src in ex.map(compile_one, SOURCES):
            if rc != 0:
                raise subprocess.CalledProcessError(rc, f"hipcc -c {src}")
    tmp = LIB + ".tmp"
    link = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + \
           [_obj(s) for s in SOURCES]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
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
