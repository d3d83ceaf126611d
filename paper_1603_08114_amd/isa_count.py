"""Instruction counts of the leapfrog loop, read from the gfx950 assembly.

Compiles csrc/rsv_traj_f64.hip and csrc/rsv_traj_f32.hip to device assembly, finds in each trajectory
kernel (identity mass, RSV terms) the loop that carries the DPP
lane shifts -- one leapfrog step over a lane's S sites -- and counts its VALU
instructions.  Dividing by S gives VALU instructions per site-update, the
per-unit figure of the ALU roofline, and its floating-point operations (an
FMA counts 2).  Writes isa_counts.json next to this file.  A measurement
tool: it reads the AMD assembly of this library's own gfx950 build.
"""
import json
import os
import re
import subprocess
import sys
import tempfile
from collections import Counter

from . import build as B

OUT = os.path.join(B.PKG, "isa_counts.json")
VARIANTS = {("f64", 4, 1): "IdLi4ELi1ELb1E", ("f64", 4, 2): "IdLi4ELi2ELb1E",
            ("f64", 4, 4): "IdLi4ELi4ELb1E", ("f64", 4, 8): "IdLi4ELi8ELb1E",
            ("f64", 8, 1): "IdLi8ELi1ELb1E", ("f64", 8, 2): "IdLi8ELi2ELb1E",
            ("f64", 8, 4): "IdLi8ELi4ELb1E", ("f64", 8, 8): "IdLi8ELi8ELb1E",
            ("f32", 8, 1): "IfLi8ELi1ELb1E", ("f32", 8, 2): "IfLi8ELi2ELb1E",
            ("f32", 8, 4): "IfLi8ELi4ELb1E",
            ("f32", 8, 8): "IfLi8ELi8ELb1E", ("f32", 16, 1): "IfLi16ELi1ELb1E",
            ("f32", 16, 2): "IfLi16ELi2ELb1E", ("f32", 16, 4): "IfLi16ELi4ELb1E"}


def assemble() -> str:
    srcs = ("rsv_traj_f64.hip", "rsv_traj_f32.hip")
    with tempfile.TemporaryDirectory() as d:
        outs = [os.path.join(d, src + ".s") for src in srcs]
        procs = [subprocess.Popen(["hipcc", f"--offload-arch={B.ARCH}", "-O3", "-std=c++17",
                                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                                   "-I", os.path.join(B.ROOT, "include"), "-I", B.CSRC,
                                   "--cuda-device-only", "-S", os.path.join(B.CSRC, src),
                                   "-o", out], stderr=subprocess.DEVNULL)
                 for src, out in zip(srcs, outs)]
        for p, src in zip(procs, srcs):
            if p.wait() != 0:
                raise RuntimeError(f"hipcc failed on {src}")
        return "\n".join(open(out).read() for out in outs)


def kernel_text(asm: str, tag: str) -> str:
    m = re.search(r"^(_ZN3rsv\w*k_traj" + tag + r"\w*):", asm, re.M)
    if not m:
        raise KeyError(tag)
    body = asm[m.end():]
    return body[: body.index(".Lfunc_end")], m.group(1)


def descriptor(asm: str, name: str) -> dict:
    m = re.search(r"\.amdhsa_kernel " + re.escape(name) + r"(.*?)\.end_amdhsa_kernel", asm, re.S)
    get = lambda k: int(re.search(r"\." + k + r" (\d+)", m.group(1)).group(1))
    return {"vgpr": get("amdhsa_next_free_vgpr"), "sgpr": get("amdhsa_next_free_sgpr"),
            "scratch_bytes": get("amdhsa_private_segment_fixed_size")}


def leapfrog_loop(text: str, n_dpp: int):
    """Instruction counts of the innermost loop that carries the lane shifts.

    The loop runs two leapfrog steps per iteration.  Blocks that hold the
    chain-end substitution (marked by an empty inline-asm statement, skipped
    by a uniform branch in every wavefront without a chain end) are left out:
    the count is the path almost every wavefront takes."""
    lines = [l.strip() for l in text.split("\n")]
    labels = {}
    for i, l in enumerate(lines):
        m = re.match(r"^(\.LBB\w+):", l)
        if m:
            labels[m.group(1)] = i
    best = None
    for i, l in enumerate(lines):
        m = re.match(r"s_cbranch_\w+ (\.LBB\w+)|s_branch (\.LBB\w+)", l)
        tgt = m and (m.group(1) or m.group(2))
        if tgt in labels and labels[tgt] < i and "Loop Header" in lines[labels[tgt]]:
            seg = lines[labels[tgt]:i + 1]
            if sum("_dpp" in x for x in seg) >= n_dpp and (best is None or len(seg) < len(best)):
                best = seg
    blocks, cur = [], []
    for x in best:
        if re.match(r"^(\.LBB\w+:|; %bb\.\d+:)", x):  # named and fall-through blocks
            blocks.append(cur)
            cur = []
        cur.append(x)
    blocks.append(cur)
    kept = [x for b in blocks if not any("ASMSTART" in y for y in b) for x in b
            if x and not x.startswith((";", ".")) and not x.endswith(":")]
    return Counter(x.split()[0] for x in kept)


def count(asm: str) -> dict:
    table = {}
    for (prec, S, NW), tag in VARIANTS.items():
        text, name = kernel_text(asm, tag)
        ops = leapfrog_loop(text, 4 if prec == "f64" else 2)
        valu = sum(v for k, v in ops.items() if k.startswith("v_"))
        fp = sum(v for k, v in ops.items() if k.startswith("v_") and prec in k)
        # each leapfrog step shifts two values between lanes: 2 DPP moves per
        # 32-bit word, so the loop body holds `steps` unrolled steps
        dpp = sum(v for k, v in ops.items() if "_dpp" in k)
        steps = dpp // (4 if prec == "f64" else 2)
        # floating-point operations of the method's arithmetic: a fused
        # multiply-add counts 2, an add, subtract, multiply or exponential 1
        flop = sum(v * (2 if ("fma" in k or "fmac" in k) else 1) for k, v in ops.items()
                   if k.startswith("v_") and prec in k
                   and any(w in k for w in ("fma", "add", "sub", "mul", "exp")))
        table[f"{prec}_S{S}_W{NW}"] = dict(
            loop_instructions=sum(ops.values()), steps_per_loop=steps,
            valu_per_site_update=valu / (S * steps), fp_valu_per_site_update=fp / (S * steps),
            flop_per_site_update=flop / (S * steps),
            **descriptor(asm, name), top_ops=dict(ops.most_common(12)))
    return table


def main():
    table = count(assemble())
    with open(OUT, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(json.dumps({k: round(v["valu_per_site_update"], 3) for k, v in table.items()}))


if __name__ == "__main__":
    sys.exit(main())
