"""The roofline's per-unit figure matches the kernel sources.

bench.py prices the trajectory kernel's launches with the VALU instructions
per site-update of its leapfrog loop, read from the gfx950 assembly into
paper_1603_08114_amd/isa_counts.json.  Rebuilding that assembly from the
current sources must give the committed counts (loop length, VALU and flop
per site-update, registers and scratch of every tile shape), so a change to
the kernels cannot leave the roofline priced on an older loop.
"""
import json
import shutil

import pytest

from paper_1603_08114_amd import isa_count


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc (gfx950 cross-compiler)")
def test_committed_counts_match_the_current_assembly():
    fresh = isa_count.count(isa_count.assemble())
    with open(isa_count.OUT) as f:
        committed = json.load(f)
    assert sorted(fresh) == sorted(committed)
    for shape, rec in committed.items():
        assert fresh[shape] == rec, shape
