"""Register, scratch and LDS use of every kernel in the product build.

The build records the compiler's resource-usage remarks for each kernel in
a table beside the objects.  No kernel may use scratch (private) memory:
on gfx950 a scratch access is a round trip through the vector memory path,
and every such case found so far came from a small array indexed at run
time or from registers spilled across a K loop.  Both were slow and both
were avoidable.  SGPR spills are allowed: they go to VGPR lanes, not to
memory.
"""
import csv
import glob
import os
import re

import pytest

from paper_2507_18969_amd import build as B


def _rows():
    if not os.path.exists(B.RESOURCES):
        pytest.skip("library not built (no kernel resource table)")
    if os.path.getmtime(B.RESOURCES) + 1 < max(os.path.getmtime(p) for p in
                                               glob.glob(os.path.join(B.CSRC, "*"))):
        pytest.skip("kernel resource table older than the sources (rebuild)")
    with open(B.RESOURCES) as f:
        return list(csv.DictReader(f, delimiter="\t"))


def test_no_kernel_uses_scratch_memory():
    rows = _rows()
    bad = [(r["kernel"], r["scratch"], r["vgpr_spill"]) for r in rows
           if int(r["scratch"]) != 0 or int(r["vgpr_spill"]) != 0]
    assert not bad, bad


def test_every_kernel_is_in_the_table():
    # each __global__ function of the sources appears (mangled) at least once
    rows = _rows()
    names = " ".join(r["kernel"] for r in rows)
    glob_re = re.compile(r"__global__\s+void\s+(?:__launch_bounds__\([^)]*\)\s+)?(\w+)\s*\(")
    missing = []
    for p in glob.glob(os.path.join(B.CSRC, "*.hip")):
        src = open(p).read()
        for k in glob_re.findall(src):
            if f"{len(k)}{k}" not in names:
                missing.append((os.path.basename(p), k))
    assert rows and not missing, missing


def test_register_budget():
    # the unified register file gives at most 512 VGPRs + AGPRs per lane
    for r in _rows():
        assert int(r["vgprs"]) + int(r["agprs"]) <= 512, r
