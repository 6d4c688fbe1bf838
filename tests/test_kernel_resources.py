"""Compile-time resource check of the step kernels (CPU only, hipcc cross
compiles for gfx950): no step or batch kernel may use scratch memory (a
spilled row buffer costs 2.5x in throughput) or drop below two waves per
SIMD (one for the FP64 two-step kernels, whose LDS rings allow no more).
The open-channel variants (mode 2, small lattices) may spill a few bytes
but no row buffer (at most 64 bytes per lane); so may the two-step kernel,
whose frame reserves a few bytes for spilled scalars."""
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1405_2232_amd", "csrc", "lbm_device.hip")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_step_kernels_use_no_scratch():
    with tempfile.TemporaryDirectory() as d:
        out = subprocess.run(
            [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-c", SRC, "-o",
             os.path.join(d, "k.o"), "-Rpass-analysis=kernel-resource-usage"],
            capture_output=True, text=True, check=True)
    cur, seen, bad = None, 0, []
    for line in out.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            continue
        if cur and ("k_tile" in cur or "k_batch" in cur or "k_pair" in cur):
            m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
            if m:
                seen += 1
                limit = 64 if (re.search(r"k_tileILi\dELi\d+ELi2E", cur) or "k_pair" in cur) else 0
                if int(m.group(1)) > limit:
                    bad.append((cur, "scratch", int(m.group(1))))
            m = re.search(r"Occupancy \[waves/SIMD\]: (\d+)", line)
            # the FP64 two-step kernels run one wave per SIMD by design (their
            # LDS rings allow two 128-lane blocks per CU)
            need = 1 if re.search(r"k_pair(_batch)?ILi0E", cur) else 2
            if m and int(m.group(1)) < need:
                bad.append((cur, "occupancy", int(m.group(1))))
    assert seen > 50
    assert not bad, bad
