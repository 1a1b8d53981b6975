"""The per-unit work bench.py prices the count kernel's roofline with (VALU instructions per group
of eight segments x 45 f0 bins per lane on the table variant's fast path) is the count that fastpath_ops.py reads from
the kernel's gfx950 assembly, for every chunk size the autotuner may pick, in the kernel's form for host-proven windows
(the benchmark's) and in its checked form.  Compiles the count
kernel to assembly on the host (no GPU needed)."""
import os
import shutil
import sys

import pytest

ROOT = os.path.join(os.path.dirname(__file__), "..")
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(__file__))


@pytest.mark.skipif(not (os.path.exists("/opt/rocm/bin/hipcc") or shutil.which("hipcc")), reason="hipcc not found")
def test_bench_floor_matches_the_assembly():
    import bench
    import fastpath_ops

    asm = fastpath_ops.assembly()
    for chunk in (128, 256, 512):
        for mode, table in ((10, bench.TABLE_OPS_PER_TS), (2, bench.TABLE_OPS_PER_TS_CHECKED)):
            valu, seg = fastpath_ops.fast_path(chunk, asm, mode)
            assert seg == 8
            assert valu / (seg * fastpath_ops.BINS_PER_LANE) == pytest.approx(table[chunk], rel=1e-12), (chunk, mode)
