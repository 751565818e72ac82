"""Host-side logic of the launch-shape autotuner (no GPU needed)."""

import ctypes

from paper_0905_2441_amd import _lib as L
from paper_0905_2441_amd import autotune


def test_candidates_respect_limits():
    # N above the split cap: at most 16 slices (one workgroup per tile)
    assert autotune.candidates(1000, 131072) == [1, 2, 3, 4, 8, 12, 16]
    # small N, long data: every candidate up to 128 slices
    assert autotune.candidates(10000, 8192) == list(autotune.CANDIDATES)
    # short data: at least MIN_PER_SLICE observations per slice
    assert autotune.candidates(20, 100) == [1, 2]
    assert autotune.candidates(1, 100) == [1]
    # the MFMA form takes at most 16
    assert max(autotune.candidates(65536, 16384, "bf16x3")) == 16


def test_buckets_are_power_of_two_ranges():
    assert autotune.bucket(1) == (1, 1)
    assert autotune.bucket(1000) == (512, 1023)
    assert autotune.bucket(1024) == (1024, 2047)
    assert autotune.bucket(131072) == (131072, 262143)


def test_launch_rule_layout_matches_header(tmp_path):
    """The binding's struct has the size and field offsets that a C compiler
    gives smc_launch_rule from include/smc.h."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    fields = [f[0] for f in L.SmcLaunchRule._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "smc.h"\nint main(void) {\n'
                   '  printf("%zu\\n", sizeof(smc_launch_rule));\n'
                   + "".join(f'  printf("%zu\\n", offsetof(smc_launch_rule, {f}));\n'
                             for f in fields)
                   + "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert got[0] == ctypes.sizeof(L.SmcLaunchRule)
    assert got[1:] == [getattr(L.SmcLaunchRule, f).offset for f in fields]
