"""The autotuner's header: whatever it measures, the header it writes defines every
constant the library reads from ``csrc/tuning.h`` and compiles."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2009_01054_amd import tune

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2009_01054_amd", "csrc")


def test_written_header_defines_every_tuned_constant(tmp_path):
    results = {}
    for key, win in (("SLICE", 1), ("SLICEWGS", 256), ("WIDE", 1), ("KPW", 1), ("R1", 64.0), ("MAXR64", 2),
                     ("MAXR32", 4), ("R8", 16.0)):
        results[key] = (win, {win: [0.1, 0.2]}, {win: 1.0}, ["workload a", "workload b"])
    rates = {"kGatherRateF64": 9.1e12, "kGatherRateF32": 1.2e13, "kTilesRateF64": 5.5e13,
             "kTilesRateF32": 1.2e14, "kTilesFull": 300.0}
    out = tmp_path / "tuning.h"
    tune.write_header(str(out), results, "gfx950", rates)
    text = out.read_text()
    names = lambda t: set(re.findall(r"constexpr\s+\w+\s+(k\w+)\s*=", t))  # noqa: E731
    committed = names(open(os.path.join(CSRC, "tuning.h")).read())
    assert committed and committed <= names(text)
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host compiler")
    src = tmp_path / "use.cc"
    src.write_text('#include "tuning.h"\nint main() { return gvt::kStage1Wide + (int)gvt::kTilesFull; }\n')
    r = subprocess.run([gxx, "-std=c++17", "-fsyntax-only", f"-I{tmp_path}", str(src)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
