"""The tiled factor's unit plan (which tiles each ticket takes, in which order), compiled from
the library's own header and checked on the host for every block count up to 40, every
number of kept columns and four strip shapes, with and without row walkers for the rows below
a kept block: each computed tile is taken exactly once, and every unit waits only for tiles
produced under smaller tickets (the walkers' outputs at the ticket of the last unit they
need), which is what makes every wait of the persistent grid end.
CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_unit_plan_covers_and_orders(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = tmp_path / "check_units"
    src = os.path.join(ROOT, "tests", "unitplan", "check_units.cpp")
    cmd = [gxx, "-std=c++17", "-O1", "-I", os.path.join(ROOT, "tests", "hoststub"),
           "-I", os.path.join(ROOT, "paper_cs_0408029_amd", "csrc"), src, "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.startswith("ok ")
