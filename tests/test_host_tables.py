"""Bin lookup tables of the runtime, checked on the host for every value
below the third-side cutoff, and the neighbour lists' pad entries, checked
against a grid of rows where the runtime lets the triplet kernel read them
(tests/host_tables_check.cpp, built from the runtime's own source with stub
launchers)."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")


def test_bin_tables_exact(tmp_path):
    if not HIPCC:
        pytest.skip("hipcc not available")
    exe = tmp_path / "host_tables_check"
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "-I" + os.path.join(ROOT, "include"),
                           "-I" + os.path.join(ROOT, "paper_1708_08619_amd", "csrc"),
                           os.path.join(ROOT, "tests", "host_tables_check.cpp"), "-o", str(exe)],
                          stderr=subprocess.DEVNULL)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout
