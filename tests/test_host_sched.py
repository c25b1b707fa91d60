"""Host logic of the runtime's work division (chunking of lone and batched runs,
server round budget and water-filling), checked on the CPU: `sched_check.cpp`
includes the library's `cls_sched.hpp` (plain C++, no HIP) and tests its
properties over random cases."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1708_00765_amd", "csrc")


def test_work_division_properties(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "sched_check"
    subprocess.run([cxx, "-std=c++17", "-O2", "-Wall", "-Werror", "-I", CSRC,
                    os.path.join(HERE, "sched_check.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert r.stdout.strip().splitlines()[-1].startswith("OK")
