"""The sweep kernel's compile-time thread roles, checked on the host: the
header that defines them (csrc/tpd_core.h) is compiled with g++ into a
small checker (tests/host/roles_check.cpp).  No GPU is used."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_roles_bijective_lanes_hold_d_bits_and_8_level_slot_rows_share_a_word(tmp_path):
    exe = tmp_path / "roles_check"
    src = os.path.join(ROOT, "tests", "host", "roles_check.cpp")
    cmd = ["g++", "-std=c++20", "-O1", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "paper_2310_13421_amd", "csrc"),
           "-I", os.path.join(ROOT, "include"), "-x", "c++", src, "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout
    lines = dict(line.split(" ", 1) for line in r.stdout.strip().splitlines())
    assert "slot_rows=0xf " in lines["XB8_DB5"] and "slot_rows=0xf " in lines["XB8_DB6"]
