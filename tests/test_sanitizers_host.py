"""The oracle and the host replays of the device schedules built with
AddressSanitizer and UndefinedBehaviorSanitizer (plain g++/gcc, no device
code: tests/host/launch_stubs.cpp stands in for the kernel launchers) and
run against each other (tests/host/emulate_check.cpp); complex128 replays
only, at -O0, to keep the build short.  Any out-of-bounds
access, use after free or undefined behaviour in the index algebra, the
work lists, the compaction or the oracle stops the run.  No GPU is used."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2310_13421_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g0", "-O0"]


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="needs gcc/g++")
def test_host_replays_and_oracle_under_asan_and_ubsan(tmp_path):
    inc = ["-D__HIP_PLATFORM_AMD__", "-DTPD_EMULATE_COMPLEX128_ONLY", "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs, procs = [], []
    o = str(tmp_path / "oracle.o")
    procs.append(subprocess.Popen(["gcc", *SAN, "-std=c99", "-ffp-contract=off", "-fopenmp", "-c",
                                   os.path.join(ROOT, "oracle", "tpd_oracle.c"), "-o", o],
                                  stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    objs.append(o)
    for src in (os.path.join(CSRC, "tpd_api.cpp"), os.path.join(CSRC, "tpd_emulate.cpp"),
                os.path.join(CSRC, "tpd_shapes.cpp"), os.path.join(ROOT, "tests", "host", "launch_stubs.cpp"),
                os.path.join(ROOT, "tests", "host", "emulate_check.cpp")):
        o = str(tmp_path / (os.path.basename(src) + ".o"))
        procs.append(subprocess.Popen(["g++", *SAN, "-std=c++20", "-ffp-contract=off", *inc, "-c", src, "-o", o],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
        objs.append(o)
    for p in procs:
        out, err = p.communicate(timeout=600)
        assert p.returncode == 0, err[-3000:]
    exe = str(tmp_path / "emulate_check")
    r = subprocess.run(["g++", *SAN, "-fopenmp", "-o", exe, *objs, "-L/opt/rocm/lib", "-lamdhip64",
                        "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=900, env=env)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "0 failure(s)" in r.stdout and r.stdout.count("ok ") >= 30, r.stdout
