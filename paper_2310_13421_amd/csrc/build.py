"""Build libtpd.so for gfx950 with hipcc (in-tree, no JIT cache).

    python -m paper_2310_13421_amd.csrc.build

Compiles the HIP kernels, the C ABI and the host schedule emulator into
paper_2310_13421_amd/libtpd.so.  Every HIP source is compiled with packed
FP32 instructions disabled and without floating-point contraction.
"""
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libtpd.so")
SOURCES = ["tpd_sweep_c128_db3.hip", "tpd_sweep_c128_db4.hip", "tpd_sweep_c128_db5.hip", "tpd_sweep_c64_db4.hip",
           "tpd_sweep_c64_db5.hip", "tpd_sweep_c64_db6.hip", "tpd_sweep_r64_db4.hip", "tpd_sweep_r64_db5.hip",
           "tpd_sweep_r64_db6.hip", "tpd_sweep_r32_db4.hip", "tpd_sweep_r32_db5.hip", "tpd_sweep_r32_db6.hip",
           "tpd_sweep_c128.hip", "tpd_sweep_c64.hip", "tpd_sweep_r64.hip", "tpd_sweep_r32.hip",
           "tpd_batched_c128.hip", "tpd_batched_c64.hip", "tpd_batched_r64.hip", "tpd_batched_r32.hip",
           "tpd_kernels.hip", "tpd_select.hip", "tpd_scratch.hip", "tpd_shapes.cpp", "tpd_emulate.cpp",
           "tpd_api.cpp"]
HOST_SOURCES = ("tpd_emulate.cpp", "tpd_shapes.cpp")  # plain host C++ (g++)
HEADERS = ["tpd_core.h", "tpd_internal.h", "tpd_sweep.h", "tpd_batched.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++20",
    "-fPIC",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"),
]


def _run(cmd):
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd))
    noise = [ln for ln in (r.stderr or "").splitlines()
             if ln.strip() and "packed-fp32-ops" not in ln and "not a recognized feature" not in ln]
    if noise:
        sys.stderr.write("\n".join(noise) + "\n")
    return time.time() - t0


def build(verbose: bool = True, jobs: int = 0) -> str:
    """Compile every source to an object (in parallel) and link libtpd.so."""
    if jobs <= 0:
        jobs = max(1, min(len(SOURCES), os.cpu_count() or 4, int(os.environ.get("MAX_JOBS", "16"))))
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.rsplit(".", 1)[0] + ".o")
        objs.append(obj)
        if src in HOST_SOURCES:
            # host-only code (the schedule's shape table, the host replay used by
            # the tests): plain host C++, no device pass
            cmd = ["g++", "-O2" if src == "tpd_shapes.cpp" else "-O1", "-std=c++20", "-fPIC", "-ffp-contract=off",
                   "-D__HIP_PLATFORM_AMD__",
                   "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-c", os.path.join(HERE, src),
                   "-o", obj]
        else:
            cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(HERE, src), "-o", obj]
        procs.append((src, cmd))
    t0 = time.time()
    running = []
    for src, cmd in procs:
        running.append((src, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
        while len([p for p in running if p[2].poll() is None]) >= jobs:
            time.sleep(0.05)
    failed = False
    for src, cmd, p in running:
        out, err = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out + err)
            failed = True
        else:
            noise = [ln for ln in (err or "").splitlines()
                     if ln.strip() and "packed-fp32-ops" not in ln and "not a recognized feature" not in ln
                     and "warning: feature flag" not in ln]
            if noise and verbose:
                sys.stderr.write(f"[{src}]\n" + "\n".join(noise) + "\n")
    if failed:
        raise RuntimeError("libtpd compilation failed")
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", tmp, *objs,
          "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"])
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s")
    return LIB


if __name__ == "__main__":
    build()
