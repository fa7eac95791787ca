"""Build libamgiga.so in the package directory (gfx950 only).

Host setup code is compiled by g++ without FMA contraction (its bits define
the aggregates); the HIP sources by hipcc for gfx950 with packed-FP32
instructions disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libamgiga.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run(cmd):
    subprocess.check_call(cmd)


def build(verbose=False):
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    host_o = os.path.join(bdir, "host_setup.o")
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-pthread", "-Wall"]
         + inc + ["-c", os.path.join(CSRC, "host_setup.cpp"), "-o", host_o])
    dev_o = os.path.join(bdir, "solver.o")
    _run([HIPCC, "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"]
         + inc + ["-c", os.path.join(CSRC, "solver.hip"), "-o", dev_o])
    # device set-up: no FMA contraction (its bits must equal the host set-up's)
    sdev_o = os.path.join(bdir, "setup_dev.o")
    _run([HIPCC, "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-ffp-contract=off",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"]
         + inc + ["-c", os.path.join(CSRC, "setup_dev.hip"), "-o", sdev_o])
    probe_o = os.path.join(bdir, "probe.o")
    _run([HIPCC, "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"]
         + inc + ["-c", os.path.join(CSRC, "probe.hip"), "-o", probe_o])
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, dev_o, sdev_o, probe_o, host_o, "-pthread",
          "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
