"""Builds the test-only matrix-core layout probe (libgsprobe.so) for gfx950."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libgsprobe.so")


def build() -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950", "-Xclang",
                           "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
                           os.path.join(HERE, "mfma_probe.hip"), "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
