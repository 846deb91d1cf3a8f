"""Compile the HIP library (libmgsqr.so) in place for gfx950."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libmgsqr.so")
SRC = os.path.join(HERE, "csrc", "mgsqr.hip")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# -ffp-contract=off: the error-free transformations need every + - * rounded
# on its own.  Packed FP32 instructions are disabled.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall"]


def build():
    tmp = SO + ".tmp%d" % os.getpid()
    subprocess.run([HIPCC] + FLAGS + ["-o", tmp, SRC], check=True)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build())
