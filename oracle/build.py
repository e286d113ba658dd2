"""Build the serial FP64 oracle (the LES step and the guess network) into
oracle/liboracle.so with gcc.

The oracle is test infrastructure; building it is part of the build check,
using it is reserved to the tests, the smoke check and the CPU baseline.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, f) for f in ("les_oracle.c", "cnn_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")

# -ffp-contract=off: no fused multiply-add, every product is rounded as written.
CMD = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
       "-ffp-contract=off", "-o"]


def build() -> str:
    tmp = LIB + ".tmp"
    cmd = CMD + [tmp] + SRCS + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
