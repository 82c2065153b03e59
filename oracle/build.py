"""Compiles the oracle's C part (first_hit.c) into oracle/libfirst_hit.so with gcc.

Test infrastructure only: building the checker is not using it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build() -> str:
    src = os.path.join(HERE, "first_hit.c")
    out = os.path.join(HERE, "libfirst_hit.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-Wall", "-Wextra", src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
