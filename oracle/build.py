"""Build step of the CPU reference: one gcc line, IEEE binary32 without
contraction (the GPU path is compiled the same way)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cbt_oracle.c")
LIB = os.path.join(HERE, "libcbt_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=gnu99", "-O2", "-ffp-contract=off", "-fno-fast-math", "-Wall",
           "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
