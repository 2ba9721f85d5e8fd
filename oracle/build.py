"""Compile the C oracle into oracle/liboracle.so (plain gcc, FP64, no
contraction of multiply-adds so every expression rounds as written).

TEST INFRASTRUCTURE: see oracle/__init__.py.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "stepper.c")
LIB = os.path.join(HERE, "liboracle.so")
SRC2D = os.path.join(HERE, "stepper2d.c")
LIB2D = os.path.join(HERE, "liboracle2d.so")


def compile_stepper(src: str, out: str, verbose: bool = False) -> str:
    """Compile a stepper source file into the shared library `out`."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    compile_stepper(SRC2D, LIB2D, verbose)
    return compile_stepper(SRC, LIB, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
