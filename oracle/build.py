"""Build the CPU oracle library (gcc, FP64, OpenMP).  Test infrastructure.

FP contraction is disabled so the FP32 decision formulas round exactly as
written; no fast-math.
"""
import subprocess
from pathlib import Path

HERE = Path(__file__).resolve().parent


def build(verbose=False, src=None, out=None):
    src = HERE / "rco.c" if src is None else Path(src)
    out = HERE / "liboracle.so" if out is None else Path(out)
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-o", str(out), str(src), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    build(verbose=True)
