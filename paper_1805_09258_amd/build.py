"""Build librc.so (HIP, gfx950) in-tree with hipcc.

Flags: -O3, gfx950 only, no FP contraction (the FP32 decision formulas must
round as written; fused operations are explicit where wanted), correctly
rounded FP32 division and square root, packed-FP32 instructions disabled.
"""
import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
SRC = ["csrc/api.cpp", "csrc/bvh.cpp", "csrc/lightbins.cpp", "csrc/kernels.hip", "csrc/learned.hip", "csrc/render.hip", "csrc/j08.hip"]
OUT = PKG / "librc.so"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off", "-fno-fast-math",
         "-fhip-fp32-correctly-rounded-divide-sqrt", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result"]


def build(verbose=False, jobs=None):
    objs = []
    procs = []
    for s in SRC:
        src = PKG / s
        obj = PKG / "csrc" / (Path(s).stem + ".o")
        lang = ["-x", "hip"] if s.endswith(".hip") or s.endswith("api.cpp") else []
        cmd = [HIPCC] + FLAGS + ["-I", str(ROOT / "include")] + lang + ["-c", str(src), "-o", str(obj)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), s))
        objs.append(str(obj))
    bad = False
    for p, s in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and "is not a recognized feature" not in l]
        if p.returncode != 0:
            bad = True
            sys.stderr.write(f"--- {s} ---\n" + "\n".join(lines) + "\n")
        elif verbose and lines:
            print("\n".join(lines))
    if bad:
        raise RuntimeError("librc build failed")
    link = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", str(OUT)] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    for o in objs:
        try:
            os.remove(o)
        except OSError:
            pass
    return OUT


if __name__ == "__main__":
    build(verbose=True)
