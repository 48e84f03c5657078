"""Build libsbmt.so for gfx950 (hipcc, in-tree).

    python -m paper_2602_19474_amd.build

Steps: regenerate the lookup-table header from ``csrc/gen_tables.py``, then
compile ``csrc/sbmt.hip`` (the meshing path), ``csrc/sbmt_post.hip`` (field
sampling and mesh quality) and ``csrc/sbmt_pde.hip`` (cotangent Laplacian and
heat steps) into ``libsbmt.so`` next to this file.  Floating
point is compiled without contraction (-ffp-contract=off) so the FP64 vertex
formulas round exactly as written; packed FP32 instructions are disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("SBMT_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_tables.py"),
                           os.path.join(CSRC, "sbmt_tables.h")])
    out = os.path.join(HERE, "libsbmt.so")
    tmp = out + ".tmp"
    cmd = [HIPCC, *HIP_FLAGS, "-o", tmp, os.path.join(CSRC, "sbmt.hip"), os.path.join(CSRC, "sbmt_post.hip"),
           os.path.join(CSRC, "sbmt_pde.hip")]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
