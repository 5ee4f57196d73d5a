"""Build libetac.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2604_20295_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libetac.so")
SOURCES = ["etac_api.cpp", "etac_forward.hip", "etac_backward.hip", "etac_mesh.hip", "etac_hand.hip"]
# The adjoint kernel keeps ~500 registers per lane live (one wave per SIMD);
# letting MFMA results live in VGPRs as well as AGPRs avoids spills there.
EXTRA = {"etac_backward.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 VALU ops stay disabled: plain FP32 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose=False):
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, "-x", "hip", *FLAGS, *EXTRA.get(src, []), "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        msgs = [ln for ln in (r.stderr or "").splitlines() if "packed-fp32-ops" not in ln]
        if r.returncode != 0:
            sys.stderr.write("\n".join(msgs) + "\n")
            raise RuntimeError(f"hipcc failed on {src}")
        if verbose and msgs:
            print("\n".join(msgs))
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
