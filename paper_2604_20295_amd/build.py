"""Build libetac.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2604_20295_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libetac.so")
# (source, object name, extra flags).  The network-adjoint kernel keeps ~450
# registers per lane live (one wave per SIMD): letting MFMA results live in
# VGPRs as well as AGPRs, and sinking loop-invariant address computations
# into the loops that use them, keeps it free of spills.  It is built from
# etac_backward.hip on its own (ETAC_BWD_NET_ONLY); the decay adjoint, which
# runs three or four workgroups per CU, is better off without the sinking.
SOURCES = [
    ("etac_api.cpp", "etac_api", []),
    ("etac_forward.hip", "etac_forward", []),
    ("etac_backward.hip", "etac_backward", ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]),
    ("etac_backward.hip", "etac_backward_net", ["-DETAC_BWD_NET_ONLY", "-mllvm", "-amdgpu-mfma-vgpr-form=1",
                                                "-mllvm", "-sink-insts-to-avoid-spills"]),
    ("etac_mesh.hip", "etac_mesh", []),
    ("etac_hand.hip", "etac_hand", []),
    ("etac_regress.hip", "etac_regress", []),
]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 VALU ops stay disabled: plain FP32 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose=False):
    objs = []
    for src, name, extra in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, name + ".o")
        cmd = [HIPCC, "-x", "hip", *FLAGS, *extra, "-c", path, "-o", obj]
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
