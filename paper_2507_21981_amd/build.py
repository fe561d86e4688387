"""Build libgsr.so, the renderer's C-ABI shared library, for gfx950.

Flags:
  -ffp-contract=off                          every a*b+c is two rounded operations unless the
                                             source writes fmaf(): the projection's key
                                             specification (tile rectangle, depth bits) is
                                             reproducible bit for bit
  -fhip-fp32-correctly-rounded-divide-sqrt   IEEE / and sqrt in FP32
  -fno-gpu-flush-denormals-to-zero           keep FP32 denormals
  -munsafe-fp-atomics                        hardware FP32 atomic add (coarse-grained memory)
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                             no packed FP32 (v_pk_*_f32) instructions
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgsr.so")
SOURCES = ["gsr_forward.hip", "gsr_backward.hip", "gsr_mesh.hip", "gsr_lidar.hip", "gsr_api.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-fhip-fp32-correctly-rounded-divide-sqrt", "-fno-gpu-flush-denormals-to-zero",
         "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-value", "-Wno-unused-result"]


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *FLAGS, *[os.path.join(CSRC, s) for s in SOURCES], "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{err}")
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
