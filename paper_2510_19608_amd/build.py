"""Build step of the HIP library (gfx950): hipcc -> libokr.so in this package.

Each source is compiled to an object of its own (in parallel), then linked.
The candidate-scoring unit is compiled with NaNs excluded: its max/min
reductions then need no NaN canonicalisation, and no value it handles is a
NaN.  (The IEEE mode bit stays on: turning it off makes the device library's
work-item and work-group id functions non-inlinable, and block indices
then reach the kernels as per-lane values, which turns every wave-uniform
table read into a per-lane vector load.)  Every other unit keeps IEEE
semantics (the load flow detects divergence through NaN-safe comparisons).
"""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libokr.so")
SOURCES = ["okr_kernels.hip", "okr_build.hip", "okr_score.hip", "okr_mixed.hip", "okr_surrogate.hip",
           "okr_greedy.hip", "okr_smice.hip", "okr_host.cpp"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
EXTRA = {"okr_score.hip": ["-fno-honor-nans"]}


def build() -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc] + FLAGS + EXTRA.get(src, []) + ["-c", "-o", obj, os.path.join(CSRC, src)]
        subprocess.run(cmd, check=True, cwd=CSRC)
        return obj

    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 6)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, check=True, cwd=CSRC)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
