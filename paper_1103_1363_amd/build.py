"""Build liblq.so (HIP, gfx950) in-tree.

Usage: python -m paper_1103_1363_amd.build [--jobs N]

Every source under csrc/ is compiled with hipcc for gfx950 into an object
file (in parallel), then linked into paper_1103_1363_amd/liblq.so.  Packed
FP32 VALU instructions are disabled for device code.
"""
from __future__ import annotations

import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "liblq.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
    # matrix-core results in ordinary VGPRs (no accumulator-register copies)
    "-Xarch_device", "-mllvm=-amdgpu-mfma-vgpr-form",
    "-I" + os.path.join(HERE, "..", "include"),
]


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))


def compile_one(src: str, build_dir: str = BUILD, defines=()) -> str:
    obj = os.path.join(build_dir, src.replace(".hip", ".o"))
    cmd = [HIPCC, *FLAGS, *("-D" + d for d in defines), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    if r.stderr.strip():
        # the host pass warns that it does not know the packed-fp32 feature
        lines = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l
                 and "is not a recognized feature" not in l and l.strip()]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")
    return obj


def build(jobs: int = 8, out: str = OUT, defines=()) -> str:
    """Compile every source and link `out`; `defines` (NAME=VALUE) select
    compile-time tuning parameters such as LQ_WAVES_F32."""
    build_dir = BUILD if out == OUT else out + ".objs"
    os.makedirs(build_dir, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        objs = list(ex.map(lambda s: compile_one(s, build_dir, defines), srcs))
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=int(os.environ.get("MAX_JOBS", "8")))
    ap.add_argument("--out", default=OUT)
    ap.add_argument("-D", "--define", action="append", default=[])
    a = ap.parse_args()
    print(build(a.jobs, os.path.abspath(a.out), a.define))


if __name__ == "__main__":
    main()
