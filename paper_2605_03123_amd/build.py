"""Build libffx.so in-tree with hipcc for gfx950.

    python -m paper_2605_03123_amd.build

Packed-FP32 instructions are disabled for the device code
(-Xclang -target-feature -Xclang -packed-fp32-ops); hipcc's host pass warns that
it does not know the feature, which is harmless.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libffx.so")
SOURCES = ["host.cpp", "drivers.cpp", "api.cpp", "gates.cpp", "sampling.cpp", "program.cpp", "batch.cpp", "kernels.hip", "segpass.hip", "batched.hip", "sample.hip", "dense.hip"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False, arch: str = "gfx950") -> str:
    objs = []
    common = ["-O3", "-std=c++17", "-fPIC", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
              "-Wall", "-Wno-unused-result"]
    # The Givens dispatch has one near-identical branch per orbital pair; letting
    # SimplifyCFG sink or hoist their common code merges them behind a runtime
    # register index, which sends the register arrays to scratch memory.
    device_flags = [f"--offload-arch={arch}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-mllvm", "-simplifycfg-sink-common=false", "-mllvm", "-simplifycfg-hoist-common=false"]
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    procs = []
    for src in SOURCES:
        obj = os.path.join(build_dir, src + ".o")
        cmd = [hipcc()] + common
        if src.endswith(".hip"):
            cmd += ["-x", "hip"] + device_flags
        else:
            cmd += ["-D__HIP_PLATFORM_AMD__"]
        cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append((src, out))
        elif verbose and out.strip():
            print(out)
    if failed:
        msg = "\n".join(f"--- {s} ---\n{o}" for s, o in failed)
        raise RuntimeError(f"hipcc failed:\n{msg}")
    tmp = LIB + ".tmp"
    link = [hipcc(), "-shared", f"--offload-arch={arch}", "-o", tmp] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
