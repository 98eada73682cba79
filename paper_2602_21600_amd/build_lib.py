"""Build libaqr.so in-tree: host C++ with g++, the gfx950 kernels with hipcc.

Every source is compiled with -ffp-contract=off: the quantiser and the
query encoding must round each FP32 operation separately, and fused
multiply-add is written explicitly where it is meant.  Packed FP32
instructions are disabled for the device code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
OUT = os.path.join(HERE, "libaqr.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HOST_SRC = ["errors.cpp", "quantize.cpp", "build.cpp", "indexio.cpp"]
HIP_SRC = ["device.hip", "density.hip", "knn.hip"]

HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-march=x86-64-v3", "-ffp-contract=off",
              "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter", "-pthread"]
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off",
             "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-parameter", "-Wno-unused-result"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False, jobs: int = 4) -> str:
    os.makedirs(BUILD, exist_ok=True)
    procs = []
    objs = []
    for src in HOST_SRC:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        cmd = ["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd)))
    for src in HIP_SRC:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        cmd = [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True)))
    failed = False
    for cmd, p in procs:
        _, err = p.communicate()
        if err:
            # hipcc's host pass warns that it does not know the packed-fp32
            # feature; that line is harmless, everything else is shown
            lines = [l for l in err.splitlines() if "packed-fp32-ops" not in l]
            if lines:
                print("\n".join(lines), file=sys.stderr)
        if verbose:
            print(" ".join(cmd), flush=True)
        if p.returncode != 0:
            failed = True
    if failed:
        raise RuntimeError("libaqr: compilation failed")
    tmp = OUT + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs, "-pthread"],
         verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
