"""Build libfipgemm.so (the C-ABI library) for gfx950 with hipcc, in-tree.

    python -m paper_2302_08417_amd.build
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libfipgemm.so")
# the two mixed-precision units first: they take the longest and compile side by side
SOURCES = ["fipgemm_mx_fp8big.hip", "fipgemm_mx.hip", "fipgemm_kernels.hip", "fipgemm_batched.hip",
           "fipgemm_scratch.hip", "fipgemm_trsm.hip", "fipgemm_api.cpp"]
ARCH = os.environ.get("FIPGEMM_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# -packed-fp32-ops: keep the compiler from forming packed FP32 ALU ops.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", f"--offload-arch={ARCH}", "-I", INCLUDE,
          "-I", CSRC]


def build(verbose: bool = False) -> str:
    objs = []
    build_dir = os.path.join(PKG, "_build")
    os.makedirs(build_dir, exist_ok=True)
    procs = []
    for src in SOURCES:  # compile the sources concurrently
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"]
        cmd = [HIPCC, *COMMON, *lang, *DEVICE_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                 stderr=subprocess.STDOUT, text=True)))
    failed = []
    for src, obj, p in procs:
        text, _ = p.communicate()
        out = "\n".join(line for line in text.splitlines() if "packed-fp32-ops" not in line)
        if p.returncode != 0:
            sys.stderr.write(out + "\n")
            failed.append(src)
        elif verbose and out.strip():
            print(out)
        objs.append(obj)
    if failed:
        raise RuntimeError(f"hipcc failed on {', '.join(failed)}")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
