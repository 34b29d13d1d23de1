"""Builds libobfft.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libobfft.so")
SOURCES = ["csrc/ob_kernels.hip", "csrc/ob_tap.hip", "csrc/crt_kernels.hip", "csrc/probe.hip", "csrc/native.hip", "csrc/capi.hip", "csrc/plan_math.cpp"]
HEADERS = ["csrc/ob_stage.h", "csrc/ob_device.h", "csrc/ob_recon.h", "csrc/crt_methods.h", "csrc/obfft_internal.h", "csrc/plan_math.h"]


def build(verbose=False, jobs=4):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             # MFMA results in ordinary VGPRs: no accumulator-register copies
             "-mllvm", "-amdgpu-mfma-vgpr-form",
             "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
             "-Wno-unused-result", "-Wno-unused-value"]
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [hipcc] + flags + ["-x", "hip", "-c", os.path.join(HERE, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    rc = [p.wait() for p in procs]
    if any(rc):
        raise RuntimeError("hipcc failed")
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
