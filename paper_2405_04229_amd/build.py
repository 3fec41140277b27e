"""Builds libcphot.so (HIP, gfx950) in-tree with hipcc."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcphot.so")
SOURCES = ["cphot_api.cpp", "cphot_kernels.hip", "cphot_surrogate.hip", "cphot_table.hip"]
ARCH = os.environ.get("CPHOT_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions stay off: they are avoided on this target. No implicit
# FMA contraction: fused operations are written out (fmaf), so one source line
# gives the same bits in every kernel instantiation it is inlined into.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-ffp-contract=off", "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
             # matrix-core results in ordinary VGPRs: no accumulator-register copies
             # before the activations, and one register file to budget
             "-mllvm", "-amdgpu-mfma-vgpr-form"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build(verbose: bool = False) -> str:
    """Compiles the sources concurrently (one hipcc per source), then links."""
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, src + ".o")
        cmds.append([hipcc(), *HIP_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    procs = [subprocess.Popen(cmd) for cmd in cmds]
    failed = [cmd for cmd, pr in zip(cmds, procs) if pr.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
