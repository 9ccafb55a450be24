"""Build the gfx950 HIP library (libppt.so) in-tree with hipcc."""
import os
import shutil
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB_PATH = os.path.join(HERE, "libppt.so")
KERNELS = os.path.join(CSRC, "ppt_kernels.hip")
KERNELS_EXT = os.path.join(CSRC, "ppt_kernels_ext.hip")
HOST = os.path.join(CSRC, "ppt_host.cpp")
SOURCES = [KERNELS, KERNELS_EXT, HOST]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # hardware float atomics (device memory here is coarse-grained)
    "-munsafe-fp-atomics",
    # packed FP32 instructions are disabled for every HIP compile in this project
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no sinking of the stores common to the cases of a switch into one store through a selected
    # address: that kept a few fields of the shading kernels' weight record in scratch memory
    # (shading 16.9 -> 15.9 ms per step without it)
    "-mllvm", "-simplifycfg-sink-common=false",
]
# The main unit: FP32 division and square root by the hardware reciprocal and square-root sequences
# (a few ulp) instead of the correctly rounded expansions (replay 5.8 -> 5.5 ms per step).  The
# light-stage variants (ppt_kernels_ext.hip) keep them correctly rounded: the smooth dielectric's
# normal-map gradient runs through its s/p rotators, which amplify rounding (with the hardware
# sequences the light-stage glass map's error against the oracle doubled, 4.8e-4 -> 9.4e-4 of 1e-3).
FAST_DIV = ["-fno-hip-fp32-correctly-rounded-divide-sqrt"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r.stderr


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(HERE, "..", "include")]
    tmpdir = tempfile.mkdtemp(prefix="ppt_build_")
    try:
        objs = []
        log = []
        for src, extra in ((KERNELS, FAST_DIV), (KERNELS_EXT, []), (HOST, [])):
            obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
            log.append(_run([hipcc] + HIPCC_FLAGS + extra + inc + ["-c", src, "-o", obj]))
            objs.append(obj)
        tmp = LIB_PATH + ".tmp"
        log.append(_run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs))
        if verbose:
            print("".join(log))
        os.replace(tmp, LIB_PATH)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
