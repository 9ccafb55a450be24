"""Build the gfx950 HIP library (libppt.so) in-tree with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB_PATH = os.path.join(HERE, "libppt.so")
SOURCES = [os.path.join(CSRC, "ppt_kernels.hip"), os.path.join(CSRC, "ppt_host.cpp")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # hardware float atomics (device memory here is coarse-grained)
    "-munsafe-fp-atomics",
    # packed FP32 instructions are disabled for every HIP compile in this project
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no sinking of the stores common to the cases of a switch into one store through a selected
    # address: that kept a few fields of the shading kernels' weight record in scratch memory
    # (shading 16.9 -> 15.9 ms per step without it)
    "-mllvm", "-simplifycfg-sink-common=false",
    # (FP32 division and square root stay correctly rounded: the faster hardware sequences took the
    # replay 5.8 -> 5.5 ms per step but doubled the error of the smooth dielectric's normal-map
    # gradient, whose s/p rotators amplify rounding: light-stage glass map 4.8e-4 -> 9.4e-4 of 1e-3)
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc] + HIPCC_FLAGS + ["-I", os.path.join(HERE, "..", "include"), "-o", tmp] + SOURCES
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    if verbose:
        print(r.stderr)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
