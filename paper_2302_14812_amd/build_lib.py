"""Build libradio.so (HIP for gfx950) next to this file.

Called by the package's build step; compiles every source of the library
each time it runs.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libradio.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-fvisibility=hidden",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-result",
]

SOURCES = ["radio_kernels.hip", "radio_spectrum.hip", "radio_push.hip", "radio_io.hip",
           "radio_runtime.cpp"]
# measurement programs run by bench.py: floating-point atomic-add throughput,
# issue cost of the vector instructions the deposit uses
ATOMICS_BENCH = os.path.join(HERE, "radio_atomics_bench")
VALU_BENCH = os.path.join(HERE, "radio_valu_bench")


def build(verbose: bool = False) -> str:
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC] + COMMON + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    for src, exe in (("atomics_bench.hip", ATOMICS_BENCH), ("valu_bench.hip", VALU_BENCH)):
        cmd = [HIPCC] + [c for c in COMMON if c not in ("-fPIC", "-fvisibility=hidden")] + [
            os.path.join(CSRC, src), "-o", exe + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(exe + ".tmp", exe)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
