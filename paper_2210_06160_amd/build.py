"""Builds librtsdf.so (HIP for gfx950) in-tree.

Flags that are part of the numerical definition:
  -ffp-contract=off                       no fused multiply-adds where the operation order
                                          decides a hit, a snap or an accept (box tests use
                                          explicit fmaf where rounding is harmless)
  -fhip-fp32-correctly-rounded-divide-sqrt  IEEE '/' and sqrtf, as on the host
  -fno-gpu-flush-denormals-to-zero        IEEE subnormals, as on the host
  -Xclang -target-feature -Xclang -packed-fp32-ops   no packed FP32 instructions
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librtsdf.so")
# VALU issue-rate probe used by the benchmark to measure the integer-ALU peak (not the path)
PROBE_SRC = "valu_peak.hip"
PROBE_LIB = os.path.join(HERE, "libvalupeak.so")
SOURCES = ["capi.cpp", "scan.hip", "voxelize.hip", "jfa.hip", "combine.hip", "lbvh.hip", "raysample.hip",
           "shadow.hip", "backward.hip"]
ARCH = os.environ.get("RTSDF_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-ffp-contract=off",
         "-fhip-fp32-correctly-rounded-divide-sqrt", "-fno-gpu-flush-denormals-to-zero",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall",
         "-Wno-unused-function", "-Wno-unused-command-line-argument"]


def _compile(src, out, defines):
    obj = os.path.join(out, os.path.basename(src) + ".o")
    cmd = ["hipcc", *FLAGS, *["-D%s=%s" % kv for kv in sorted(defines.items())], "-x", "hip", "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj


def build(verbose=False, defines=None, out=OUT, lib=LIB):
    """Compiles every source and links `lib`.  `defines` override csrc/tuning.h values."""
    os.makedirs(out, exist_ok=True)
    defines = dict(defines or {})
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, out, defines), SOURCES))
    tmp = lib + ".tmp"
    subprocess.check_call(["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, lib)
    if lib == LIB:
        build_probe()
    if verbose:
        print(lib)
    return lib


def build_probe(out=OUT):
    """Compiles and links the VALU issue-rate probe (libvalupeak.so)."""
    os.makedirs(out, exist_ok=True)
    obj = _compile(PROBE_SRC, out, {})
    tmp = PROBE_LIB + ".tmp"
    subprocess.check_call(["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", obj, "-o", tmp])
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
