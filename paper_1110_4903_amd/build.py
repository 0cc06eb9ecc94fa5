"""Build libkin.so (HIP, gfx950) in-tree.

    python -m paper_1110_4903_amd.build

Steps: embed the lane-layout device template as a string (csrc/kin_lane_template.inc), then
compile the C-ABI runtime, the code generator and the precompiled wave-layout kernels with
hipcc into paper_1110_4903_amd/libkin.so, linked against hipRTC.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libkin.so")
SOURCES = ["kin_runtime.cpp", "kin_codegen.cpp", "kin_wave.hip", "kin_global.hip", "kin_order.hip", "kin_fluid.hip"]
HEADERS = ["kin_internal.h", "kin_lane_template.h", "kin_xlane.h"]

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
ARCH = os.environ.get("KIN_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", "-Wno-unused-value",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the wave layout fully unrolls its elimination so matrix rows stay in registers
    "-mllvm", "-pragma-unroll-threshold=1000000",
]


def embed_template() -> str:
    """Write the device template as a C++ raw string literal (re-written only if changed)."""
    src = os.path.join(CSRC, "kin_lane_template.h")
    dst = os.path.join(CSRC, "kin_lane_template.inc")
    with open(src) as f:
        body = f.read()
    if ")KINTPL\"" in body:
        raise RuntimeError("template contains the raw-string delimiter")
    text = 'R"KINTPL(' + body + ')KINTPL"\n'
    if not os.path.exists(dst) or open(dst).read() != text:
        with open(dst, "w") as f:
            f.write(text)
    return dst


def build(verbose: bool = False) -> str:
    embed_template()
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for s in SOURCES:
        obj = os.path.join(build_dir, os.path.splitext(s)[0] + ".o")
        cmd = [HIPCC, *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               "-c", os.path.join(CSRC, s), "-o", obj]
        if s.endswith(".cpp"):
            cmd.insert(1, "-x")
            cmd.insert(2, "hip")
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = SO + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lhiprtc"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, SO)
    return SO


def build_abi_check(verbose: bool = False) -> str:
    """The C-only check of the ABI (tests/abi_c/kin_abi_check.c), linked against libkin.so."""
    src = os.path.join(ROOT, "tests", "abi_c", "kin_abi_check.c")
    exe = os.path.join(ROOT, "tests", "abi_c", "kin_abi_check")
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-I", os.path.join(ROOT, "include"), src,
           "-L", HERE, "-lkin", "-Wl,-rpath," + HERE, "-Wl,-rpath,/opt/rocm/lib", "-lm", "-o", exe]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return exe


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
