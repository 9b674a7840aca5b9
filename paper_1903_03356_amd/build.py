"""Builds the HIP library ``liblbib.so`` for gfx950, in-tree.

    python -m paper_1903_03356_amd.build
"""
from __future__ import annotations

import os
import re
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbib.so")
SOURCES = ["lbib_kernels.hip", "lbib_adjoint.hip", "lbib_api.hip"]
ARCH = os.environ.get("LBIB_OFFLOAD_ARCH", "gfx950")


# Packed FP32 instructions (v_pk_add/mul/fma_f32) are kept out of the device
# code: the target feature below switches them off in the gfx950 pass.  The
# host pass does not know the feature and prints "not a recognized feature for
# this target (ignoring feature)"; that warning concerns x86 code only.  The
# build does not rely on the flag alone: ``check_no_packed_fp32`` compiles every
# source to gfx950 assembly with the same flags and fails on any such opcode.
NO_PACKED_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
PACKED_FP32_OPCODE = re.compile(r"\bv_pk_(?:add|mul|fma)_f32\b")


def common_flags() -> list:
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC"] + NO_PACKED_FP32 + [
        "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def hipcc_cmd(out: str) -> list:
    return ["hipcc", "-shared"] + common_flags() + ["-o", out] + [
        os.path.join(CSRC, s) for s in SOURCES]


def check_no_packed_fp32(verbose: bool = False) -> None:
    """Compile each source's device code to assembly with the library's flags
    and raise if a packed FP32 opcode appears."""
    with tempfile.TemporaryDirectory() as tmp:
        for src in SOURCES:
            asm = os.path.join(tmp, src + ".s")
            cmd = ["hipcc", "--cuda-device-only", "-S"] + common_flags() + [
                "-o", asm, os.path.join(CSRC, src)]
            subprocess.run(cmd, check=True, stderr=subprocess.DEVNULL if not verbose else None)
            with open(asm) as f:
                hits = sorted(set(PACKED_FP32_OPCODE.findall(f.read())))
            if hits:
                raise RuntimeError(f"{src}: packed FP32 opcodes in the gfx950 code: {hits}")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = hipcc_cmd(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    check_no_packed_fp32()
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
