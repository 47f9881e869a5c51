"""Build libmr.so in-tree with hipcc for gfx950, and beside it
libmr.code.json: the SHA-256 of each source's gfx950 machine code.

Flags: -O3 for gfx950 only; -ffp-contract=off so that no multiply-add is
fused (the arithmetic contract in include/mr.h); packed FP32 instructions are
disabled; correctly rounded FP32 division and square root are HIP's default
and are left on.
"""
from __future__ import annotations

import hashlib
import json
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmr.so")
# SHA-256 of each source's gfx950 machine code, written beside the library
CODE = os.path.join(HERE, "libmr.code.json")
LLVM = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin")

SOURCES = ["api.cpp", "k_masks.hip", "k_compact.hip", "k_ssao.hip", "k_ssao_tiles.hip", "k_shadow.hip", "k_ssgi.hip",
           "k_fused.hip",
           "k_merge.hip",
           "k_lean.hip", "k_bilateral.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-x", "hip", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-fvisibility=hidden", "-Wall", "-Wno-unused-function", "-Wno-bitwise-instead-of-logical", "-I", INCLUDE, "-I", CSRC]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def device_code_sha256(obj: str) -> str | None:
    """SHA-256 of the gfx950 machine code and kernel descriptors (.text and
    .rodata of the device code object) in an object file, or None when it
    has no device code.  The same for every build of the same code: comments, and host
    declarations the kernels do not use, leave it unchanged."""
    with tempfile.TemporaryDirectory() as t:
        fb, co = os.path.join(t, "fatbin"), os.path.join(t, "co")
        r = subprocess.run([os.path.join(LLVM, "llvm-objcopy"), "--dump-section", f".hip_fatbin={fb}", obj,
                            os.path.join(t, "host.o")], capture_output=True, text=True)
        if r.returncode != 0 or not os.path.exists(fb):
            return None
        subprocess.run([os.path.join(LLVM, "clang-offload-bundler"), "--unbundle", "--type=o",
                        "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--input={fb}", f"--output={co}"],
                       check=True, capture_output=True)
        h = hashlib.sha256()
        text = False
        for sec in (".text", ".rodata"):  # a section the code object lacks counts as empty
            out = os.path.join(t, sec[1:])
            r = subprocess.run([os.path.join(LLVM, "llvm-objcopy"), "--dump-section", f"{sec}={out}", co,
                                os.path.join(t, "dev.o")], capture_output=True)
            data = b""
            if r.returncode == 0 and os.path.exists(out):
                with open(out, "rb") as f:
                    data = f.read()
            text = text or (sec == ".text" and len(data) > 0)
            h.update(sec.encode() + b"\0" + data)
        return h.hexdigest() if text else None


def build(verbose: bool = False) -> str:
    """Compile every kernel source and link libmr.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    code = {src: device_code_sha256(obj) for src, obj in zip(SOURCES, objs)}
    with open(CODE, "w") as f:
        json.dump({k: v for k, v in code.items() if v}, f, indent=1, sort_keys=True)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
