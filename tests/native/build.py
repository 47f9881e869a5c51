"""Build the native GPU check programs of the test suite into
tests/native/_bin/: the HIP programs (tests/native/*.hip) with the library's
compiler flags, and the C clients of the library (tests/native/abi_frame.c,
after libmr.so is built) with gcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
BIN = os.path.join(HERE, "_bin")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
PROGRAMS = ["recip_check"]
# C clients of the library (gcc, linked against libmr.so and the HIP runtime)
C_PROGRAMS = ["abi_frame"]
ROOT = os.path.dirname(os.path.dirname(HERE))
LIBDIR = os.path.join(ROOT, "paper_1906_04576_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def path(name: str) -> str:
    return os.path.join(BIN, name)


def build(verbose: bool = False) -> None:
    os.makedirs(BIN, exist_ok=True)
    for name in PROGRAMS:
        cmd = [HIPCC] + FLAGS + [os.path.join(HERE, name + ".hip"), "-o", path(name)]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {name}:\n{r.stderr}")
        if verbose:
            print("built", path(name))
    for name in C_PROGRAMS:
        rpath = "$ORIGIN/" + os.path.relpath(LIBDIR, BIN) + ":" + os.path.join(ROCM, "lib")
        cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
               "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), os.path.join(HERE, name + ".c"),
               "-L", LIBDIR, "-lmr", "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lm", "-Wl,-rpath," + rpath,
               "-o", path(name)]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"gcc failed for {name}:\n{r.stderr}")
        if verbose:
            print("built", path(name))


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
