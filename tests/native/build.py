"""Build the native GPU check programs of the test suite (tests/native/*.hip)
into tests/native/_bin/ with the library's compiler flags."""
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


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
