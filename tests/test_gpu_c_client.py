"""A C program (tests/native/abi_frame.c, built by tests/native/build.py)
runs frames on the GPU through the C boundary alone: hipMalloc'd buffers,
mr_workspace_bytes, mr_frame on the multi-resolution and naive paths and
mr_frame_tune, on a plane whose images are exactly 0."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "native", "_bin", "abi_frame")


def test_c_client_runs_frames():
    assert os.path.exists(EXE), "build it first: python tests/native/build.py (or __graft_entry__.build())"
    print("[gpu] tests/native/_bin/abi_frame", flush=True)
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    print(r.stdout, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failure(s)" in r.stdout and "FAIL" not in r.stdout
