"""The bench reports a kernel's stored counters only while the library holds
the machine code they were taken on: the build records the SHA-256 of each
source's gfx950 code (.text and .rodata of its device code object) in
libmr.code.json, the same for every build of the same code, unchanged by
comments and changed by code."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_1906_04576_amd import build as B  # noqa: E402

KERNEL = """#include <hip/hip_runtime.h>
// %s
__global__ void k(float* o, float a) { o[threadIdx.x] = o[threadIdx.x] * a + %s; }
"""


def _obj(tmp_path, name, comment, const):
    src = tmp_path / (name + ".hip")
    src.write_text(KERNEL % (comment, const))
    obj = tmp_path / (name + ".o")
    flags, skip = [], False
    for f in B.FLAGS:
        if skip:
            skip = False
            continue
        if f == "-I":
            skip = True
            continue
        flags.append(f)
    r = subprocess.run([B.HIPCC] + flags + ["-c", str(src), "-o", str(obj)], capture_output=True, text=True,
                       timeout=300)
    if r.returncode != 0:
        pytest.skip("hipcc unavailable: " + r.stderr[-300:])
    return str(obj)


def test_code_hash_follows_code_not_comments(tmp_path):
    h1 = B.device_code_sha256(_obj(tmp_path, "a", "first", "1.0f"))
    h2 = B.device_code_sha256(_obj(tmp_path, "b", "a different comment", "1.0f"))
    h3 = B.device_code_sha256(_obj(tmp_path, "c", "first", "2.0f"))
    assert h1 and len(h1) == 64
    assert h1 == h2
    assert h3 != h1


def test_the_build_records_the_evaluation_kernels():
    code = json.load(open(B.CODE))
    assert len(code.get("k_ssao.hip", "")) == 64
    assert "api.cpp" not in code  # no device code


def test_counters_follow_the_recorded_code(tmp_path):
    p = tmp_path / "code.json"
    p.write_text(json.dumps({"k_ssao.hip": bench.COUNTER_CODE["k_ssao_multi"][1]}))
    assert bench.counters_current("k_ssao_multi", str(p))
    p.write_text(json.dumps({"k_ssao.hip": "0" * 64}))
    assert not bench.counters_current("k_ssao_multi", str(p))
    assert not bench.counters_current("k_ssao_multi", str(tmp_path / "missing.json"))
