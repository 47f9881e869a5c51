"""The bench reports a kernel's stored counters only while the kernel's
code is the one they were taken with: the hash covers the code of the .hip
file and every header it includes, transitively, comments and white space
aside."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _write(d, name, text):
    with open(os.path.join(d, name), "w") as f:
        f.write(text)


def test_hash_covers_included_headers(tmp_path):
    a, b = tmp_path / "src", tmp_path / "inc"
    a.mkdir()
    b.mkdir()
    _write(a, "k.hip", '#include "x.hpp"\n#include <hip/hip_runtime.h>\n')
    _write(a, "x.hpp", '#pragma once\n  #  include "y.h"\n')
    _write(b, "y.h", "int v = 1;\n")
    h0 = bench.source_closure_sha256("k.hip", [str(a), str(b)])
    assert h0 == bench.source_closure_sha256("k.hip", [str(a), str(b)])
    _write(b, "y.h", "int v = 2;\n")              # a header two levels down
    h1 = bench.source_closure_sha256("k.hip", [str(a), str(b)])
    assert h1 != h0
    _write(b, "y.h", "int v = 2;  // a comment\n/* another */\n")  # comments and white space only
    assert bench.source_closure_sha256("k.hip", [str(a), str(b)]) == h1
    _write(b, "y.h", 'const char* s = "// kept"; int v = 2;\n')  # a string is code
    assert bench.source_closure_sha256("k.hip", [str(a), str(b)]) != h1


def test_code_only():
    src = b'int a; // c\n/* x\n y */ const char* s = "/* no */";  char q = \'\\\'\';\n\tint  b;'
    assert bench.code_only(src) == b'int a; const char* s = "/* no */"; char q = \'\\\'\'; int b;'


def test_missing_header_is_an_error(tmp_path):
    _write(tmp_path, "k.hip", '#include "nowhere.hpp"\n')
    with pytest.raises(FileNotFoundError):
        bench.source_closure_sha256("k.hip", [str(tmp_path)])


def test_the_evaluation_kernel_closure_holds_its_headers():
    # every header the evaluation kernel includes is found among the sources
    assert len(bench.source_closure_sha256("k_ssao.hip")) == 64
