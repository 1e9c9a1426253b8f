"""The oracle and the GPU library stay independent: the package never imports
the oracle, the shared library neither links nor exports oracle code, the C
oracle includes only the C standard headers, and the package's sources name
nothing under oracle/.  The seeded input generators (workloads.py) are the one
module both sides use, and they hold no generator arithmetic."""
import ast
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1412_8266_amd")
LIB = os.path.join(PKG, "libmrg32k3a_gpu.so")


def _py_files(d):
    for base, _, files in os.walk(d):
        for f in files:
            if f.endswith(".py"):
                yield os.path.join(base, f)


def _imported_modules(path):
    tree = ast.parse(open(path).read(), path)
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            for a in node.names:
                yield a.name
        elif isinstance(node, ast.ImportFrom):
            yield node.module or ""


def test_package_never_imports_the_oracle():
    for path in _py_files(PKG):
        for mod in _imported_modules(path):
            assert mod.split(".")[0] != "oracle", (path, mod)


def test_native_sources_name_no_oracle_file():
    csrc = os.path.join(PKG, "csrc")
    for f in os.listdir(csrc) + [os.path.join("..", "..", "include", h)
                                 for h in os.listdir(os.path.join(ROOT, "include"))]:
        text = open(os.path.join(csrc, f)).read()
        assert "mrg32k3a_oracle" not in text and "orc_" not in text, f


@pytest.mark.parametrize("name", ["mrg32k3a_oracle.c", "tinymt_oracle.c"])
def test_oracle_c_includes_only_the_c_library(name):
    src = open(os.path.join(ROOT, "oracle", name)).read()
    heads = re.findall(r"#include\s*[<\"]([^>\"]+)[>\"]", src)
    assert heads and all(h in ("stdint.h", "stddef.h", "string.h", "stdlib.h", "stdio.h")
                         for h in heads), heads


def test_workloads_hold_no_generator_arithmetic():
    text = open(os.path.join(PKG, "workloads.py")).read()
    for word in ("4294967087", "4294944443", "1403580", "810728", "527612", "1370589"):
        assert word not in text, word


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_links_and_exports_no_oracle_code():
    needed = subprocess.run(["readelf", "-d", LIB], capture_output=True, text=True).stdout
    assert "oracle" not in needed
    syms = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True,
                          text=True).stdout
    assert syms and not re.search(r"\borc_", syms)


def test_importing_the_package_leaves_the_oracle_unloaded():
    code = ("import sys; sys.path.insert(0, %r)\n"
            "try:\n    import paper_1412_8266_amd\nexcept Exception:\n    pass\n"
            "print(any(m == 'oracle' or m.startswith('oracle.') for m in sys.modules))" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         timeout=300, cwd="/")
    assert out.stdout.strip().splitlines()[-1] == "False", out.stdout + out.stderr
