"""Repository discipline (CPU): the product package never reaches the oracle,
the binding fails loudly without the HIP library, and the oracle shares no
source with the HIP path."""
import ast
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2006_16861_amd")


def _py_files(d):
    for base, _, files in os.walk(d):
        for f in files:
            if f.endswith(".py"):
                yield os.path.join(base, f)


def _imports(path):
    tree = ast.parse(open(path).read(), path)
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            for a in node.names:
                yield a.name
        elif isinstance(node, ast.ImportFrom):
            yield node.module or ""


def test_package_never_imports_the_oracle():
    for f in _py_files(PKG):
        for mod in _imports(f):
            assert not mod.split(".")[0] == "oracle", f"{f} imports {mod}"


def test_native_sources_do_not_include_oracle_headers():
    csrc = os.path.join(PKG, "csrc")
    for f in os.listdir(csrc):
        txt = open(os.path.join(csrc, f), errors="ignore").read()
        assert "tdpo" not in txt, f
    txt = open(os.path.join(ROOT, "oracle", "tdpo.c")).read()
    assert not re.search(r'#include\s+"(tdp\.h|tdp_internal\.h)"', txt)


def test_bench_uses_the_oracle_only_in_its_cpu_baseline():
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    users = set()
    for fn in ast.walk(tree):
        if isinstance(fn, ast.FunctionDef):
            for node in ast.walk(fn):
                if isinstance(node, (ast.Import, ast.ImportFrom)):
                    names = [a.name for a in node.names] if isinstance(node, ast.Import) else [node.module]
                    if any(n and n.split(".")[0] == "oracle" for n in names):
                        users.add(fn.name)
    assert users <= {"cpu_baseline"}, users
    src = open(os.path.join(ROOT, "bench.py")).read()
    # the one-thread leg runs the oracle in a child process from cpu_baseline
    assert "import bench, oracle" in src


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    from paper_2006_16861_amd import tdp
    monkeypatch.setattr(tdp, "_lib", None)
    with pytest.raises(RuntimeError) as e:
        tdp.load(str(tmp_path / "missing.so"))
    assert "not found" in str(e.value)
