"""The oracle and the library share no code: no module under oracle/ imports the
product package, and the product package neither imports nor loads the oracle."""
import ast
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = "paper_1602_05510_amd"


def _imports(path):
    tree = ast.parse(open(path).read(), filename=path)
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            for a in node.names:
                yield a.name
        elif isinstance(node, ast.ImportFrom):
            yield node.module or ""


def _files(top, exts):
    for dirpath, _, names in os.walk(os.path.join(ROOT, top)):
        if "__pycache__" in dirpath:
            continue
        for n in names:
            if n.endswith(exts):
                yield os.path.join(dirpath, n)


def test_oracle_imports_nothing_from_the_product():
    for p in _files("oracle", (".py",)):
        for mod in _imports(p):
            assert not mod.startswith(PKG), f"{p} imports {mod}"
    for p in _files("oracle", (".c", ".h")):
        src = open(p).read()
        assert "hesp_core.h" not in src and "hesp.h" not in src and PKG not in src, p


def test_product_never_touches_the_oracle():
    for p in _files(PKG, (".py",)):
        for mod in _imports(p):
            assert not mod.startswith("oracle"), f"{p} imports {mod}"
        assert "liboracle" not in open(p).read(), p
    for p in _files(os.path.join(PKG, "csrc"), (".hip", ".cpp", ".h")):
        src = open(p).read()
        assert "oracle" not in src.lower(), p
