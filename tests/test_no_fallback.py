"""The product path has no CPU fallback and never touches the oracle."""
import ast
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2606_06386_amd")


def test_package_never_imports_the_oracle():
    for f in sorted(os.listdir(PKG)):
        if not f.endswith(".py"):
            continue
        tree = ast.parse(open(os.path.join(PKG, f)).read())
        for node in ast.walk(tree):
            names = []
            if isinstance(node, ast.Import):
                names = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                names = [node.module or ""]
            assert not any(n == "oracle" or n.startswith("oracle.") for n in names), f


def test_missing_library_raises(monkeypatch):
    from paper_2606_06386_amd import binding, build
    monkeypatch.setattr(build, "LIB", os.path.join(ROOT, "no-such-libmpdiv.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        binding.lib()
