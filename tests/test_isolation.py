"""The oracle and the product path stay apart, and the product path has no
fallback: the package and the C sources name nothing under oracle/, the
oracle names nothing of the package but the seeded input generators, and the
binding raises when the HIP library is missing instead of computing
anything itself."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2012_11077_amd")
ORACLE = os.path.join(ROOT, "oracle")


def _sources(top, exts):
    for d, _, files in os.walk(top):
        if "_build" in d or "__pycache__" in d:
            continue
        for f in files:
            if f.endswith(exts):
                yield os.path.join(d, f)


def test_product_names_no_oracle():
    pat = re.compile(r"^\s*(import\s+oracle|from\s+oracle\b)|#include\s*[<\"][^>\"]*oracle", re.M)
    hits = []
    for p in list(_sources(PKG, (".py", ".hip", ".cpp", ".h"))) + list(_sources(os.path.join(ROOT, "include"), (".h",))):
        with open(p) as f:
            if pat.search(f.read()):
                hits.append(os.path.relpath(p, ROOT))
    assert not hits, hits


def test_oracle_uses_only_the_input_generators():
    pat = re.compile(r"^\s*(?:import|from)\s+paper_2012_11077_amd(?:\.(\w+))?", re.M)
    for p in _sources(ORACLE, (".py", ".c", ".h")):
        with open(p) as f:
            for m in pat.finditer(f.read()):
                assert m.group(1) == "synth", (p, m.group(0))


def test_binding_raises_without_library(monkeypatch, tmp_path):
    from paper_2012_11077_amd import cfar2d as C
    monkeypatch.setattr(C, "LIB_PATH", str(tmp_path / "libcfar2d.so"))
    monkeypatch.setattr(C, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        C.lib()
