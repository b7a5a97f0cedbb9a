"""The C-ABI library loads and exports every function declared in include/*.h."""

import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(recoil_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


def test_exports_every_declared_symbol():
    import paper_2306_12141_amd._lib as L
    names = _declared()
    assert len(names) >= 12
    missing = [n for n in sorted(names) if not hasattr(L.lib, n)]
    assert not missing, missing


def test_library_is_gfx950_hip():
    so = os.path.join(ROOT, "paper_2306_12141_amd", "librecoil.so")
    data = open(so, "rb").read()
    assert b"gfx950" in data
    import paper_2306_12141_amd as rc
    assert "gfx950" in rc.version()
