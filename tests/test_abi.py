"""The C-ABI library builds, loads and exports every entry point declared in
include/nucleus.h (no compute calls: these run without a GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nucleus.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nd_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2306_08623_amd import nucleus
    if not os.path.exists(nucleus.LIB_PATH):
        from paper_2306_08623_amd import build
        build.build()
    return nucleus.load_library()


def test_header_declares_the_binding_exports():
    from paper_2306_08623_amd import nucleus
    assert _declared() == sorted(nucleus.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", lib._name], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\bT (nd_[a-z_]+)\b", out))
    assert set(_declared()) <= exported


def test_status_strings_without_gpu(lib):
    # a pure host function: safe without a device
    assert lib.nd_status_str(0) == b"ok"
    assert b"overflow" in lib.nd_status_str(5)


def test_library_links_no_oracle_code(lib):
    out = subprocess.run(["nm", "-D", lib._name], capture_output=True, text=True).stdout
    assert "ndo_" not in out
