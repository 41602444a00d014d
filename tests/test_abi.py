"""The C-ABI library builds, loads and exports every symbol include/mm.h declares
(CPU only: no call that touches a GPU)."""
import os
import re
import subprocess

import pytest

from paper_1406_7635_amd import build as mmbuild
from paper_1406_7635_amd import mm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "mm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mm.LIB_PATH):
        mmbuild.build()
    return mm.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(mm.EXPORTS), set(names) ^ set(mm.EXPORTS)


def test_exported_symbols_are_c_linkage():
    out = subprocess.run(["nm", "-D", "--defined-only", mm.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (mm_[a-z0-9_]+)$", out, flags=re.M))
    assert set(_declared()) <= exported


def test_strerror_is_host_only(lib):
    for code, name in mm.STATUS.items():
        s = lib.mm_strerror(code).decode()
        assert s and s != "unknown status", name
    assert lib.mm_strerror(12345).decode() == "unknown status"


def test_struct_sizes_match_header():
    import ctypes
    assert ctypes.sizeof(mm.Params) == 8 * (5 * 256 + 2 * 768 + 256 * 257 // 2 + 1)
    assert ctypes.sizeof(mm.Grid) == 3 * 4 + 4 + 3 * 8 + 3 * 4 + 4  # natural alignment padding


def test_fft_stage_emulation():
    """Host emulation of the LDS Stockham FFT (every length 1..4096, both
    directions) against a direct DFT."""
    exe = mmbuild.build_fft_host_check()
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout
