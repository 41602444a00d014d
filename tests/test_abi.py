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


def build_fft_host_check(sanitize=False):
    """The host emulation of the LDS FFT stages (tests/fft_host_check.cpp);
    with sanitize, host code built with AddressSanitizer and UBSan."""
    os.makedirs(mmbuild.OBJ, exist_ok=True)
    exe = os.path.join(mmbuild.OBJ, "fft_host_check" + ("_san" if sanitize else ""))
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fft_host_check.cpp")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"] if sanitize else []
    cmd = [mmbuild.HIPCC] + mmbuild.FLAGS + san + ["-x", "hip", src, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stderr
    return exe


def test_fft_stage_emulation():
    """Host emulation of the LDS Stockham FFT (every length 1..4096, both
    directions) against a direct DFT."""
    exe = build_fft_host_check()
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout


def test_fft_stage_emulation_sanitized():
    """The same emulation with AddressSanitizer and UBSan on the host code."""
    exe = build_fft_host_check(sanitize=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout
    assert "runtime error" not in r.stderr


def test_abi_validation_sanitized():
    """Argument validation and error cleanup of the C ABI's host code, built
    with AddressSanitizer (leak checks included) and UBSan and run without a
    GPU (tests/abi_host_check.cpp): every documented status, no report."""
    os.makedirs(mmbuild.OBJ, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in [x for x in mmbuild.SOURCES if x.endswith(".cpp")]:
        obj = os.path.join(mmbuild.OBJ, "san_" + os.path.splitext(src)[0] + ".o")
        cmd = [mmbuild.HIPCC] + mmbuild.FLAGS + san + ["-x", "hip", "-c", os.path.join(mmbuild.CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, " ".join(cmd) + "\n" + r.stderr
        objs.append(obj)
    kern = [os.path.join(mmbuild.OBJ, os.path.splitext(x)[0] + ".o") for x in mmbuild.SOURCES if x.endswith(".hip")]
    if not all(os.path.exists(k) for k in kern):
        mmbuild.build()
    exe = os.path.join(mmbuild.OBJ, "abi_host_check_san")
    drv = os.path.join(os.path.dirname(os.path.abspath(__file__)), "abi_host_check.cpp")
    cmd = [mmbuild.HIPCC] + mmbuild.FLAGS + san + ["-x", "hip", drv, "-x", "none"] + objs + kern + ["-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stderr
    env = dict(os.environ, HIP_VISIBLE_DEVICES="-1", ROCR_VISIBLE_DEVICES="-1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
