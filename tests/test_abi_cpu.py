"""The C-ABI library loads and exports every symbol include/pvfl.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pvfl.h")
LIB = os.path.join(ROOT, "paper_2405_00482_amd", "libpvfl.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pvfl_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for must in ("pvfl_keygen", "pvfl_rotkeys_gen", "pvfl_plan_create", "pvfl_matmul_ct_pt",
                 "pvfl_encrypt_coeffs", "pvfl_decrypt_coeffs", "pvfl_export_coeffs"):
        assert must in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpvfl.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (pvfl_[a-z0-9_]+)", out))
    assert set(declared_symbols()) <= exported


def test_binding_imports_without_gpu():
    from paper_2405_00482_amd import pvfl
    assert pvfl.PLAN_HYBRID == 0
