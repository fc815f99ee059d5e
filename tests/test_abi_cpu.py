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


def test_binding_refuses_wrong_tensors_before_the_library():
    """the binding checks dtype, device, contiguity and size of every buffer
    it hands to the library (a wrong tensor would otherwise become an
    out-of-bounds device access); a CPU tensor is refused without a GPU"""
    import torch
    from paper_2405_00482_amd import pvfl
    for t, dtype, nbytes, status in ((torch.zeros(4, dtype=torch.float64), "float64", 0, pvfl.E_INVALID),
                                     (None, "float64", 0, pvfl.E_INVALID)):
        with pytest.raises(pvfl.PvflError) as e:
            pvfl._dev(t, "buffer", nbytes, dtype)
        assert e.value.status == status
    with pytest.raises(pvfl.PvflError) as e:
        pvfl._dev_rows(torch.zeros(3, 4, dtype=torch.float32), "matrix", 3, 4)
    assert e.value.status == pvfl.E_INVALID
