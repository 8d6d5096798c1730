"""The C-ABI library loads and exports every function include/sacd.h
declares (CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sacd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sacd_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ["sacd_create_tensor", "sacd_init_factors", "sacd_sweep", "sacd_fit",
                     "sacd_run_until", "sacd_destroy_model", "sacd_destroy_tensor"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2003_03572_amd import sacd
    if not os.path.exists(sacd.LIB_PATH):
        pytest.fail(f"{sacd.LIB_PATH} is not built: run python -m paper_2003_03572_amd.build")
    lib = ctypes.CDLL(sacd.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_library_static_entry_points_without_gpu():
    from paper_2003_03572_amd import sacd
    L = sacd.lib()
    assert L.sacd_version().decode() == "0.1.0"
    assert L.sacd_status_string(-2).decode() == "index out of range"
    # argument checks happen before any device call
    out = ctypes.c_void_p()
    rc = L.sacd_init_factors(None, 8, ctypes.c_uint64(1), 0, 0, ctypes.byref(out))
    assert rc == -1
    assert b"NULL" in L.sacd_last_error()


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2003_03572_amd import sacd
    monkeypatch.setattr(sacd, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(sacd, "_lib", None)
    with pytest.raises(RuntimeError):
        sacd.lib()


def test_job_bytes_bound_without_gpu():
    """The admission bound is host arithmetic: positive, growing with nnz and rank."""
    from paper_2003_03572_amd import sacd
    r8, t8 = sacd.job_bytes((100, 200, 300), 10_000, 8)
    r64, _ = sacd.job_bytes((100, 200, 300), 10_000, 64)
    rbig, tbig = sacd.job_bytes((100, 200, 300), 100_000, 8)
    assert 0 < r8 < r64 and r8 < rbig and 0 < t8 < tbig
    # at least the three sorted copies (12 bytes per entry each) and the factors
    assert r8 >= 36 * 10_000 + 4 * 8 * 600
