"""Host-side checks of the C ABI (no GPU needed): the built library loads and
exports every function include/*.h declares; the Python binding refuses to
run without it instead of falling back to anything else."""
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("adr.h", "adr_cnn.h")]
LIB = os.path.join(ROOT, "paper_1308_5215_amd", "libadr.so")


def declared():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(adr_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_every_header_is_checked():
    found = sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))
    assert found == sorted(os.path.basename(h) for h in HEADERS)


def test_header_declares_the_three_calls_of_the_method():
    names = declared()
    for n in ("adr_assemble", "adr_ilu0", "adr_bicgstab_solve"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libadr.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(adr_[a-z0-9_]+)$", out, flags=re.M))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libadr.so not built")
def test_library_loads_and_binding_lists_every_symbol():
    from paper_1308_5215_amd import _lib
    L = _lib.load()
    for n in declared():
        assert hasattr(L, n), n
    assert set(_lib.EXPORTS) == set(declared())
    assert L.adr_status_str(0) == b"ok"
    assert L.adr_status_str(4) == b"zero or non-finite pivot"


def test_binding_fails_loudly_without_the_library(tmp_path, monkeypatch):
    from paper_1308_5215_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(OSError):
        _lib.load()


def test_status_numbering_matches_the_oracle():
    from oracle import core
    from paper_1308_5215_amd import _lib
    for name in ("OK", "ERR_ARG", "MAXIT", "BREAKDOWN_RHO", "OMEGA_ZERO", "ZERO_PIVOT", "NONFINITE"):
        assert getattr(core, name) == getattr(_lib, name)


def test_amplification_helper():
    """The paper's amplification factor ||r^{k+1}|| / ||r^k|| of a history."""
    import paper_1308_5215_amd as adr
    np.testing.assert_array_equal(adr.amplification([4.0, 2.0, 1.0, 0.25]), [0.5, 0.5, 0.25])


@pytest.mark.skipif(not os.path.exists(LIB), reason="libadr.so not built")
def test_schedule_settings_reject_a_missing_problem():
    """The sweep-schedule settings check their arguments on the host before any
    device work: a NULL problem is an argument error, and reports no ring."""
    from paper_1308_5215_amd import _lib
    L = _lib.load()
    assert L.adr_set_sweep_ring(None, 1) == _lib.ERR_ARG
    assert b"NULL" in L.adr_last_error()
    assert L.adr_set_sweep_rows(None, 32) == _lib.ERR_ARG
    assert L.adr_sweep_ring(None) == 0
