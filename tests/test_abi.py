"""The C-ABI library builds, loads and exports every entry point that
include/dcgs.h declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dcgs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dcgs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    from paper_2511_23030_amd import build, dcgs
    if not os.path.exists(dcgs.LIB_PATH):
        build.build()
    return dcgs.LIB_PATH


def test_header_declares_the_method_calls():
    names = declared_functions()
    for required in ("dcgs_select_chunks", "dcgs_compact", "dcgs_render_fwd",
                     "dcgs_render_bwd", "dcgs_adam_step"):
        assert required in names
    assert len(names) >= 20


def test_library_exports_every_declared_symbol(libpath):
    L = ctypes.CDLL(libpath)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_signatures_cover_the_header(libpath):
    from paper_2511_23030_amd import dcgs
    assert set(declared_functions()) == set(dcgs.SIGNATURES)
    L = dcgs.lib()
    assert L.dcgs_version().decode().startswith("dcgs")


def test_null_arguments_are_rejected_without_touching_the_device(libpath):
    from paper_2511_23030_amd import dcgs
    L = dcgs.lib()
    assert L.dcgs_create(None, 0) == 1              # DCGS_E_INVALID
    assert L.dcgs_render_fwd(None, None, None, 0, 0, 0, None, 0, None, 1, None, 16, 16, 0,
                             None, None, None, None) == 1
    assert L.dcgs_adam_step(None, None, None, 0, 0, None, None) == 1
    assert L.dcgs_state_info(None, None, None, None, None) == 1
    assert L.dcgs_last_error(None) == b"null context"


def test_pair_overflow_decision_is_taken_in_64_bits(libpath):
    """The decision each forward takes on its pair count (the device sums
    the count in 64 bits): a count that a 32-bit sum would wrap to a small
    number, or that 32-bit pair indexing cannot address, is an overflow."""
    from paper_2511_23030_amd import dcgs
    L = dcgs.lib()
    OK, CAP = 0, 2
    eager = 2**63 - 1               # an eager forward sizes its buffers after the count
    assert L.dcgs_pairs_fit(0, eager) == OK
    assert L.dcgs_pairs_fit(2**31 - 1, eager) == OK
    assert L.dcgs_pairs_fit(2**31, eager) == CAP     # beyond int32 ranges / list positions
    assert L.dcgs_pairs_fit(2**32, eager) == CAP     # wraps to 0 in a 32-bit sum
    assert L.dcgs_pairs_fit(2**32 + 5, eager) == CAP  # wraps to 5
    assert L.dcgs_pairs_fit(1000, 999) == CAP        # a window's pair capacity
    assert L.dcgs_pairs_fit(999, 999) == OK


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2511_23030_amd import dcgs
    monkeypatch.setattr(dcgs, "_lib", None)
    monkeypatch.setattr(dcgs, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(dcgs.LibraryMissing):
        dcgs.lib()
