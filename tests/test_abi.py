"""The C ABI library loads and exports every function that include/sdf.h
declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "sdf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sdf_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("sdf_index_build", "sdf_search", "sdf_search_batch", "sdf_result_copy",
              "sdf_result_free", "sdf_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1807_00205_amd import sdf
    lib = ctypes.CDLL(sdf.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(sdf.EXPORTS) == _declared()


def test_binding_layouts_match_header():
    from paper_1807_00205_amd import sdf
    assert sdf.CANDIDATE_DTYPE.itemsize == 56
    assert sdf.SEED_DTYPE.itemsize == 24
    assert ctypes.sizeof(sdf._Span) == 24
    assert ctypes.sizeof(sdf._SearchParams) == 16
