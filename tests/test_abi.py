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
    assert ctypes.sizeof(sdf._Tuning) == 4 * len(sdf.TUNING_FIELDS) == 100


def test_tuning_is_per_thread():
    """Settings (host state only, no GPU call) are the calling thread's:
    another thread keeps the library's choices; the context puts the
    previous settings back; a workgroup size other than 512 or 1024 is
    rejected."""
    import threading
    from paper_1807_00205_amd import sdf
    assert all(v == sdf.AUTO for v in sdf.get_tuning().values())
    seen = {}
    with sdf.tuning(tile_core=640, tile_threads=512):
        with sdf.tuning(kept_cap=64):
            t = sdf.get_tuning()
            assert (t["tile_core"], t["tile_threads"], t["kept_cap"]) == (640, 512, 64)
        th = threading.Thread(target=lambda: seen.update(sdf.get_tuning()))
        th.start()
        th.join()
        assert sdf.get_tuning()["kept_cap"] == sdf.AUTO
    assert all(v == sdf.AUTO for v in seen.values())
    assert all(v == sdf.AUTO for v in sdf.get_tuning().values())
    try:
        sdf.set_tuning(tile_threads=256)
        raise AssertionError("tile_threads 256 accepted")
    except sdf.SdfError as e:
        assert e.code == sdf.SDF_EINVAL
    assert sdf.get_tuning()["tile_threads"] == sdf.AUTO
