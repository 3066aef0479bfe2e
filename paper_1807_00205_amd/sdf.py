"""ctypes binding of the C ABI declared in ``include/sdf.h``.

Argument marshalling only: every step of indexing and search runs in the HIP
kernels of ``libsdf.so``.  Loading fails loudly when the library has not been
built; there is no CPU path.
"""
from __future__ import annotations

import contextlib
import ctypes
import itertools
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsdf.so")

SDF_OK, SDF_EINVAL, SDF_ENOMEM, SDF_EDEVICE, SDF_ERANGE, SDF_EBUSY, SDF_EINTERNAL = (
    0, -1, -2, -3, -4, -5, -6)
SDF_TIMING = 1
SDF_SEED_ESTIMATE = 2
SDF_EXTEND = 4
STOP_BOUND, STOP_CAP, STOP_OVERLAP, STOP_ESTIMATE = 1, 2, 3, 4

CANDIDATE_DTYPE = np.dtype([("query_id", "<u4"), ("strand", "<u4"), ("q_seq", "<u4"),
                            ("t_seq", "<u4"), ("q_begin", "<u8"), ("q_end", "<u8"),
                            ("t_begin", "<u8"), ("t_end", "<u8"), ("n_seeds", "<u4"),
                            ("max_shared", "<u4")])
# sdf_region: a region pair and, after an extension, its final estimate
# (m / s) and stop codes (forward | backward << 8).
REGION_DTYPE = np.dtype([("strand", "<u4"), ("q_seq", "<u4"), ("t_seq", "<u4"), ("stop", "<u4"),
                         ("q_begin", "<u8"), ("q_end", "<u8"), ("t_begin", "<u8"),
                         ("t_end", "<u8"), ("m", "<u4"), ("s", "<u4")])
# sdf_sd: one final SD (Section 3.3) with its CIGAR operations at
# [cigar_off, cigar_off + cigar_len) of the operation array.
SD_DTYPE = np.dtype([("region", "<u8"), ("strand", "<u4"), ("q_seq", "<u4"), ("t_seq", "<u4"),
                     ("_pad", "<u4"), ("q_begin", "<u8"), ("q_end", "<u8"), ("t_begin", "<u8"),
                     ("t_end", "<u8"), ("aln_len", "<u4"), ("matches", "<u4"),
                     ("mismatches", "<u4"), ("ins", "<u4"), ("dels", "<u4"), ("gap_opens", "<u4"),
                     ("transitions", "<u4"), ("transversions", "<u4"), ("k2p", "<f8"),
                     ("jc", "<f8"), ("cigar_off", "<u8"), ("cigar_len", "<u8")])
CIGAR_CHARS = {7: "=", 8: "X", 1: "I", 2: "D"}
SEED_DTYPE = np.dtype([("query_id", "<u4"), ("i", "<u4"), ("j", "<u4"), ("strand", "<u4"),
                       ("shared", "<u4"), ("sketch", "<u4")])
EXPORTS = ["sdf_last_error", "sdf_index_build", "sdf_index_info", "sdf_index_hit_density",
           "sdf_index_minimizers",
           "sdf_index_entries", "sdf_index_packed", "sdf_index_free", "sdf_search",
           "sdf_search_batch", "sdf_result_count", "sdf_result_copy", "sdf_result_seed_count",
           "sdf_result_seeds", "sdf_result_timing", "sdf_result_stats", "sdf_result_free",
           "sdf_extend", "sdf_result_regions", "sdf_qgram_filter", "sdf_autotune",
           "sdf_search_batch_noalloc", "sdf_plan_create", "sdf_plan_run", "sdf_plan_info",
           "sdf_plan_free", "sdf_search_batch_capped", "sdf_align_regions", "sdf_sds_count",
           "sdf_sds_copy", "sdf_sds_free", "sdf_tuning_defaults", "sdf_set_tuning",
           "sdf_get_tuning", "sdf_index_save", "sdf_index_load", "sdf_index_shape"]
NOALLOC_SCRATCH_BYTES = 128 << 20
# Section 3.2 pads every potential SD region by a number of bases that grows
# with its size but gives no formula: here a tenth of each side's length at
# both ends.
PAD_FRAC = 0.1
NOALLOC_MAX_SPANS = 65536
NOALLOC_MAX_QUERY_BASES = 8_000_000


def _flags(timing: bool, estimate: bool, extend: bool = False) -> int:
    return ((SDF_TIMING if timing else 0) | (SDF_SEED_ESTIMATE if estimate else 0) |
            (SDF_EXTEND if extend else 0))


class SdfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("sdf error %d: %s" % (code, msg))
        self.code = code


class _IndexParams(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("w", ctypes.c_uint32)]


AUTO = 0xFFFFFFFF
TUNING_FIELDS = ("tile_threads", "tile_core", "hits_per_part", "wg_per_cu", "span_few_max",
                 "kept_cap", "phase_prof", "chain_fused_max", "cand_sort_general",
                 "cand_sort_small_max", "cand_tie_max", "est_lds_cap", "est_reg_cap",
                 "est_first_amax", "ext_h0", "ext_lds_words", "ext_hb0", "ext_hdiv",
                 "ext_batch_min", "ext_ecap", "ext_stats", "align_wave_cells",
                 "align_wave_lds_cols", "align_lds_blocks", "align_lds_ids")


class _Tuning(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint32) for f in TUNING_FIELDS]


class _SearchParams(ctypes.Structure):
    _fields_ = [("max_error", ctypes.c_double), ("min_len", ctypes.c_uint32),
                ("flags", ctypes.c_uint32)]


class _ExtendParams(ctypes.Structure):
    _fields_ = [("max_error", ctypes.c_double), ("max_len", ctypes.c_uint64)]


class _QgramParams(ctypes.Structure):
    _fields_ = [("max_error", ctypes.c_double), ("gap_rate", ctypes.c_double),
                ("q", ctypes.c_uint32), ("_pad", ctypes.c_uint32)]


class _PlanParams(ctypes.Structure):
    _fields_ = [("seed_cap", ctypes.c_uint64), ("cand_cap", ctypes.c_uint64)]


class _AlignParams(ctypes.Structure):
    _fields_ = [("max_error", ctypes.c_double), ("min_len", ctypes.c_uint32),
                ("k", ctypes.c_uint32), ("pad_frac", ctypes.c_double)]


class _Span(ctypes.Structure):
    _fields_ = [("seq", ctypes.c_uint32), ("_pad", ctypes.c_uint32),
                ("begin", ctypes.c_uint64), ("end", ctypes.c_uint64)]


# sdf_span as a NumPy record: for long span lists, filling one is several
# times faster than building one ctypes structure per span
_SPAN_DTYPE = np.dtype([("seq", np.uint32), ("_pad", np.uint32), ("begin", np.uint64),
                        ("end", np.uint64)])
assert _SPAN_DTYPE.itemsize == ctypes.sizeof(_Span)


def _span_array(spans):
    """(seq, begin, end) triples as a contiguous sdf_span array (at least one
    record, so the pointer is never NULL) and their count.  Values that do
    not fit the fields wrap as ctypes would wrap them; the library rejects
    them."""
    spans = list(spans)
    n = len(spans)
    if n < 32:  # few spans: ctypes directly is cheaper than the NumPy calls
        c = (_Span * max(1, n))(*[_Span(q, 0, b, e) for (q, b, e) in spans])
        return np.frombuffer(bytearray(c), dtype=_SPAN_DTYPE), n
    arr = np.zeros(n, _SPAN_DTYPE)
    a = None
    try:
        # triples of integers only (floats would be truncated by fromiter)
        if (set(map(len, spans)) == {3}
                and all(issubclass(t, (int, np.integer))
                        for t in set(map(type, itertools.chain.from_iterable(spans))))):
            a = np.fromiter(itertools.chain.from_iterable(spans), np.int64, 3 * n).reshape(n, 3)
            if (a < 0).any():
                a = None
    except (OverflowError, ValueError, TypeError):
        a = None
    if a is not None:
        arr["seq"] = a[:, 0].astype(np.uint32, casting="unsafe")
        arr["begin"] = a[:, 1].astype(np.uint64)
        arr["end"] = a[:, 2].astype(np.uint64)
    else:  # anything else goes through ctypes, which converts or raises as before
        c = (_Span * n)(*[_Span(q, 0, b, e) for (q, b, e) in spans])
        arr = np.frombuffer(bytearray(c), dtype=_SPAN_DTYPE).copy()
    return arr, n


_lib = None


def _share_torch_runtime():
    """PyTorch ships its own HIP runtime under the same soname.  Loading it
    first makes libsdf.so bind to that one runtime, so streams and device
    state are shared with torch instead of two runtimes competing for the
    device."""
    try:
        import torch  # noqa: F401
    except ImportError:
        return


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsdf.so is not built; run paper_1807_00205_amd/build.py "
                              "(or __graft_entry__.build())")
        _share_torch_runtime()
        L = ctypes.CDLL(LIB_PATH)
        vp, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        P = ctypes.POINTER
        st = ctypes.c_int32
        L.sdf_last_error.restype = ctypes.c_char_p
        L.sdf_index_build.restype = st
        L.sdf_index_build.argtypes = [vp, vp, u32, P(_IndexParams), vp, P(vp)]
        L.sdf_index_info.restype = st
        L.sdf_index_info.argtypes = [vp, P(u64), P(u64), P(u64)]
        L.sdf_index_hit_density.restype = st
        L.sdf_index_hit_density.argtypes = [vp, P(ctypes.c_double)]
        L.sdf_index_minimizers.restype = st
        L.sdf_index_minimizers.argtypes = [vp, vp, vp, vp, u64, P(u64)]
        L.sdf_index_entries.restype = st
        L.sdf_index_entries.argtypes = [vp, vp, vp, vp, u64, P(u64)]
        L.sdf_index_packed.restype = st
        L.sdf_index_packed.argtypes = [vp, vp, vp, vp]
        L.sdf_index_free.restype = None
        L.sdf_index_free.argtypes = [vp]
        L.sdf_search.restype = st
        L.sdf_search.argtypes = [vp, P(_Span), P(_SearchParams), vp, P(vp)]
        L.sdf_search_batch.restype = st
        L.sdf_search_batch.argtypes = [vp, vp, u32, P(_SearchParams), vp, P(vp)]
        L.sdf_result_count.restype = st
        L.sdf_result_count.argtypes = [vp, P(u64)]
        L.sdf_result_copy.restype = st
        L.sdf_result_copy.argtypes = [vp, vp, u64, P(u64)]
        L.sdf_result_seed_count.restype = st
        L.sdf_result_seed_count.argtypes = [vp, P(u64)]
        L.sdf_result_seeds.restype = st
        L.sdf_result_seeds.argtypes = [vp, vp, u64, P(u64)]
        L.sdf_result_timing.restype = st
        L.sdf_result_timing.argtypes = [vp, P(ctypes.c_float), u32]
        L.sdf_result_stats.restype = st
        L.sdf_result_stats.argtypes = [vp, P(u64), u32]
        L.sdf_result_free.restype = None
        L.sdf_result_free.argtypes = [vp]
        L.sdf_extend.restype = st
        L.sdf_extend.argtypes = [vp, vp, u64, P(_ExtendParams), vp, vp]
        L.sdf_autotune.restype = st
        L.sdf_index_save.restype = st
        L.sdf_index_save.argtypes = [vp, ctypes.c_char_p, vp]
        L.sdf_index_load.restype = st
        L.sdf_index_load.argtypes = [ctypes.c_char_p, vp, P(vp)]
        L.sdf_index_shape.restype = st
        L.sdf_index_shape.argtypes = [vp, P(u32), P(u32), P(u32), vp, u32]
        L.sdf_tuning_defaults.restype = None
        L.sdf_tuning_defaults.argtypes = [P(_Tuning)]
        L.sdf_set_tuning.restype = st
        L.sdf_set_tuning.argtypes = [P(_Tuning)]
        L.sdf_get_tuning.restype = st
        L.sdf_get_tuning.argtypes = [P(_Tuning)]
        L.sdf_autotune.argtypes = [vp, vp, u32, P(_SearchParams), vp, P(_Tuning),
                                   P(ctypes.c_float), u32]
        L.sdf_qgram_filter.restype = st
        L.sdf_qgram_filter.argtypes = [vp, vp, u64, P(_QgramParams), vp, vp, vp]
        L.sdf_result_regions.restype = st
        L.sdf_result_regions.argtypes = [vp, vp, u64, P(u64)]
        L.sdf_align_regions.restype = st
        L.sdf_align_regions.argtypes = [vp, vp, u64, P(_AlignParams), vp, P(vp)]
        L.sdf_sds_count.restype = st
        L.sdf_sds_count.argtypes = [vp, P(u64), P(u64)]
        L.sdf_sds_copy.restype = st
        L.sdf_sds_copy.argtypes = [vp, vp, u64, vp, u64]
        L.sdf_sds_free.restype = None
        L.sdf_sds_free.argtypes = [vp]
        L.sdf_search_batch_capped.restype = st
        L.sdf_search_batch_capped.argtypes = [vp, vp, u32, P(_SearchParams), u64, vp, P(vp),
                                              P(u64)]
        L.sdf_plan_create.restype = st
        L.sdf_plan_create.argtypes = [vp, vp, u32, P(_SearchParams), P(_PlanParams), vp, P(vp)]
        L.sdf_plan_run.restype = st
        L.sdf_plan_run.argtypes = [vp, vp, P(vp)]
        L.sdf_plan_info.restype = st
        L.sdf_plan_info.argtypes = [vp, P(u64), P(u64), P(u64), P(u64)]
        L.sdf_plan_free.restype = None
        L.sdf_plan_free.argtypes = [vp]
        L.sdf_search_batch_noalloc.restype = st
        L.sdf_search_batch_noalloc.argtypes = [vp, vp, u32, P(_SearchParams), vp, vp, u64,
                                               P(u64)]
        assert REGION_DTYPE.itemsize == 56
        assert SD_DTYPE.itemsize == 120
        _lib = L
    return _lib


def _check(rc: int):
    if rc != SDF_OK:
        raise SdfError(rc, lib().sdf_last_error().decode())


def get_tuning() -> dict:
    """The calling thread's schedule and test settings (``sdf_get_tuning``);
    AUTO marks the library's choice."""
    t = _Tuning()
    _check(lib().sdf_get_tuning(ctypes.byref(t)))
    return {f: int(getattr(t, f)) for f in TUNING_FIELDS}


def set_tuning(**settings) -> None:
    """Installs settings for the calling thread (``sdf_set_tuning``); fields
    not given (or given as None) keep the library's choice."""
    t = _Tuning()
    lib().sdf_tuning_defaults(ctypes.byref(t))
    for k, v in settings.items():
        if k not in TUNING_FIELDS:
            raise TypeError("unknown setting %r" % k)
        setattr(t, k, AUTO if v is None else int(v))
    _check(lib().sdf_set_tuning(ctypes.byref(t)))


@contextlib.contextmanager
def tuning(**settings):
    """The calling thread's settings with these changed, for the duration of
    the block; the previous ones are put back after it."""
    prev = get_tuning()
    cur = dict(prev)
    cur.update(settings)
    set_tuning(**cur)
    try:
        yield
    finally:
        set_tuning(**prev)


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


class Result:
    """Candidates (and seeds) of one search; owns the library result."""

    def __init__(self, handle):
        self._h = handle

    def close(self):
        if self._h:
            lib().sdf_result_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def candidates(self) -> np.ndarray:
        n = ctypes.c_uint64()
        _check(lib().sdf_result_count(self._h, ctypes.byref(n)))
        out = np.empty(n.value, CANDIDATE_DTYPE)
        w = ctypes.c_uint64()
        _check(lib().sdf_result_copy(self._h, out.ctypes.data_as(ctypes.c_void_p), n.value,
                                     ctypes.byref(w)))
        return out

    def seeds(self) -> np.ndarray:
        n = ctypes.c_uint64()
        _check(lib().sdf_result_seed_count(self._h, ctypes.byref(n)))
        out = np.empty(n.value, SEED_DTYPE)
        w = ctypes.c_uint64()
        _check(lib().sdf_result_seeds(self._h, out.ctypes.data_as(ctypes.c_void_p), n.value,
                                      ctypes.byref(w)))
        return out

    def regions(self) -> np.ndarray:
        """Extended region of every candidate (search run with extend=True)."""
        n = ctypes.c_uint64()
        _check(lib().sdf_result_count(self._h, ctypes.byref(n)))
        out = np.empty(n.value, REGION_DTYPE)
        w = ctypes.c_uint64()
        _check(lib().sdf_result_regions(self._h, out.ctypes.data_as(ctypes.c_void_p), n.value,
                                        ctypes.byref(w)))
        return out

    def timing(self) -> np.ndarray:
        """[setup, tile kernel, chaining, output sort, whole search, extension] ms."""
        ms = (ctypes.c_float * 6)()
        _check(lib().sdf_result_timing(self._h, ms, 6))
        return np.array(ms[:], dtype=np.float64)

    def _stats(self):
        v = (ctypes.c_uint64 * 16)()
        _check(lib().sdf_result_stats(self._h, v, 16))
        return [int(x) for x in v]

    def stats(self, extension: bool = False) -> dict:
        v = self._stats()
        keys = ["windows", "hits", "kept", "tiles", "partitions", "seeds", "candidate_evals",
                "scan_words"]
        if extension:
            keys += ["ext_insertions", "ext_continued", "ext_ranks", "ext_rank_us",
                     "ext_phase_us", "ext_slowest_region_us"]
        return dict(zip(keys, v))

    def schedule(self) -> Tuple[int, int]:
        """(window starts per tile, tile workgroup threads) the search ran."""
        v = self._stats()
        return v[14], v[15]


class Plan:
    """A batched search of fixed spans captured as a HIP graph
    (``sdf_plan_create``); ``run()`` replays it (``sdf_plan_run``)."""

    def __init__(self, index, spans, max_error=0.25, min_len=1000, seed_cap=0, cand_cap=0,
                 stream=None):
        arr, nspans = _span_array(spans)
        p = _SearchParams(max_error, min_len, 0)
        pp = _PlanParams(seed_cap, cand_cap)
        h = ctypes.c_void_p()
        _check(lib().sdf_plan_create(index._h, arr.ctypes.data_as(ctypes.c_void_p), nspans,
                                     ctypes.byref(p), ctypes.byref(pp), _stream_ptr(stream),
                                     ctypes.byref(h)))
        self._h = h.value
        self._index = index  # the index must outlive the plan

    def run(self, stream=None) -> Result:
        h = ctypes.c_void_p()
        _check(lib().sdf_plan_run(self._h, _stream_ptr(stream), ctypes.byref(h)))
        return Result(h.value)

    def info(self) -> dict:
        v = [ctypes.c_uint64() for _ in range(4)]
        _check(lib().sdf_plan_info(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(["seed_cap", "cand_cap", "replays", "fallbacks"], [x.value for x in v]))

    def close(self):
        if getattr(self, "_h", None):
            lib().sdf_plan_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Index:
    """Device-resident index of a set of sequences (``sdf_index_build``)."""

    def __init__(self, seqs: Sequence, k: int = 12, w: int = 16, stream=None):
        bufs = [np.ascontiguousarray(np.frombuffer(s, dtype=np.uint8) if isinstance(s, bytes)
                                     else s, dtype=np.uint8) for s in seqs]
        self._keep = bufs
        n = len(bufs)
        ptrs = (ctypes.c_void_p * max(n, 1))(*[b.ctypes.data for b in bufs])
        lens = (ctypes.c_uint64 * max(n, 1))(*[len(b) for b in bufs])
        p = _IndexParams(k, w)
        h = ctypes.c_void_p()
        _check(lib().sdf_index_build(ctypes.cast(ptrs, ctypes.c_void_p),
                                     ctypes.cast(lens, ctypes.c_void_p), n, ctypes.byref(p),
                                     _stream_ptr(stream), ctypes.byref(h)))
        self._h = h.value
        self._keep = None
        self.k, self.w = k, w
        self.lengths = [len(b) for b in bufs]

    @classmethod
    def load(cls, path: str, stream=None) -> "Index":
        """An index read from a file written by ``save`` (``sdf_index_load``)."""
        h = ctypes.c_void_p()
        _check(lib().sdf_index_load(os.fsencode(path), _stream_ptr(stream), ctypes.byref(h)))
        self = cls.__new__(cls)
        self._h = h.value
        self._keep = None
        k, w, n = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().sdf_index_shape(self._h, ctypes.byref(k), ctypes.byref(w), ctypes.byref(n),
                                     None, 0))
        lens = np.zeros(max(1, n.value), np.uint64)
        _check(lib().sdf_index_shape(self._h, None, None, None,
                                     lens.ctypes.data_as(ctypes.c_void_p), n.value))
        self.k, self.w = k.value, w.value
        self.lengths = [int(x) for x in lens[:n.value]]
        return self

    def save(self, path: str, stream=None) -> None:
        """Writes the index to a file (``sdf_index_save``)."""
        _check(lib().sdf_index_save(self._h, os.fsencode(path), _stream_ptr(stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib().sdf_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> Tuple[int, int, int]:
        a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().sdf_index_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def hit_density(self) -> float:
        """Mean number of target occurrences of a query minimizer's hash."""
        v = ctypes.c_double()
        _check(lib().sdf_index_hit_density(self._h, ctypes.byref(v)))
        return v.value

    def minimizers(self):
        nm, _, _ = self.info()
        pos = np.empty(nm, np.uint32)
        h = np.empty(nm, np.uint32)
        fl = np.empty(nm, np.uint8)
        w = ctypes.c_uint64()
        _check(lib().sdf_index_minimizers(self._h, pos.ctypes.data_as(ctypes.c_void_p),
                                          h.ctypes.data_as(ctypes.c_void_p),
                                          fl.ctypes.data_as(ctypes.c_void_p), nm, ctypes.byref(w)))
        return pos, h, fl

    def entries(self):
        _, ne, _ = self.info()
        h = np.empty(ne, np.uint32)
        st = np.empty(ne, np.uint8)
        pos = np.empty(ne, np.uint32)
        w = ctypes.c_uint64()
        _check(lib().sdf_index_entries(self._h, h.ctypes.data_as(ctypes.c_void_p),
                                       st.ctypes.data_as(ctypes.c_void_p),
                                       pos.ctypes.data_as(ctypes.c_void_p), ne, ctypes.byref(w)))
        return h, st, pos

    def packed(self):
        total = sum(self.lengths)
        pk = np.empty((total + 15) // 16, np.uint32)
        mk = np.empty((total + 31) // 32, np.uint32)
        gp = np.empty((total + 31) // 32, np.uint32)
        _check(lib().sdf_index_packed(self._h, pk.ctypes.data_as(ctypes.c_void_p),
                                      mk.ctypes.data_as(ctypes.c_void_p),
                                      gp.ctypes.data_as(ctypes.c_void_p)))
        return pk, mk, gp

    def extend(self, regions, max_error: float = 0.25, max_len: int = 1000000,
               stream=None) -> np.ndarray:
        """Extends regions (a REGION_DTYPE array, or rows (strand, q_seq,
        q_begin, q_end, t_seq, t_begin, t_end)) by ``sdf_extend``."""
        if isinstance(regions, np.ndarray) and regions.dtype == REGION_DTYPE:
            inp = np.ascontiguousarray(regions)
        else:
            rows = list(regions)
            inp = np.zeros(len(rows), REGION_DTYPE)
            for u, (o, qs, qb, qe, ts, tb, te) in enumerate(rows):
                inp[u] = (o, qs, ts, 0, qb, qe, tb, te, 0, 0)
        out = np.empty(len(inp), REGION_DTYPE)
        p = _ExtendParams(max_error, max_len)
        _check(lib().sdf_extend(self._h, inp.ctypes.data_as(ctypes.c_void_p), len(inp),
                                ctypes.byref(p), _stream_ptr(stream),
                                out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def autotune(self, spans: Iterable[Tuple[int, int, int]], max_error: float = 0.25,
                 min_len: int = 1000, stream=None):
        """Times the tile kernel on these spans with every schedule
        (``sdf_autotune``); returns (window starts, workgroup threads,
        {(threads, window starts): ms}) of the fastest.  The index is not
        changed: searches use the schedule where the caller installs it
        (``set_tuning(tile_core=..., tile_threads=...)`` or ``tuning(...)``).
        No spans: the calling thread's settings, nothing timed."""
        arr, nspans = _span_array(spans)
        p = _SearchParams(max_error, min_len, 0)
        out = _Tuning()
        ms = (ctypes.c_float * 16)()
        _check(lib().sdf_autotune(self._h, arr.ctypes.data_as(ctypes.c_void_p), nspans,
                                  ctypes.byref(p), _stream_ptr(stream), ctypes.byref(out), ms,
                                  16))
        sched = [(1024, c) for c in range(512, 1025, 64)]
        if min_len <= 1023 + self.k:
            sched.append((512, 512))
        times = {k: float(ms[i]) for i, k in enumerate(sched)} if spans else {}
        return int(out.tile_core), int(out.tile_threads), times

    def qgram_filter(self, regions: np.ndarray, q: int, gap_rate: float,
                     max_error: float = 0.25, stream=None):
        """Section 3.2 q-gram filter of REGION_DTYPE regions: (shared q-mer
        counts Q, pass flags)."""
        inp = np.ascontiguousarray(regions)
        assert inp.dtype == REGION_DTYPE
        shared = np.empty(len(inp), np.uint64)
        ok = np.empty(len(inp), np.uint8)
        p = _QgramParams(max_error, gap_rate, q, 0)
        _check(lib().sdf_qgram_filter(self._h, inp.ctypes.data_as(ctypes.c_void_p), len(inp),
                                      ctypes.byref(p), _stream_ptr(stream),
                                      shared.ctypes.data_as(ctypes.c_void_p),
                                      ok.ctypes.data_as(ctypes.c_void_p)))
        return shared, ok.astype(bool)

    def search(self, span: Tuple[int, int, int], max_error: float = 0.25, min_len: int = 1000,
               timing: bool = False, stream=None, estimate: bool = False,
               extend: bool = False) -> Result:
        sp = _Span(span[0], 0, span[1], span[2])
        p = _SearchParams(max_error, min_len, _flags(timing, estimate, extend))
        h = ctypes.c_void_p()
        _check(lib().sdf_search(self._h, ctypes.byref(sp), ctypes.byref(p), _stream_ptr(stream),
                                ctypes.byref(h)))
        return Result(h.value)

    def search_batch(self, spans: Iterable[Tuple[int, int, int]], max_error: float = 0.25,
                     min_len: int = 1000, timing: bool = False, stream=None,
                     estimate: bool = False, extend: bool = False) -> Result:
        arr, nspans = _span_array(spans)
        p = _SearchParams(max_error, min_len, _flags(timing, estimate, extend))
        h = ctypes.c_void_p()
        _check(lib().sdf_search_batch(self._h, arr.ctypes.data_as(ctypes.c_void_p), nspans,
                                      ctypes.byref(p), _stream_ptr(stream), ctypes.byref(h)))
        return Result(h.value)

    def search_batch_noalloc(self, spans: Iterable[Tuple[int, int, int]],
                             max_error: float = 0.25, min_len: int = 1000, cap: int = None,
                             stream=None) -> np.ndarray:
        """The batched search through ``sdf_search_batch_noalloc`` (no memory
        allocated by the library; device buffers come from its fixed scratch
        area).  Returns the candidates in the order of ``Result.candidates``;
        with ``cap``, at most that many are copied (the array is sized by the
        count the library reports)."""
        arr, nspans = _span_array(spans)
        p = _SearchParams(max_error, min_len, 0)
        n = ctypes.c_uint64()
        if cap is None:
            cap = 65536
        out = np.empty(max(1, cap), CANDIDATE_DTYPE)
        _check(lib().sdf_search_batch_noalloc(self._h, arr.ctypes.data_as(ctypes.c_void_p),
                                              nspans, ctypes.byref(p), _stream_ptr(stream),
                                              out.ctypes.data_as(ctypes.c_void_p), cap,
                                              ctypes.byref(n)))
        return out[:min(cap, n.value)].copy(), n.value

    def search_batch_capped(self, spans: Iterable[Tuple[int, int, int]], max_bytes: int,
                            max_error: float = 0.25, min_len: int = 1000, stream=None):
        """``sdf_search_batch`` within a device-memory reservation of
        ``max_bytes``: returns (Result, peak bytes held); raises SdfError with
        SDF_ENOMEM when the search would need more."""
        arr, nspans = _span_array(spans)
        p = _SearchParams(max_error, min_len, 0)
        h = ctypes.c_void_p()
        peak = ctypes.c_uint64()
        _check(lib().sdf_search_batch_capped(self._h, arr.ctypes.data_as(ctypes.c_void_p), nspans,
                                             ctypes.byref(p), max_bytes, _stream_ptr(stream),
                                             ctypes.byref(h), ctypes.byref(peak)))
        return Result(h.value), peak.value

    def plan(self, spans: Iterable[Tuple[int, int, int]], max_error: float = 0.25,
             min_len: int = 1000, seed_cap: int = 0, cand_cap: int = 0, stream=None) -> Plan:
        """The batched search of these spans captured as a HIP graph."""
        return Plan(self, spans, max_error, min_len, seed_cap, cand_cap, stream)

    def align_regions(self, regions, k: int = 11, min_len: int = 1000, max_error: float = 0.25,
                      pad_frac: float = PAD_FRAC, stream=None):
        """Final SDs (Section 3.3) of region pairs (a REGION_DTYPE array, as
        from an extension), each side padded first by pad_frac of its length
        at both ends (Section 3.2): (SD_DTYPE records, CIGAR operations)."""
        inp = np.ascontiguousarray(regions)
        assert inp.dtype == REGION_DTYPE
        p = _AlignParams(max_error, min_len, k, pad_frac)
        h = ctypes.c_void_p()
        _check(lib().sdf_align_regions(self._h, inp.ctypes.data_as(ctypes.c_void_p), len(inp),
                                       ctypes.byref(p), _stream_ptr(stream), ctypes.byref(h)))
        try:
            nsd, nops = ctypes.c_uint64(), ctypes.c_uint64()
            _check(lib().sdf_sds_count(h, ctypes.byref(nsd), ctypes.byref(nops)))
            sd = np.zeros(nsd.value, SD_DTYPE)
            ops = np.zeros(nops.value, np.uint32)
            _check(lib().sdf_sds_copy(h, sd.ctypes.data_as(ctypes.c_void_p), nsd.value,
                                      ops.ctypes.data_as(ctypes.c_void_p), nops.value))
        finally:
            lib().sdf_sds_free(h)
        return sd, ops


def cigar_string(ops: np.ndarray) -> str:
    """CIGAR text of operations (len << 4 | op)."""
    return "".join("%d%s" % (int(v) >> 4, CIGAR_CHARS[int(v) & 15]) for v in ops)


def to_bedpe(sd: np.ndarray, ops: np.ndarray, names: Sequence[str]) -> List[str]:
    """BEDPE lines (chrom1, start1, end1, chrom2, start2, end2, name, score,
    strand1, strand2, then alignment length, identity, K2P, JC and CIGAR) of
    final SD records."""
    lines = []
    for s in sd:
        o = int(s["cigar_off"])
        cig = cigar_string(ops[o:o + int(s["cigar_len"])])
        ident = int(s["matches"]) / max(1, int(s["aln_len"]))
        lines.append("\t".join([names[int(s["q_seq"])], str(int(s["q_begin"])), str(int(s["q_end"])),
                                names[int(s["t_seq"])], str(int(s["t_begin"])), str(int(s["t_end"])),
                                "sd%d" % int(s["region"]), str(int(s["aln_len"])), "+",
                                "-" if int(s["strand"]) else "+", str(int(s["aln_len"])),
                                "%.4f" % ident, "%.6f" % float(s["k2p"]), "%.6f" % float(s["jc"]),
                                cig]))
    return lines
