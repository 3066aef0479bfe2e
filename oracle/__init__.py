"""CPU oracle for the winnowed-minimizer Jaccard seed filter and seed chaining.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
(``paper_1807_00205_amd``) never imports it, and the two share no code.

``sdf_oracle.c`` holds the plain C definition (see its header); this module
builds it with gcc and wraps it with ctypes.  ``brute.py`` holds an
independent pure-Python restatement used on tiny inputs to pin the C code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sdf_oracle.c")
_SRC2 = os.path.join(_HERE, "sd_align.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SEED_DTYPE = np.dtype([("query_id", "<u4"), ("i", "<u4"), ("j", "<u4"),
                       ("strand", "<u4"), ("shared", "<u4"), ("sketch", "<u4")])
# Extended region (Section 3.2): global coordinates, numerator and sketch size
# of the final state, stop codes (forward | backward << 8).
EXT_DTYPE = np.dtype([("q_begin", "<u8"), ("q_end", "<u8"), ("t_begin", "<u8"),
                      ("t_end", "<u8"), ("m", "<u8"), ("s", "<u8"), ("stop", "<u8")])
EXT_BOUND, EXT_CAP, EXT_OVERLAP, EXT_ESTIMATE = 1, 2, 3, 4
# A final SD (Section 3.3): region index, strand, sequences and per-sequence
# coordinates (BEDPE), alignment counts, distances, and its CIGAR operations
# (len << 4 | op; op 7 '=', 8 'X', 1 'I', 2 'D') at [cigar_off, +cigar_len).
SD_DTYPE = np.dtype([("region", "<u8"), ("strand", "<u4"), ("q_seq", "<u4"), ("t_seq", "<u4"),
                     ("_pad", "<u4"), ("q_begin", "<u8"), ("q_end", "<u8"), ("t_begin", "<u8"),
                     ("t_end", "<u8"), ("aln_len", "<u4"), ("matches", "<u4"),
                     ("mismatches", "<u4"), ("ins", "<u4"), ("dels", "<u4"), ("gap_opens", "<u4"),
                     ("transitions", "<u4"), ("transversions", "<u4"), ("k2p", "<f8"),
                     ("jc", "<f8"), ("cigar_off", "<u8"), ("cigar_len", "<u8")])
CAND_DTYPE = np.dtype([("query_id", "<u4"), ("strand", "<u4"), ("q_seq", "<u4"),
                       ("t_seq", "<u4"), ("q_begin", "<u8"), ("q_end", "<u8"),
                       ("t_begin", "<u8"), ("t_end", "<u8"), ("n_seeds", "<u4"),
                       ("max_shared", "<u4")])


def _stale() -> bool:
    if not os.path.exists(_LIB):
        return True
    t = os.path.getmtime(_LIB)
    return t < os.path.getmtime(_SRC) or t < os.path.getmtime(_SRC2)


def build(force: bool = True) -> str:
    """Compile the oracle (gcc, OpenMP) into ``oracle/liboracle.so``."""
    if force or _stale():
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, _SRC, _SRC2, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _stale():
            build()
        L = ctypes.CDLL(_LIB)
        vp, u32, u64, dbl = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        P = ctypes.POINTER
        L.or_hash.restype = u32
        L.or_hash.argtypes = [u32, u32]
        L.or_encode.argtypes = [vp, u64, vp, vp]
        L.or_hash_many.argtypes = [vp, u64, u32, vp]
        L.or_kmer_table.argtypes = [vp, vp, u32, u32, vp, vp, vp, vp]
        L.or_index_build.restype = vp
        L.or_index_build.argtypes = [vp, vp, u32, u32, u32]
        L.or_index_free.argtypes = [vp]
        L.or_index_n_minimizers.restype = u64
        L.or_index_n_minimizers.argtypes = [vp]
        L.or_index_n_eligible.restype = u64
        L.or_index_n_eligible.argtypes = [vp]
        L.or_index_minimizers.argtypes = [vp, vp, vp, vp]
        L.or_index_entries.argtypes = [vp, vp, vp, vp]
        L.or_params.restype = ctypes.c_int
        L.or_params.argtypes = [dbl, u32, u32, P(dbl), P(u32), P(u32)]
        L.or_threshold.restype = u32
        L.or_threshold.argtypes = [dbl, u32]
        L.or_sketch_size.restype = u32
        L.or_sketch_size.argtypes = [vp, u64, u32]
        L.or_count.restype = u32
        L.or_count.argtypes = [vp, u64, u64, u32, u32]
        L.or_estimate.restype = u32
        L.or_estimate.argtypes = [vp, u64, u64, u32, u32]
        L.or_search.restype = vp
        L.or_search.argtypes = [vp, vp, u32, dbl, u32, ctypes.c_int, ctypes.c_int, P(ctypes.c_int)]
        L.or_result_nseeds.restype = u64
        L.or_result_nseeds.argtypes = [vp]
        L.or_result_ncands.restype = u64
        L.or_result_ncands.argtypes = [vp]
        L.or_result_seeds.argtypes = [vp, vp]
        L.or_result_cands.argtypes = [vp, vp]
        L.or_result_free.argtypes = [vp]
        L.or_extend.restype = ctypes.c_int
        L.or_extend.argtypes = [vp, vp, u32, dbl, u64, vp]
        L.or_extend_many.restype = u64
        L.or_extend_many.argtypes = [vp, vp, u64, dbl, u64, ctypes.c_int, vp]
        L.or_qgram_shared.restype = u64
        L.or_qgram_shared.argtypes = [vp, vp, u32, u32]
        L.or_qgram_bound.restype = dbl
        L.or_qgram_bound.argtypes = [u64, dbl, u32, dbl]
        L.or_seed_size.restype = ctypes.c_int
        L.or_cand_size.restype = ctypes.c_int
        L.or_sd_align.restype = vp
        L.or_sd_align.argtypes = [vp, vp, u32, vp, u64, u32, u32, dbl, dbl, ctypes.c_int]
        L.or_sd_count.restype = u64
        L.or_sd_count.argtypes = [vp]
        L.or_sd_ops_count.restype = u64
        L.or_sd_ops_count.argtypes = [vp]
        L.or_sd_size.restype = ctypes.c_int
        L.or_sd_copy.argtypes = [vp, vp, vp]
        L.or_sd_free.argtypes = [vp]
        L.or_align_pair.restype = u64
        L.or_align_pair.argtypes = [vp, u32, vp, u32, vp, u64]
        assert L.or_seed_size() == SEED_DTYPE.itemsize
        assert L.or_cand_size() == CAND_DTYPE.itemsize
        assert L.or_sd_size() == SD_DTYPE.itemsize
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def kmer_hash(x: int, k: int) -> int:
    return int(lib().or_hash(x, k))


def hash_many(x: np.ndarray, k: int) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.uint32)
    out = np.empty_like(x)
    lib().or_hash_many(_ptr(x), len(x), k, _ptr(out))
    return out


def encode(seq: np.ndarray):
    seq = np.ascontiguousarray(seq, dtype=np.uint8)
    code = np.empty(len(seq), np.uint8)
    lower = np.empty(len(seq), np.uint8)
    lib().or_encode(_ptr(seq), len(seq), _ptr(code), _ptr(lower))
    return code, lower


def kmer_table(bytes_: np.ndarray, off: np.ndarray, k: int):
    b = np.ascontiguousarray(bytes_, dtype=np.uint8)
    off = np.ascontiguousarray(off, dtype=np.uint64)
    n = len(b)
    f = np.empty(n, np.uint32)
    r = np.empty(n, np.uint32)
    h = np.empty(n, np.uint32)
    fl = np.empty(n, np.uint8)
    lib().or_kmer_table(_ptr(b), _ptr(off), len(off) - 1, k, _ptr(f), _ptr(r), _ptr(h), _ptr(fl))
    return f, r, h, fl


def params(max_error: float, min_len: int, k: int):
    tau = ctypes.c_double()
    n = ctypes.c_uint32()
    mo = ctypes.c_uint32()
    rc = lib().or_params(max_error, min_len, k, ctypes.byref(tau), ctypes.byref(n),
                         ctypes.byref(mo))
    if rc != 0:
        raise ValueError("invalid parameters")
    return tau.value, n.value, mo.value


def qgram_bound(n: int, max_error: float, q: int, gap_rate: float) -> float:
    """The Section 3.2 q-gram bound for a shorter side of n bases."""
    return float(lib().or_qgram_bound(n, max_error, q, gap_rate))


def threshold(tau: float, s: int) -> int:
    return int(lib().or_threshold(tau, s))


class OracleIndex:
    def __init__(self, bytes_: np.ndarray, off: np.ndarray, k: int = 12, w: int = 16):
        self._b = np.ascontiguousarray(bytes_, dtype=np.uint8)
        self._off = np.ascontiguousarray(off, dtype=np.uint64)
        self.k, self.w = k, w
        self._h = lib().or_index_build(_ptr(self._b), _ptr(self._off), len(self._off) - 1, k, w)
        if not self._h:
            raise ValueError("invalid index parameters")

    def close(self):
        if self._h:
            lib().or_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_minimizers(self) -> int:
        return int(lib().or_index_n_minimizers(self._h))

    @property
    def n_eligible(self) -> int:
        return int(lib().or_index_n_eligible(self._h))

    def minimizers(self):
        n = self.n_minimizers
        pos = np.empty(n, np.uint32)
        h = np.empty(n, np.uint32)
        fl = np.empty(n, np.uint8)
        lib().or_index_minimizers(self._h, _ptr(pos), _ptr(h), _ptr(fl))
        return pos, h, fl

    def entries(self):
        n = self.n_eligible
        h = np.empty(n, np.uint32)
        st = np.empty(n, np.uint8)
        pos = np.empty(n, np.uint32)
        lib().or_index_entries(self._h, _ptr(h), _ptr(st), _ptr(pos))
        return h, st, pos

    def sketch_size(self, i: int, n: int) -> int:
        return int(lib().or_sketch_size(self._h, i, n))

    def count(self, i: int, j: int, o: int, n: int) -> int:
        return int(lib().or_count(self._h, i, j, o, n))

    def estimate(self, i: int, j: int, o: int, n: int) -> int:
        """Numerator m of the winnowed MinHash estimate m / s_i."""
        return int(lib().or_estimate(self._h, i, j, o, n))

    def extend(self, regions, tau: float, max_len: int = 1000000, threads: int = 0):
        """Extends regions (rows q0, q1, t0, t1, o in global coordinates) by
        the Section 3.2 procedure; returns an EXT_DTYPE array."""
        r = np.ascontiguousarray(np.array(regions, dtype=np.uint64).reshape(-1, 5))
        out = np.zeros(len(r), EXT_DTYPE)
        bad = lib().or_extend_many(self._h, _ptr(r), len(r), tau, max_len, threads, _ptr(out))
        if bad:
            raise ValueError("%d invalid regions" % bad)
        return out

    def qgram_shared(self, region, q: int) -> int:
        """Q of Section 3.2 for one region (q0, q1, t0, t1, o), global coordinates."""
        r = np.ascontiguousarray(np.array(region[:4], dtype=np.uint64))
        return int(lib().or_qgram_shared(self._h, _ptr(r), int(region[4]), q))

    def search(self, spans, max_error: float = 0.25, min_len: int = 1000, threads: int = 0,
               estimate: bool = False):
        sp = np.ascontiguousarray(np.array(spans, dtype=np.uint64).reshape(-1, 3))
        st = ctypes.c_int()
        r = lib().or_search(self._h, _ptr(sp), len(sp), max_error, min_len, int(estimate),
                            threads, ctypes.byref(st))
        if st.value != 0:
            raise ValueError("oracle search failed: status %d" % st.value)
        try:
            ns = int(lib().or_result_nseeds(r))
            nc = int(lib().or_result_ncands(r))
            seeds = np.empty(ns, SEED_DTYPE)
            cands = np.empty(nc, CAND_DTYPE)
            lib().or_result_seeds(r, _ptr(seeds))
            lib().or_result_cands(r, _ptr(cands))
        finally:
            lib().or_result_free(r)
        return seeds, cands


def sd_align(bytes_: np.ndarray, off: np.ndarray, rows, k: int = 11, min_len: int = 1000,
             max_error: float = 0.25, threads: int = 0, pad_frac: float = 0.0):
    """Final SDs (Section 3.3) of region pairs given as rows (q0, q1, t0, t1,
    strand) of global coordinates, each side padded first by pad_frac of its
    length at both ends (Section 3.2): (SD_DTYPE array, CIGAR operations)."""
    b = np.ascontiguousarray(bytes_, dtype=np.uint8)
    off = np.ascontiguousarray(off, dtype=np.uint64)
    r = np.ascontiguousarray(np.array(rows, dtype=np.uint64).reshape(-1, 5))
    h = lib().or_sd_align(_ptr(b), _ptr(off), len(off) - 1, _ptr(r), len(r), k, min_len,
                          max_error, pad_frac, threads)
    if not h:
        raise ValueError("invalid region rows or parameters")
    try:
        sd = np.zeros(int(lib().or_sd_count(h)), SD_DTYPE)
        ops = np.zeros(int(lib().or_sd_ops_count(h)), np.uint32)
        lib().or_sd_copy(h, _ptr(sd), _ptr(ops))
    finally:
        lib().or_sd_free(h)
    return sd, ops


def align_pair(q: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Global alignment (the Section 3.3 reading: match 2, mismatch -4, gap
    4 + 2 L) of two code strings (0..3, 4 = N): CIGAR operations."""
    q = np.ascontiguousarray(q, dtype=np.uint8)
    t = np.ascontiguousarray(t, dtype=np.uint8)
    cap = len(q) + len(t) + 1
    ops = np.zeros(cap, np.uint32)
    n = int(lib().or_align_pair(_ptr(q), len(q), _ptr(t), len(t), _ptr(ops), cap))
    return ops[:n]
