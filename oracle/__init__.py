"""CPU oracle for exact planted (l,d)-motif search (ctypes binding).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the product path
never does. It shares no code with the GPU library (``pms_oracle.c`` states
what it computes and which passages of the thesis each part follows).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pms_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OR_OK, OR_EINVAL, OR_EBASE, OR_ENOMEM = 0, -1, -2, -3


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (x86-64-v3: runs on any recent host)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-fPIC",
                               "-shared", "-std=c11", "-pthread", "-o", tmp,
                               _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.oracle_o1.restype = ctypes.c_int
        lib.oracle_o1.argtypes = [
            ctypes.c_char_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.POINTER(u64p), ctypes.POINTER(ctypes.c_size_t), u64p, u64p]
        lib.oracle_o0.restype = ctypes.c_int
        lib.oracle_o0.argtypes = [
            ctypes.c_char_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_int, ctypes.c_int, ctypes.POINTER(u64p),
            ctypes.POINTER(ctypes.c_size_t)]
        for fn in (lib.oracle_q1, lib.oracle_q0):
            fn.restype = ctypes.c_int
            fn.argtypes = [
                ctypes.c_char_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                ctypes.c_int, ctypes.c_int, ctypes.c_int,
                ctypes.POINTER(u64p), ctypes.POINTER(ctypes.c_size_t)]
        lib.oracle_p1.restype = ctypes.c_int
        lib.oracle_p1.argtypes = [
            ctypes.c_char_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_int, ctypes.c_int, ctypes.POINTER(u64p),
            ctypes.POINTER(ctypes.c_size_t), u64p]
        lib.oracle_s1.restype = ctypes.c_int
        lib.oracle_s1.argtypes = [
            ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int, ctypes.c_int,
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.POINTER(u64p), ctypes.POINTER(ctypes.c_size_t)]
        lib.oracle_s0.restype = ctypes.c_int
        lib.oracle_s0.argtypes = [
            ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int, ctypes.c_int,
            ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.POINTER(u64p), ctypes.POINTER(ctypes.c_size_t)]
        lib.oracle_hit_count.restype = ctypes.c_int
        lib.oracle_hit_count.argtypes = [
            ctypes.c_char_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_int, ctypes.c_uint64]
        lib.oracle_is_motif.restype = ctypes.c_int
        lib.oracle_is_motif.argtypes = [
            ctypes.c_char_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_int, ctypes.c_uint64]
        lib.oracle_nb.restype = ctypes.c_uint64
        lib.oracle_nb.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.oracle_groups.restype = ctypes.c_int
        lib.oracle_groups.argtypes = [ctypes.c_char_p, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_uint32),
                                      ctypes.POINTER(ctypes.c_uint32)]
        lib.oracle_hamming_groups.restype = ctypes.c_int
        lib.oracle_hamming_groups.argtypes = [ctypes.c_uint32] * 4
        lib.oracle_hamming_naive.restype = ctypes.c_int
        lib.oracle_hamming_naive.argtypes = [ctypes.c_char_p, ctypes.c_char_p,
                                             ctypes.c_int]
        lib.oracle_lmer_code.restype = ctypes.c_uint64
        lib.oracle_lmer_code.argtypes = [ctypes.c_char_p, ctypes.c_int]
        lib.oracle_encode.restype = ctypes.c_int
        lib.oracle_encode.argtypes = [ctypes.c_char_p, ctypes.c_longlong,
                                      ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_longlong)]
        lib.oracle_o1_wide.restype = ctypes.c_int
        lib.oracle_o1_wide.argtypes = [
            ctypes.c_char_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_int, ctypes.c_int, ctypes.POINTER(u64p),
            ctypes.POINTER(ctypes.c_size_t), u64p]
        lib.oracle_is_motif_wide.restype = ctypes.c_int
        lib.oracle_is_motif_wide.argtypes = [
            ctypes.c_char_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
        lib.oracle_free.argtypes = [ctypes.c_void_p]
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, rc, what):
        super().__init__("%s failed with status %d" % (what, rc))
        self.rc = rc


def _seq_bytes(seqs) -> bytes:
    if isinstance(seqs, (bytes, bytearray)):
        return bytes(seqs)
    if isinstance(seqs, np.ndarray):
        return seqs.astype(np.uint8).tobytes()
    return b"".join(seqs)


def _take(ptr, count) -> np.ndarray:
    lib = _load()
    if count:
        arr = np.ctypeslib.as_array(ptr, shape=(count,)).copy()
    else:
        arr = np.zeros(0, dtype=np.uint64)
    lib.oracle_free(ptr)
    return arr.astype(np.uint64)


def o1(seqs, n, m, l, d, ref_begin=0, ref_end=-1, threads=0,
       per_ref=False):
    """Sample-driven oracle. Returns (motifs, H_canon[, per-reference H])."""
    lib = _load()
    buf = _seq_bytes(seqs)
    assert len(buf) == n * m
    out = ctypes.POINTER(ctypes.c_uint64)()
    count = ctypes.c_size_t(0)
    h = ctypes.c_uint64(0)
    L = m - l + 1
    span = (L if ref_end < 0 else min(ref_end, L)) - ref_begin
    pr = np.zeros(max(span, 1), dtype=np.uint64) if per_ref else None
    prp = (pr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
           if per_ref else None)
    rc = lib.oracle_o1(buf, n, m, l, d, ref_begin, ref_end, threads,
                       ctypes.byref(out), ctypes.byref(count),
                       ctypes.byref(h), prp)
    if rc != OR_OK:
        raise OracleError(rc, "oracle_o1")
    motifs = _take(out, count.value)
    if per_ref:
        return motifs, int(h.value), pr[:span]
    return motifs, int(h.value)


def o0(seqs, n, m, l, d, threads=0) -> np.ndarray:
    """Pattern-driven brute force over all 4^l codes."""
    lib = _load()
    buf = _seq_bytes(seqs)
    assert len(buf) == n * m
    out = ctypes.POINTER(ctypes.c_uint64)()
    count = ctypes.c_size_t(0)
    rc = lib.oracle_o0(buf, n, m, l, d, threads, ctypes.byref(out),
                       ctypes.byref(count))
    if rc != OR_OK:
        raise OracleError(rc, "oracle_o0")
    return _take(out, count.value)


def _quorum(fn, name, seqs, n, m, l, d, q, threads):
    buf = _seq_bytes(seqs)
    assert len(buf) == n * m
    out = ctypes.POINTER(ctypes.c_uint64)()
    count = ctypes.c_size_t(0)
    rc = fn(buf, n, m, l, d, q, threads, ctypes.byref(out),
            ctypes.byref(count))
    if rc != OR_OK:
        raise OracleError(rc, name)
    return _take(out, count.value)


def q1(seqs, n, m, l, d, q, threads=0) -> np.ndarray:
    """(l,d,q)-motifs from the spheres of the l-mers of s_1..s_{n-q+1}
    (Observation 3.1)."""
    return _quorum(_load().oracle_q1, "oracle_q1", seqs, n, m, l, d, q,
                   threads)


def q0(seqs, n, m, l, d, q, threads=0) -> np.ndarray:
    """(l,d,q)-motifs by brute force over all 4^l codes."""
    return _quorum(_load().oracle_q0, "oracle_q0", seqs, n, m, l, d, q,
                   threads)


def p1(seqs, n, m, l, d, threads=0):
    """Pair-based (Observation 3.3): (motifs, number of candidates)."""
    buf = _seq_bytes(seqs)
    assert len(buf) == n * m
    out = ctypes.POINTER(ctypes.c_uint64)()
    count = ctypes.c_size_t(0)
    nc = ctypes.c_uint64(0)
    rc = _load().oracle_p1(buf, n, m, l, d, threads, ctypes.byref(out),
                           ctypes.byref(count), ctypes.byref(nc))
    if rc != OR_OK:
        raise OracleError(rc, "oracle_p1")
    return _take(out, count.value), int(nc.value)


def s1(seqs, alphabet: bytes, n, m, l, d, threads=0) -> np.ndarray:
    """(l,d)-motifs over the given alphabet, sample-driven; codes in base
    len(alphabet), first letter in the top digit."""
    buf = _seq_bytes(seqs)
    assert len(buf) == n * m
    out = ctypes.POINTER(ctypes.c_uint64)()
    count = ctypes.c_size_t(0)
    rc = _load().oracle_s1(buf, bytes(alphabet), len(alphabet), n, m, l, d,
                           threads, ctypes.byref(out), ctypes.byref(count))
    if rc != OR_OK:
        raise OracleError(rc, "oracle_s1")
    return _take(out, count.value)


def s0(seqs, alphabet: bytes, n, m, l, d) -> np.ndarray:
    """(l,d)-motifs over the given alphabet by brute force (small spaces)."""
    buf = _seq_bytes(seqs)
    assert len(buf) == n * m
    out = ctypes.POINTER(ctypes.c_uint64)()
    count = ctypes.c_size_t(0)
    rc = _load().oracle_s0(buf, bytes(alphabet), len(alphabet), n, m, l, d,
                           ctypes.byref(out), ctypes.byref(count))
    if rc != OR_OK:
        raise OracleError(rc, "oracle_s0")
    return _take(out, count.value)


def hit_count(seqs, n, m, l, d, code) -> int:
    """Number of strings with an l-mer within distance d of the code."""
    rc = _load().oracle_hit_count(_seq_bytes(seqs), n, m, l, d, int(code))
    if rc < 0:
        raise OracleError(rc, "oracle_hit_count")
    return rc


def is_motif(seqs, n, m, l, d, code) -> bool:
    rc = _load().oracle_is_motif(_seq_bytes(seqs), n, m, l, d, int(code))
    if rc < 0:
        raise OracleError(rc, "oracle_is_motif")
    return rc == 1


def o1_wide(seqs, n, m, l, d, threads=0):
    """W1, the sample-driven oracle for 1 <= l <= 64: (codes, H_canon), the
    codes as Python ints (up to 128 bits), ascending."""
    lib = _load()
    buf = _seq_bytes(seqs)
    assert len(buf) == n * m
    out = ctypes.POINTER(ctypes.c_uint64)()
    count = ctypes.c_size_t(0)
    h = ctypes.c_uint64(0)
    rc = lib.oracle_o1_wide(buf, n, m, l, d, threads, ctypes.byref(out),
                            ctypes.byref(count), ctypes.byref(h))
    if rc != OR_OK:
        raise OracleError(rc, "oracle_o1_wide")
    words = _take(out, 2 * count.value)
    codes = [(int(words[2 * i]) << 64) | int(words[2 * i + 1])
             for i in range(count.value)]
    return codes, int(h.value)


def is_motif_wide(seqs, n, m, l, d, code) -> bool:
    code = int(code)
    rc = _load().oracle_is_motif_wide(_seq_bytes(seqs), n, m, l, d,
                                      (code >> 64) & (2**64 - 1),
                                      code & (2**64 - 1))
    if rc < 0:
        raise OracleError(rc, "oracle_is_motif_wide")
    return rc == 1


def nb(l, d, sigma=4) -> int:
    return int(_load().oracle_nb(l, d, sigma))


def groups(lmer: bytes):
    g1, g0 = ctypes.c_uint32(0), ctypes.c_uint32(0)
    rc = _load().oracle_groups(lmer, len(lmer), ctypes.byref(g1),
                               ctypes.byref(g0))
    if rc != OR_OK:
        raise OracleError(rc, "oracle_groups")
    return int(g1.value), int(g0.value)


def hamming_groups(a, b) -> int:
    return int(_load().oracle_hamming_groups(a[0], a[1], b[0], b[1]))


def hamming_naive(a: bytes, b: bytes) -> int:
    return int(_load().oracle_hamming_naive(a, b, len(a)))


def lmer_code(lmer: bytes) -> int:
    return int(_load().oracle_lmer_code(lmer, len(lmer)))


def encode(seqs: bytes):
    """ASCII -> base codes; returns (status, codes, index of first bad byte)."""
    buf = np.zeros(len(seqs), dtype=np.uint8)
    bad = ctypes.c_longlong(0)
    rc = _load().oracle_encode(seqs, len(seqs), buf.ctypes.data,
                               ctypes.byref(bad))
    return rc, buf, int(bad.value)


def decode_code(code: int, l: int) -> bytes:
    return bytes(b"ACGT"[(int(code) >> (2 * (l - 1 - j))) & 3]
                 for j in range(l))
