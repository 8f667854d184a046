"""Seeded synthetic planted-motif instances (FM model) and workload recipes.

This package only draws random inputs: ASCII DNA sequences with one planted
(l, d) motif occurrence per sequence. It holds none of the motif-search
arithmetic, so the CPU oracle and the GPU library both consume its bytes
without sharing code. The random source is xoshiro256** seeded by SplitMix64
(``pmsgen.c`` states the planting rule and the draw order).

The workloads mirror the thesis's experimental setting (Table 3.2: DNA,
n = 20 sequences of length m = 600) with planted motifs generated the way its
FM-model datasets were (Sec. 3.4); those datasets are not available, so these
synthetic instances stand in for them.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pmsgen.c")
_LIB = os.path.join(_HERE, "libpmsgen.so")


def build(force: bool = True) -> str:
    """Compile libpmsgen.so with gcc (portable x86-64 flags)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.pmsgen_rng_new.restype = ctypes.c_void_p
        lib.pmsgen_rng_new.argtypes = [ctypes.c_uint64]
        lib.pmsgen_rng_free.argtypes = [ctypes.c_void_p]
        lib.pmsgen_next.restype = ctypes.c_uint64
        lib.pmsgen_next.argtypes = [ctypes.c_void_p]
        lib.pmsgen_bounded.restype = ctypes.c_uint64
        lib.pmsgen_bounded.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        lib.pmsgen_uniform01.restype = ctypes.c_double
        lib.pmsgen_uniform01.argtypes = [ctypes.c_void_p]
        lib.pmsgen_splitmix64.restype = ctypes.c_uint64
        lib.pmsgen_splitmix64.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
        lib.pmsgen_planted_alpha.restype = ctypes.c_int
        lib.pmsgen_planted_alpha.argtypes = [
            ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_int, ctypes.c_char_p, ctypes.c_int, ctypes.c_char_p,
            ctypes.c_char_p]
        lib.pmsgen_planted.restype = ctypes.c_int
        lib.pmsgen_planted.argtypes = [
            ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
            ctypes.c_int, ctypes.c_char_p, ctypes.c_char_p,
            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        _lib = lib
    return _lib


class Rng:
    """xoshiro256** stream (C implementation)."""

    def __init__(self, seed: int):
        self._lib = _load()
        self._h = self._lib.pmsgen_rng_new(ctypes.c_uint64(seed & (2**64 - 1)))

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h:
            self._lib.pmsgen_rng_free(h)

    def next(self) -> int:
        return int(self._lib.pmsgen_next(self._h))

    def bounded(self, n: int) -> int:
        return int(self._lib.pmsgen_bounded(self._h, n))

    def uniform01(self) -> float:
        return float(self._lib.pmsgen_uniform01(self._h))


@dataclass
class Instance:
    """One planted PMS instance. ``seqs`` is n*m ASCII bytes, row-major."""
    seed: int
    n: int
    m: int
    l: int
    d: int
    seqs: bytes
    motif: bytes = b""
    positions: list = field(default_factory=list)
    mutated: list = field(default_factory=list)

    def rows(self) -> list:
        return [self.seqs[i * self.m:(i + 1) * self.m] for i in range(self.n)]


def planted(seed: int, n: int, m: int, l: int, d: int) -> Instance:
    """One FM-model instance: n sequences of length m, one (l, d) plant each."""
    lib = _load()
    seqs = ctypes.create_string_buffer(n * m)
    motif = ctypes.create_string_buffer(max(l, 1))
    pos = (ctypes.c_int32 * n)()
    mut = (ctypes.c_int32 * max(n * d, 1))()
    rc = lib.pmsgen_planted(ctypes.c_uint64(seed), n, m, l, d, seqs, motif,
                            pos, mut)
    if rc != 0:
        raise ValueError("pmsgen_planted: bad sizes n=%d m=%d l=%d d=%d"
                         % (n, m, l, d))
    return Instance(seed=seed, n=n, m=m, l=l, d=d, seqs=seqs.raw[:n * m],
                    motif=motif.raw[:l], positions=list(pos),
                    mutated=[list(mut[i * d:(i + 1) * d]) for i in range(n)])


PROTEIN = b"ACDEFGHIKLMNPQRSTVWY"   # the 20 amino-acid letters


def planted_alpha(seed: int, n: int, m: int, l: int, d: int,
                  alphabet: bytes = PROTEIN) -> Instance:
    """FM-model instance over an arbitrary alphabet (2..32 letters)."""
    lib = _load()
    seqs = ctypes.create_string_buffer(n * m)
    motif = ctypes.create_string_buffer(max(l, 1))
    rc = lib.pmsgen_planted_alpha(ctypes.c_uint64(seed), n, m, l, d,
                                  bytes(alphabet), len(alphabet), seqs, motif)
    if rc != 0:
        raise ValueError("pmsgen_planted_alpha: bad sizes or alphabet")
    return Instance(seed=seed, n=n, m=m, l=l, d=d, seqs=seqs.raw[:n * m],
                    motif=motif.raw[:l])


# ---------------------------------------------------------------------------
# Workload recipes (sizes of the thesis's Table 3.2 and of the batched and
# served mixes built on them).
# ---------------------------------------------------------------------------

PLAIN_CONFIGS = {
    "pms_9_2": (20, 600, 9, 2),
    "pms_13_4": (20, 600, 13, 4),
    "pms_17_6": (20, 600, 17, 6),
    "pms_19_7": (20, 600, 19, 7),
}

BATCH_CLASSES = [(9, 2), (11, 3), (13, 4), (15, 5)]
SERVE_CLASSES = [(9, 2), (11, 3), (13, 4), (15, 5), (17, 6), (19, 7)]
SERVE_WEIGHTS = [30, 25, 20, 15, 8, 2]


def plain(name: str, seed: int) -> Instance:
    n, m, l, d = PLAIN_CONFIGS[name]
    return planted(seed, n, m, l, d)


def batched(seed: int = 7, count: int = 256) -> list:
    """(l,d) uniform over BATCH_CLASSES, n in [10,40], m in [300,1000]."""
    r = Rng(seed)
    out = []
    for _ in range(count):
        l, d = BATCH_CLASSES[r.bounded(len(BATCH_CLASSES))]
        n = 10 + r.bounded(31)
        m = 300 + r.bounded(701)
        inst_seed = r.next()
        out.append(planted(inst_seed, n, m, l, d))
    return out


@dataclass
class Request:
    index: int
    arrival_unit: float   # arrival time at rate 1 (scale by 1/lambda)
    inst: Instance


def served(seed: int = 11, count: int = 2000, classes=None, weights=None,
           n: int = 20) -> list:
    """Poisson stream: (l,d) by weight, n = 20, m in [400,800].

    Arrival times are cumulative Exp(1) gaps; a caller running at rate
    lambda uses arrival_unit / lambda.
    """
    classes = classes or SERVE_CLASSES
    weights = weights or SERVE_WEIGHTS
    total_w = sum(weights)
    r = Rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        u = r.bounded(total_w)
        acc = 0
        for (ld, w) in zip(classes, weights):
            acc += w
            if u < acc:
                l, d = ld
                break
        m = 400 + r.bounded(401)
        inst_seed = r.next()
        t += -math.log1p(-r.uniform01())
        out.append(Request(i, t, planted(inst_seed, n, m, l, d)))
    return out


def as_array(inst: Instance) -> np.ndarray:
    return np.frombuffer(inst.seqs, dtype=np.uint8).reshape(inst.n, inst.m)


# Pure-Python mirror of the stream, used only to cross-check the C code.
_M64 = 2**64 - 1


def py_splitmix64(x: int):
    x = (x + 0x9E3779B97F4A7C15) & _M64
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return x, z ^ (z >> 31)


class PyRng:
    def __init__(self, seed: int):
        x = seed & _M64
        self.s = []
        for _ in range(4):
            x, v = py_splitmix64(x)
            self.s.append(v)

    def next(self) -> int:
        s = self.s
        rot = lambda v, k: ((v << k) | (v >> (64 - k))) & _M64
        result = (rot((s[1] * 5) & _M64, 7) * 9) & _M64
        t = (s[1] << 17) & _M64
        s[2] ^= s[0]
        s[3] ^= s[1]
        s[1] ^= s[2]
        s[0] ^= s[3]
        s[2] ^= t
        s[3] = rot(s[3], 45)
        return result
