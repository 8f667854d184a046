"""Exact planted (l,d)-motif search on MI355X (gfx950): Python binding.

Thin ctypes marshalling over the C ABI of ``libpms.so`` (``include/pms.h``):
every step of the search runs in the library's HIP kernels. There is no
fallback: if the library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpms.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "pms.h")

PMS_OK, PMS_PENDING = 0, 1
PMS_EINVAL, PMS_EBASE, PMS_ENOMEM, PMS_EDEVICE, PMS_EBUSY = -1, -2, -3, -4, -5
PATH_AUTO, PATH_FILTER, PATH_BITSET, PATH_TILED, PATH_PAIR = 0, 1, 2, 3, 4
PATH_NAMES = {PATH_FILTER: "filter", PATH_BITSET: "bitset", PATH_TILED: "tiled",
              PATH_PAIR: "pair"}


class PmsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_STATUS.get(status, status), message))
        self.status = status


_STATUS = {PMS_EINVAL: "PMS_EINVAL", PMS_EBASE: "PMS_EBASE",
           PMS_ENOMEM: "PMS_ENOMEM", PMS_EDEVICE: "PMS_EDEVICE",
           PMS_EBUSY: "PMS_EBUSY", PMS_PENDING: "PMS_PENDING"}


class Options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("path", ctypes.c_int),
                ("mem_budget_bytes", ctypes.c_size_t),
                ("tune_cache", ctypes.c_char_p),
                ("serve_slots", ctypes.c_int), ("serve_queue", ctypes.c_int),
                ("tile_threads", ctypes.c_int),
                ("serve_launch_ms", ctypes.c_double),
                ("pair_partner", ctypes.c_int)]


class CInstance(ctypes.Structure):
    _fields_ = [("seqs", ctypes.c_char_p), ("n", ctypes.c_int),
                ("m", ctypes.c_int), ("l", ctypes.c_int), ("d", ctypes.c_int),
                ("q", ctypes.c_int)]


class CResult(ctypes.Structure):
    _fields_ = [("motifs", ctypes.POINTER(ctypes.c_uint64)),
                ("count", ctypes.c_size_t), ("status", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int), ("tile_suffix", ctypes.c_int),
                ("ms_total", ctypes.c_double), ("ms_index", ctypes.c_double),
                ("ms_main", ctypes.c_double), ("ms_output", ctypes.c_double),
                ("main_launches", ctypes.c_uint64),
                ("hcanon", ctypes.c_uint64), ("tiles", ctypes.c_uint64),
                ("tile_passes", ctypes.c_uint64), ("marks", ctypes.c_uint64),
                ("filter_tests", ctypes.c_uint64),
                ("bytes_main", ctypes.c_uint64), ("retries", ctypes.c_uint64),
                ("pairs", ctypes.c_uint64), ("candidates", ctypes.c_uint64),
                ("tile_threads", ctypes.c_int),
                ("graph_replayed", ctypes.c_int)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("launches", ctypes.c_uint64),
                ("max_inflight", ctypes.c_uint64),
                ("busy_ms", ctypes.c_double), ("retries", ctypes.c_uint64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpms.so and declare its signatures (raises if it is absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libpms.so not built: run __graft_entry__.build() "
                          "(or python paper_2403_00306_amd/build.py)")
    # One HIP runtime per process: torch ships its own libamdhip64 and
    # requests it by a name that does not match an already loaded system
    # copy, so load torch first; libpms then binds to the same runtime
    # (same soname) and torch-owned buffers and streams are shared.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp, i, sz, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_uint64
    sig = {
        "pms_default_options": (None, [P(Options)]),
        "pms_create": (i, [P(vp), P(Options)]),
        "pms_destroy": (None, [vp]),
        "pms_last_error": (ctypes.c_char_p, [vp]),
        "pms_status_string": (ctypes.c_char_p, [i]),
        "pms_solve": (i, [vp, ctypes.c_char_p, i, i, i, i,
                          P(P(ctypes.c_uint64)), P(sz)]),
        "pms_solve_device": (i, [vp, vp, i, i, i, i, vp, vp, sz, P(sz)]),
        "pms_solve_device_noalloc": (i, [vp, vp, i, i, i, i, vp, vp, sz,
                                         P(sz)]),
        "pms_solve_quorum": (i, [vp, ctypes.c_char_p, i, i, i, i, i,
                                 P(P(ctypes.c_uint64)), P(sz)]),
        "pms_solve_quorum_device": (i, [vp, vp, i, i, i, i, i, vp, vp, sz,
                                        P(sz)]),
        "pms_solve_alphabet": (i, [vp, ctypes.c_char_p, i, ctypes.c_char_p,
                                   i, i, i, i, P(P(ctypes.c_uint64)), P(sz)]),
        "pms_solve_alphabet_device": (i, [vp, ctypes.c_char_p, i, vp, i, i,
                                          i, i, vp, vp, sz, P(sz)]),
        "pms_solve_wide": (i, [vp, ctypes.c_char_p, i, i, i, i,
                               P(P(ctypes.c_uint64)), P(sz)]),
        "pms_solve_wide_device": (i, [vp, vp, i, i, i, i, vp, vp, sz,
                                      P(sz)]),
        "pms_solve_batch": (i, [vp, P(CInstance), i, P(CResult)]),
        "pms_submit": (i, [vp, P(CInstance), P(u64)]),
        "pms_poll": (i, [vp, u64, P(CResult)]),
        "pms_wait": (i, [vp, u64, i, P(CResult)]),
        "pms_release": (i, [vp, u64]),
        "pms_ticket_times": (i, [vp, u64, P(ctypes.c_double),
                                 P(ctypes.c_double), P(ctypes.c_double)]),
        "pms_clock_ms": (ctypes.c_double, []),
        "pms_test_rate": (i, [vp, P(ctypes.c_double)]),
        "pms_lds_rate": (i, [vp, P(ctypes.c_double)]),
        "pms_last_stats": (i, [vp, P(Stats)]),
        "pms_serve_stats_get": (i, [vp, P(ServeStats)]),
        "pms_last_hcanon_per_ref": (i, [vp, P(ctypes.c_uint64), sz]),
        "pms_autotune": (i, [vp, i, i, i, i, P(i), P(i)]),
        "pms_set_tile_config": (i, [vp, i, i, i, i]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def header_functions(path: str = HEADER) -> list:
    """Names of the functions declared in include/pms.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pms_[a-z_]+)\s*\(", text)))


def _as_bytes(seqs) -> bytes:
    if isinstance(seqs, (bytes, bytearray)):
        return bytes(seqs)
    if isinstance(seqs, np.ndarray):
        return seqs.astype(np.uint8).tobytes()
    if isinstance(seqs, (list, tuple)):
        return b"".join(seqs)
    raise TypeError("seqs must be bytes, a uint8 array or a list of rows")


@dataclass
class Request:
    ticket: int
    n: int
    m: int
    l: int
    d: int


class Context:
    """One libpms context (one device, one stream, one serving engine)."""

    def __init__(self, device: int = 0, path: int = PATH_AUTO,
                 mem_budget_bytes: int = 0, tune_cache: str | None = None,
                 serve_slots: int = 0, serve_queue: int = 0,
                 tile_threads: int = 0, serve_launch_ms: float = 0.0,
                 pair_partner: int = 0):
        self._lib = load_library()
        opt = Options()
        self._lib.pms_default_options(ctypes.byref(opt))
        opt.device = device
        opt.path = path
        opt.mem_budget_bytes = mem_budget_bytes
        opt.tune_cache = tune_cache.encode() if tune_cache else None
        opt.serve_slots = serve_slots
        opt.serve_queue = serve_queue
        opt.tile_threads = tile_threads
        opt.serve_launch_ms = serve_launch_ms
        opt.pair_partner = pair_partner
        h = ctypes.c_void_p()
        rc = self._lib.pms_create(ctypes.byref(h), ctypes.byref(opt))
        if rc != PMS_OK:
            raise PmsError(rc, self._lib.pms_last_error(None).decode())
        self._h = h

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        h, self._h = getattr(self, "_h", None), None
        if h:
            self._lib.pms_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc: int):
        if rc < 0:
            raise PmsError(rc, self._lib.pms_last_error(self._h).decode())
        return rc

    @property
    def handle(self):
        return self._h

    # -- plain -------------------------------------------------------------
    def solve(self, seqs, n: int, m: int, l: int, d: int) -> np.ndarray:
        buf = _as_bytes(seqs)
        if len(buf) != n * m:
            raise ValueError("seqs holds %d bytes, expected n*m=%d"
                             % (len(buf), n * m))
        ptr = ctypes.POINTER(ctypes.c_uint64)()
        cnt = ctypes.c_size_t(0)
        self._check(self._lib.pms_solve(self._h, buf, n, m, l, d,
                                        ctypes.byref(ptr), ctypes.byref(cnt)))
        if cnt.value == 0:
            return np.zeros(0, dtype=np.uint64)
        return np.ctypeslib.as_array(ptr, shape=(cnt.value,)).copy()

    def solve_device(self, d_seqs: int, n: int, m: int, l: int, d: int,
                     d_out: int, cap: int, stream: int = 0) -> int:
        """Device-resident solve; pointers are integers (e.g. from torch's
        ``tensor.data_ptr()`` and ``torch.cuda.Stream.cuda_stream``)."""
        cnt = ctypes.c_size_t(0)
        rc = self._lib.pms_solve_device(self._h, ctypes.c_void_p(d_seqs), n,
                                        m, l, d, ctypes.c_void_p(stream),
                                        ctypes.c_void_p(d_out), cap,
                                        ctypes.byref(cnt))
        if rc == PMS_ENOMEM and cnt.value > cap:
            err = PmsError(rc, self._lib.pms_last_error(self._h).decode())
            err.needed = cnt.value
            raise err
        self._check(rc)
        return cnt.value

    def solve_device_noalloc(self, d_seqs: int, n: int, m: int, l: int,
                             d: int, d_out: int, cap: int,
                             stream: int = 0) -> int:
        """solve_device that allocates nothing (tiled path, fixed device
        scratch); same arguments and errors."""
        cnt = ctypes.c_size_t(0)
        rc = self._lib.pms_solve_device_noalloc(
            self._h, ctypes.c_void_p(d_seqs), n, m, l, d,
            ctypes.c_void_p(stream), ctypes.c_void_p(d_out), cap,
            ctypes.byref(cnt))
        if rc == PMS_ENOMEM and cnt.value > 0:
            err = PmsError(rc, self._lib.pms_last_error(self._h).decode())
            err.needed = cnt.value
            raise err
        self._check(rc)
        return cnt.value

    def solve_quorum(self, seqs, n: int, m: int, l: int, d: int,
                     q: int) -> np.ndarray:
        """(l,d,q)-motifs: l-mers with a d-neighbour in at least q strings."""
        buf = _as_bytes(seqs)
        if len(buf) != n * m:
            raise ValueError("seqs holds %d bytes, expected n*m=%d"
                             % (len(buf), n * m))
        ptr = ctypes.POINTER(ctypes.c_uint64)()
        cnt = ctypes.c_size_t(0)
        self._check(self._lib.pms_solve_quorum(self._h, buf, n, m, l, d, q,
                                               ctypes.byref(ptr),
                                               ctypes.byref(cnt)))
        if cnt.value == 0:
            return np.zeros(0, dtype=np.uint64)
        return np.ctypeslib.as_array(ptr, shape=(cnt.value,)).copy()

    def solve_quorum_device(self, d_seqs: int, n: int, m: int, l: int,
                            d: int, q: int, d_out: int, cap: int,
                            stream: int = 0) -> int:
        """Device-resident quorum solve (as solve_device)."""
        cnt = ctypes.c_size_t(0)
        rc = self._lib.pms_solve_quorum_device(
            self._h, ctypes.c_void_p(d_seqs), n, m, l, d, q,
            ctypes.c_void_p(stream), ctypes.c_void_p(d_out), cap,
            ctypes.byref(cnt))
        if rc == PMS_ENOMEM and cnt.value > cap:
            err = PmsError(rc, self._lib.pms_last_error(self._h).decode())
            err.needed = cnt.value
            raise err
        self._check(rc)
        return cnt.value

    def solve_alphabet(self, alphabet: bytes, seqs, n: int, m: int, l: int,
                       d: int) -> np.ndarray:
        """Motifs over the given alphabet; codes in base len(alphabet)."""
        buf = _as_bytes(seqs)
        if len(buf) != n * m:
            raise ValueError("seqs holds %d bytes, expected n*m=%d"
                             % (len(buf), n * m))
        a = bytes(alphabet)
        ptr = ctypes.POINTER(ctypes.c_uint64)()
        cnt = ctypes.c_size_t(0)
        self._check(self._lib.pms_solve_alphabet(self._h, a, len(a), buf, n,
                                                 m, l, d, ctypes.byref(ptr),
                                                 ctypes.byref(cnt)))
        if cnt.value == 0:
            return np.zeros(0, dtype=np.uint64)
        return np.ctypeslib.as_array(ptr, shape=(cnt.value,)).copy()

    def solve_alphabet_device(self, alphabet: bytes, d_seqs: int, n: int,
                              m: int, l: int, d: int, d_out: int, cap: int,
                              stream: int = 0) -> int:
        """Device-resident solve_alphabet (as solve_device)."""
        a = bytes(alphabet)
        cnt = ctypes.c_size_t(0)
        rc = self._lib.pms_solve_alphabet_device(
            self._h, a, len(a), ctypes.c_void_p(d_seqs), n, m, l, d,
            ctypes.c_void_p(stream), ctypes.c_void_p(d_out), cap,
            ctypes.byref(cnt))
        if rc == PMS_ENOMEM and cnt.value > cap:
            err = PmsError(rc, self._lib.pms_last_error(self._h).decode())
            err.needed = cnt.value
            raise err
        self._check(rc)
        return cnt.value

    def solve_wide(self, seqs, n: int, m: int, l: int, d: int) -> np.ndarray:
        """Motifs of length up to 64: a (count, 2) uint64 array, row i the
        high and low word of motif i's 128-bit code, ascending."""
        buf = _as_bytes(seqs)
        if len(buf) != n * m:
            raise ValueError("seqs holds %d bytes, expected n*m=%d"
                             % (len(buf), n * m))
        ptr = ctypes.POINTER(ctypes.c_uint64)()
        cnt = ctypes.c_size_t(0)
        self._check(self._lib.pms_solve_wide(self._h, buf, n, m, l, d,
                                             ctypes.byref(ptr),
                                             ctypes.byref(cnt)))
        if cnt.value == 0:
            return np.zeros((0, 2), dtype=np.uint64)
        return np.ctypeslib.as_array(
            ptr, shape=(2 * cnt.value,)).copy().reshape(cnt.value, 2)

    def solve_wide_device(self, d_seqs: int, n: int, m: int, l: int, d: int,
                          d_out: int, cap: int, stream: int = 0) -> int:
        """Device-resident solve_wide: d_out holds 2*cap uint64 words;
        returns the number of motifs."""
        cnt = ctypes.c_size_t(0)
        rc = self._lib.pms_solve_wide_device(
            self._h, ctypes.c_void_p(d_seqs), n, m, l, d,
            ctypes.c_void_p(stream), ctypes.c_void_p(d_out), cap,
            ctypes.byref(cnt))
        if rc == PMS_ENOMEM and cnt.value > cap:
            err = PmsError(rc, self._lib.pms_last_error(self._h).decode())
            err.needed = cnt.value
            raise err
        self._check(rc)
        return cnt.value

    # -- batch -------------------------------------------------------------
    def solve_batch(self, instances) -> list:
        """instances: iterable of (seqs, n, m, l, d[, q]) or objects with
        those attributes (q, the quorum, optional: 0 or n for the plain
        search). Returns a list of uint64 arrays (or PmsError objects for
        instances that failed)."""
        insts = []
        keep = []
        for x in instances:
            if isinstance(x, tuple):
                seqs, n, m, l, d = x[:5]
                q = x[5] if len(x) > 5 else 0
            else:
                seqs, n, m, l, d = x.seqs, x.n, x.m, x.l, x.d
                q = getattr(x, "q", 0)
            b = _as_bytes(seqs)
            keep.append(b)
            insts.append(CInstance(b, n, m, l, d, q))
        k = len(insts)
        arr = (CInstance * max(k, 1))(*insts)
        res = (CResult * max(k, 1))()
        rc = self._lib.pms_solve_batch(self._h, arr, k, res)
        if rc == PMS_EDEVICE or rc == PMS_ENOMEM:
            self._check(rc)
        out = []
        for i in range(k):
            r = res[i]
            if r.status != PMS_OK:
                out.append(PmsError(r.status, "batch instance %d" % i))
            elif r.count == 0:
                out.append(np.zeros(0, dtype=np.uint64))
            else:
                out.append(np.ctypeslib.as_array(r.motifs,
                                                 shape=(r.count,)).copy())
        return out

    # -- serving -----------------------------------------------------------
    def submit(self, seqs, n: int, m: int, l: int, d: int) -> int:
        b = _as_bytes(seqs)
        inst = CInstance(b, n, m, l, d)
        t = ctypes.c_uint64(0)
        self._check(self._lib.pms_submit(self._h, ctypes.byref(inst),
                                         ctypes.byref(t)))
        return int(t.value)

    def _result(self, rc, r):
        if rc == PMS_PENDING:
            return None
        if rc < 0:
            raise PmsError(rc, self._lib.pms_last_error(self._h).decode())
        if r.count == 0:
            return np.zeros(0, dtype=np.uint64)
        return np.ctypeslib.as_array(r.motifs, shape=(r.count,)).copy()

    def poll(self, ticket: int):
        r = CResult()
        rc = self._lib.pms_poll(self._h, ticket, ctypes.byref(r))
        return self._result(rc, r)

    def wait(self, ticket: int, timeout_ms: int = -1):
        r = CResult()
        rc = self._lib.pms_wait(self._h, ticket, timeout_ms, ctypes.byref(r))
        return self._result(rc, r)

    def release(self, ticket: int):
        self._check(self._lib.pms_release(self._h, ticket))

    def ticket_times(self, ticket: int):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(self._lib.pms_ticket_times(self._h, ticket,
                                               ctypes.byref(a),
                                               ctypes.byref(b),
                                               ctypes.byref(c)))
        return a.value, b.value, c.value

    def clock_ms(self) -> float:
        return float(self._lib.pms_clock_ms())

    def test_rate(self) -> float:
        """Hamming tests/s of the filter's instruction mix on this device
        (calibration of the integer peak; runs a short kernel)."""
        r = ctypes.c_double(0.0)
        self._check(self._lib.pms_test_rate(self._h, ctypes.byref(r)))
        return float(r.value)

    def lds_rate(self) -> float:
        """Device-wide rate of single-bit LDS atomic ORs (lane ORs/s)."""
        r = ctypes.c_double(0)
        self._check(self._lib.pms_lds_rate(self._h, ctypes.byref(r)))
        return r.value

    def serve_stats(self) -> dict:
        s = ServeStats()
        self._check(self._lib.pms_serve_stats_get(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in ServeStats._fields_}

    # -- introspection and tuning -------------------------------------------
    def stats(self) -> dict:
        s = Stats()
        self._check(self._lib.pms_last_stats(self._h, ctypes.byref(s)))
        d = {f: getattr(s, f) for f, _ in Stats._fields_}
        d["path_name"] = PATH_NAMES.get(d["path"], "?")
        return d

    def hcanon_per_ref(self, n_refs: int) -> np.ndarray:
        out = np.zeros(n_refs, dtype=np.uint64)
        self._check(self._lib.pms_last_hcanon_per_ref(
            self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
            n_refs))
        return out

    def autotune(self, n: int, m: int, l: int, d: int):
        s, t = ctypes.c_int(0), ctypes.c_int(0)
        self._check(self._lib.pms_autotune(self._h, n, m, l, d,
                                           ctypes.byref(s), ctypes.byref(t)))
        return s.value, t.value

    def set_tile_config(self, l: int, d: int, s: int, surv_t: int):
        self._check(self._lib.pms_set_tile_config(self._h, l, d, s, surv_t))
