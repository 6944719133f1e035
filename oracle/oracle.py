"""ctypes front-end of the byte-by-byte C oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  The product path (the HIP library and its
binding) never imports this module, and this module imports nothing from it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# flag bits, record and verdict layouts -- declared here independently
SRC_UNADDR, SRC_UNDEF, SRC_UNALLOC, SRC_OVERRUN = 1, 2, 4, 8
DST_UNADDR, DST_UNALLOC, DST_OVERRUN, OVERLAP, BAD_KIND = 16, 32, 64, 128, 256
NONE = 0xFFFF_FFFF_FFFF_FFFF
MODE_CHECK, MODE_PROPAGATE = 1, 2
RACE_SRC, RACE_DST, RACE_UNCHECKED = 1, 2, 4
PTR_UNALLOC = 1
PTR = np.dtype([("flags", "<u4"), ("reserved", "<u4"), ("base", "<u8"), ("avail", "<u8")])
REC = np.dtype([("src", "<u8"), ("dst", "<u8"), ("n", "<u8"), ("kind", "<u4"), ("reserved", "<u4")])
VER = np.dtype([("flags", "<u4"), ("reserved", "<u4"), ("first_bad", "<u8"),
                ("undef_bytes", "<u8"), ("avail", "<u8")])


def build(cc: str = "gcc", out: str = LIB, src: str = SRC, extra=()) -> str:
    """Compile the oracle: plain C, -O2, no vector intrinsics."""
    cmd = [cc, "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra", *extra, "-o", out, src]
    subprocess.run(cmd, check=True)
    return out


_lib = None
_lock = threading.Lock()


def load(path: str = LIB):
    global _lib
    with _lock:
        if _lib is None or path != LIB:
            if not os.path.exists(path):
                build(out=path)
            lib = ctypes.CDLL(path)
            lib.oracle_run.restype = ctypes.c_int
            lib.oracle_run.argtypes = [
                ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]
            lib.oracle_pointers.restype = None
            lib.oracle_pointers.argtypes = [ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                            ctypes.c_void_p, ctypes.c_void_p]
            lib.oracle_race.restype = None
            lib.oracle_race.argtypes = [
                ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
            if path != LIB:
                return lib
            _lib = lib
    return _lib


class OracleState:
    """Host region plus live allocations, all as numpy arrays owned here.

    hv: uint8[hl]; ha: uint64[ceil(hl/64)]; allocs: list of (base, size, V)."""

    def __init__(self, hb, hl, hv, ha, bases, sizes, vs, lib=None):
        self.hb, self.hl = int(hb), int(hl)
        self.hv = np.ascontiguousarray(hv, np.uint8)
        self.ha = np.ascontiguousarray(ha, np.uint64)
        assert self.hv.size == self.hl and self.ha.size >= (self.hl + 63) // 64
        self.bases = np.ascontiguousarray(bases, np.uint64)
        self.sizes = np.ascontiguousarray(sizes, np.uint64)
        self.vs = [np.ascontiguousarray(v, np.uint8) for v in vs]
        assert len(self.vs) == self.bases.size == self.sizes.size
        for v, s in zip(self.vs, self.sizes):
            assert v.size == int(s)
        self._ptrs = (ctypes.c_void_p * max(1, len(self.vs)))(*[v.ctypes.data for v in self.vs])
        self.lib = lib or load()

    def alloc_index(self, base) -> int:
        return int(np.flatnonzero(self.bases == np.uint64(base))[0])

    def run(self, records, check=True, propagate=False) -> np.ndarray:
        recs = np.ascontiguousarray(records, REC)
        out = np.zeros(recs.size, VER)
        mode = (MODE_CHECK if check else 0) | (MODE_PROPAGATE if propagate else 0)
        rc = self.lib.oracle_run(self.hb, self.hl, self.hv.ctypes.data, self.ha.ctypes.data,
                                 len(self.vs), self.bases.ctypes.data, self.sizes.ctypes.data,
                                 ctypes.cast(self._ptrs, ctypes.c_void_p),
                                 recs.size, recs.ctypes.data, out.ctypes.data, mode)
        if rc != 0:
            raise MemoryError("oracle snapshot allocation failed")
        return out

    def run2d(self, records2d, check=True, propagate=False) -> np.ndarray:
        """Pitched 2D copies: all rows of all records as one batch (snapshot
        semantics), then one verdict per record (see combine_rows)."""
        rows, first, counts = expand_rows(records2d)
        rv = self.run(rows, check=check, propagate=propagate)
        return combine_rows(records2d, rv, first, counts)

    def run_threads(self, records, threads: int) -> np.ndarray:
        """Check-only evaluation split over contiguous record ranges on
        `threads` host threads (ctypes releases the GIL during the call)."""
        recs = np.ascontiguousarray(records, REC)
        out = np.zeros(recs.size, VER)
        bounds = np.linspace(0, recs.size, threads + 1).astype(np.int64)

        def work(a, b):
            if b > a:
                self.lib.oracle_run(self.hb, self.hl, self.hv.ctypes.data, self.ha.ctypes.data,
                                    len(self.vs), self.bases.ctypes.data, self.sizes.ctypes.data,
                                    ctypes.cast(self._ptrs, ctypes.c_void_p), b - a,
                                    recs[a:b].ctypes.data, out[a:b].ctypes.data, MODE_CHECK)

        ts = [threading.Thread(target=work, args=(int(bounds[i]), int(bounds[i + 1])))
              for i in range(threads)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        return out


REC2D = np.dtype([("src", "<u8"), ("dst", "<u8"), ("width", "<u8"), ("rows", "<u8"), ("spitch", "<u8"),
                  ("dpitch", "<u8"), ("kind", "<u4"), ("reserved", "<u4", (3,))])


def expand_rows(records2d):
    """The row records of pitched 2D copies (the strided copies of the
    footnote to Sec. 2's error list): row r of a record reads
    [src + r*spitch, + width) and writes [dst + r*dpitch, + width).  Returns
    the rows and, per 2D record, the index of its first row."""
    r2 = np.ascontiguousarray(records2d, REC2D)
    counts = np.where(r2["width"] > 0, r2["rows"], 0).astype(np.int64)
    first = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)
    rows = np.zeros(int(counts.sum()), REC)
    k = 0
    for t in range(r2.size):
        for r in range(int(counts[t])):
            rows[k] = (int(r2["src"][t]) + r * int(r2["spitch"][t]), int(r2["dst"][t]) + r * int(r2["dpitch"][t]),
                       int(r2["width"][t]), int(r2["kind"][t]), 0)
            k += 1
    return rows, first, counts


def combine_rows(records2d, row_verdicts, first, counts):
    """One verdict per 2D record from its rows' verdicts: the bytes of the copy
    are numbered row by row (byte c of row r is r*width + c), so flags are the
    OR over rows, first_bad the smallest r*width + first_bad_r, undef_bytes the
    sum, and avail the first row's (bytes from the copy's start pointer to the
    end of its allocation).  No rows: {0, NONE, 0, 0}; a bad kind with rows
    gives the rows' BAD_KIND."""
    r2 = np.ascontiguousarray(records2d, REC2D)
    out = np.zeros(r2.size, VER)
    out["first_bad"] = NONE
    for t in range(r2.size):
        w = int(r2["width"][t])
        for r in range(int(counts[t])):
            v = row_verdicts[int(first[t]) + r]
            out["flags"][t] |= v["flags"]
            if int(v["first_bad"]) != NONE:
                out["first_bad"][t] = min(int(out["first_bad"][t]), r * w + int(v["first_bad"]))
            out["undef_bytes"][t] += v["undef_bytes"]
        if counts[t]:
            out["avail"][t] = row_verdicts[int(first[t])]["avail"]
    return out


def race(records, streams, epochs=None, which=None, threads: int = 1, lib=None) -> np.ndarray:
    """Concurrent-access flags (RACE_*) of the records listed in `which`
    (default: all), each compared with every other record of the batch;
    the reading of Sec. 2's concurrent accesses is stated in oracle.c."""
    lib = lib or load()
    recs = np.ascontiguousarray(records, REC)
    st = np.ascontiguousarray(streams, np.uint32)
    ep = None if epochs is None else np.ascontiguousarray(epochs, np.uint32)
    assert st.size == recs.size and (ep is None or ep.size == recs.size)
    idx = np.arange(recs.size, dtype=np.uint64) if which is None else np.ascontiguousarray(which, np.uint64)
    out = np.zeros(idx.size, np.uint32)
    bounds = np.linspace(0, idx.size, max(1, threads) + 1).astype(np.int64)

    def work(a, b):
        if b > a:
            lib.oracle_race(recs.size, recs.ctypes.data, st.ctypes.data,
                            None if ep is None else ep.ctypes.data, b - a,
                            idx[a:b].ctypes.data, out[a:b].ctypes.data)

    ts = [threading.Thread(target=work, args=(int(bounds[i]), int(bounds[i + 1])))
          for i in range(len(bounds) - 1)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    return out


def conflict(ra, rb, sa, sb, ea=0, eb=0):
    """(dst_hit, src_hit) of record a against one other record b: whether
    a's written bytes meet b's read or written bytes, and whether a's read
    bytes meet b's written bytes, when the two are unordered (different
    streams, same epoch) and both are checked.  One pair, by definition."""
    def checked(r):
        return int(r["kind"]) <= 2

    def meets(a, na, b, nb):
        return na > 0 and nb > 0 and a < b + nb and b < a + na

    if not (checked(ra) and checked(rb)) or int(ea) != int(eb) or int(sa) == int(sb):
        return False, False
    n_a, n_b = int(ra["n"]), int(rb["n"])
    dst = meets(int(ra["dst"]), n_a, int(rb["dst"]), n_b) or meets(int(ra["dst"]), n_a, int(rb["src"]), n_b)
    src = meets(int(ra["src"]), n_a, int(rb["dst"]), n_b)
    return dst, src


def pointers(bases, sizes, ptrs, lib=None) -> np.ndarray:
    """Check pointers (kernel arguments, Sec. 5.1) against live allocations
    given as base and size arrays; the reading is stated in oracle.c."""
    lib = lib or load()
    b = np.ascontiguousarray(bases, np.uint64)
    z = np.ascontiguousarray(sizes, np.uint64)
    p = np.ascontiguousarray(ptrs, np.uint64)
    out = np.zeros(p.size, PTR)
    lib.oracle_pointers(b.size, b.ctypes.data, z.ctypes.data, p.size, p.ctypes.data, out.ctypes.data)
    return out
