"""Brute-force set-definition checker for tiny universes.

TEST INFRASTRUCTURE ONLY.  A second, independent formulation of the transfer
check, written with Python sets over absolute addresses instead of the C
oracle's per-index loop, so that a slip in either one shows up when the two
are compared over every small case.

The model (Cudagrind, arXiv 1310.0901): host memory carries A (addressable)
and V (defined) shadow (Sec. 1.1); device memory is a set of live linear
allocations kept per context (Sec. 2, Fig. 2 caption); a copy is checked for
unallocated or too-small device ranges and for non-addressable or undefined
source bytes (Sec. 2's error list); V is carried along host/device copies in
all three directions (Sec. 5).
"""
from __future__ import annotations

NONE = (1 << 64) - 1
SRC_UNADDR, SRC_UNDEF, SRC_UNALLOC, SRC_OVERRUN = 1, 2, 4, 8
DST_UNADDR, DST_UNALLOC, DST_OVERRUN, OVERLAP, BAD_KIND = 16, 32, 64, 128, 256


class World:
    """hb: host base; hv: dict addr->V byte for every host byte of the region;
    haddr: set of addressable host addresses; allocs: dict base -> list of V."""

    def __init__(self, hb, hv_list, a_list, allocs):
        self.hv = {hb + x: int(b) for x, b in enumerate(hv_list)}
        self.haddr = {hb + x for x, a in enumerate(a_list) if a}
        self.allocs = {int(b): [int(x) for x in v] for b, v in allocs.items()}

    def copy(self):
        w = World.__new__(World)
        w.hv = dict(self.hv)
        w.haddr = set(self.haddr)
        w.allocs = {b: list(v) for b, v in self.allocs.items()}
        return w

    def dev_bytes(self):
        """address -> (base of its allocation)"""
        return {b + k: b for b, v in self.allocs.items() for k in range(len(v))}


def verdict(world: World, kind, src, dst, n):
    """Verdict of one record plus the dict of destination writes it implies."""
    if kind not in (0, 1, 2):
        return (BAD_KIND, NONE, 0, 0), {}
    if n == 0:
        return (0, NONE, 0, 0), {}
    owner = world.dev_bytes()
    idx = range(n)
    src_host, dst_host = kind == 0, kind == 1
    flags = 0

    def side(p, is_host, unalloc_flag, overrun_flag):
        nonlocal flags
        if is_host:
            good = {i for i in idx if p + i in world.haddr}
            return good, None
        base = owner.get(p)
        if base is None:
            flags |= unalloc_flag
            return set(), 0
        # bytes of the same allocation, contiguous from p
        good = {i for i in idx if owner.get(p + i) == base}
        av = base + len(world.allocs[base]) - p
        if len(good) < n:
            flags |= overrun_flag
        return good, av

    ok_s, av_s = side(src, src_host, SRC_UNALLOC, SRC_OVERRUN)
    ok_d, av_d = side(dst, dst_host, DST_UNALLOC, DST_OVERRUN)

    def vsrc(i):
        if src_host:
            return world.hv[src + i]
        base = owner[src + i]
        return world.allocs[base][src + i - base]

    undef = {i for i in ok_s if vsrc(i) != 0}
    bad = (set(idx) - ok_s) | (set(idx) - ok_d) | undef
    if src_host and ok_s != set(idx):
        flags |= SRC_UNADDR
    if dst_host and ok_d != set(idx):
        flags |= DST_UNADDR
    if undef:
        flags |= SRC_UNDEF
    if kind == 2 and set(range(src, src + n)) & set(range(dst, dst + n)):
        flags |= OVERLAP
    avail = min([a for a in (av_s, av_d) if a is not None])
    writes = {}
    if not flags & OVERLAP:
        for i in ok_d:
            writes[dst + i] = vsrc(i) if i in ok_s else 0xFF
    return (flags, min(bad) if bad else NONE, len(undef), avail), writes


def apply_writes(world: World, writes: dict, dst_host: bool):
    owner = world.dev_bytes()
    for addr, val in writes.items():
        if dst_host:
            world.hv[addr] = val
        else:
            b = owner[addr]
            world.allocs[b][addr - b] = val


def run_snapshot(world: World, records, propagate=False):
    """All records read the state before the call; writes land afterwards."""
    out, pending = [], []
    for kind, src, dst, n in records:
        v, w = verdict(world, kind, src, dst, n)
        out.append(v)
        pending.append((w, kind == 1))
    after = world.copy()
    if propagate:
        for w, dh in pending:
            apply_writes(after, w, dh)
    return out, after


def run_sequential(world: World, records, propagate=False):
    """Records applied one after another, each seeing the previous writes."""
    cur = world.copy()
    out = []
    for kind, src, dst, n in records:
        v, w = verdict(cur, kind, src, dst, n)
        out.append(v)
        if propagate:
            apply_writes(cur, w, kind == 1)
    return out, cur


def race_flags(rows, streams, epochs=None):
    """Concurrent-access flags by byte sets: every byte a record reads or
    writes is entered in a map byte -> accesses; a record is flagged where
    one of its bytes is also written (for its reads) or read or written (for
    its writes) by a record of another stream in the same epoch.  rows are
    (kind, src, dst, n) tuples as in run_snapshot; flags use 1 = source,
    2 = destination, 4 = not checked (see oracle.c for the reading).

    Ranges are sets of integers (they may run past 2^64).  So that ranges of
    any length can be enumerated, the bytes are taken piece by piece: between
    two consecutive range ends every byte lies in the same ranges, so one byte
    per piece stands for all of them."""
    epochs = epochs or [0] * len(rows)
    unchecked = {t for t, row in enumerate(rows) if row[0] > 2}
    cuts = sorted({x for t, (kind, src, dst, n) in enumerate(rows) if t not in unchecked
                   for x in (src, src + n, dst, dst + n)})
    touched = {}
    for t, (kind, src, dst, n) in enumerate(rows):
        if t in unchecked:
            continue
        for lo, hi, how in ((src, src + n, "r"), (dst, dst + n, "w")):
            for x in cuts:
                if lo <= x < hi:   # x starts a piece that lies inside [lo, hi)
                    touched.setdefault(x, []).append((t, how))
    flags = [4 if t in unchecked else 0 for t in range(len(rows))]
    for x, acc in touched.items():
        for t, how in acc:
            for u, how_u in acc:
                if u == t or streams[u] == streams[t] or epochs[u] != epochs[t]:
                    continue
                if how == "w":
                    flags[t] |= 2
                elif how_u == "w":
                    flags[t] |= 1
    return flags


def pointer_checks(allocs, ptrs):
    """(flags, base, avail) of each pointer by address sets: the allocation
    whose byte set holds p, else the one whose byte set holds p - 1 and ends at
    p; allocs maps base -> size (see oracle.c for the reading)."""
    owner = {}
    for b, z in allocs.items():
        for x in range(b, b + z):
            owner[x] = b
    out = []
    for p in ptrs:
        if p in owner:
            b = owner[p]
        elif p - 1 in owner and owner[p - 1] + allocs[owner[p - 1]] == p:
            b = owner[p - 1]
        else:
            out.append((1, 0, 0))
            continue
        out.append((0, b, b + allocs[b] - p))
    return out
