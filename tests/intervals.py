"""Interval-arithmetic evaluation of expected verdicts, straight from a
workload's sparse description (runs of undefined bytes, A holes, allocation
bounds), with no byte loop.

It is a second route to the same result as the byte-by-byte oracle and is
used in two ways: on small configurations it must agree with the oracle
record for record (so a slip in either one shows), and on full-size
configurations, where a byte loop is too slow, it checks every verdict the
GPU produces.  Only used by tests.

Covers workloads whose V background is a constant (configurations 1-3);
configuration 4's periodic pattern has its own closed form in the tests.
"""
from __future__ import annotations

import numpy as np

NONE = np.uint64(0xFFFF_FFFF_FFFF_FFFF)
SRC_UNADDR, SRC_UNDEF, SRC_UNALLOC, SRC_OVERRUN = 1, 2, 4, 8
DST_UNADDR, DST_UNALLOC, DST_OVERRUN, OVERLAP, BAD_KIND = 16, 32, 64, 128, 256


def merge(a, b):
    """Union of intervals [a, b) as sorted disjoint arrays."""
    a = np.asarray(a, np.int64); b = np.asarray(b, np.int64)
    keep = b > a
    a, b = a[keep], b[keep]
    if a.size == 0:
        return a, b
    o = np.argsort(a, kind="stable")
    a, b = a[o], b[o]
    run_max = np.maximum.accumulate(b)
    start_new = np.ones(a.size, bool)
    start_new[1:] = a[1:] > run_max[:-1]
    grp = np.cumsum(start_new) - 1
    na = a[start_new]
    nb = np.zeros(na.size, np.int64)
    np.maximum.at(nb, grp, b)
    return na, nb


def subtract(a, b, ha, hb):
    """[a,b) minus [ha,hb), all sorted disjoint."""
    if ha.size == 0 or a.size == 0:
        return a.copy(), b.copy()
    pts = []
    # sweep: build complement of holes then intersect
    ca = np.concatenate([[np.iinfo(np.int64).min // 2], hb])
    cb = np.concatenate([ha, [np.iinfo(np.int64).max // 2]])
    return intersect(a, b, ca, cb)


def intersect(a, b, c, d):
    """Intersection of two sorted disjoint interval sets."""
    i = j = 0
    oa, ob = [], []
    while i < a.size and j < c.size:
        lo, hi = max(a[i], c[j]), min(b[i], d[j])
        if lo < hi:
            oa.append(lo); ob.append(hi)
        if b[i] < d[j]:
            i += 1
        else:
            j += 1
    return np.array(oa, np.int64), np.array(ob, np.int64)


class IntervalSet:
    """Sorted disjoint intervals with vectorised measure / first-point queries."""

    def __init__(self, a, b):
        self.a, self.b = merge(a, b)
        self.cum = np.concatenate([[0], np.cumsum(self.b - self.a)])

    def measure_below(self, x):
        x = np.asarray(x, np.int64)
        j = np.searchsorted(self.a, x, side="left")      # intervals starting before x
        full = self.cum[j]
        last = np.where(j > 0, np.maximum(self.b[np.maximum(j - 1, 0)] - x, 0), 0) if self.a.size else 0
        return full - last

    def measure(self, lo, hi):
        return np.where(np.asarray(hi) > np.asarray(lo), self.measure_below(hi) - self.measure_below(lo), 0)

    def first_at_or_after(self, x, hi):
        """First point p >= x of the set with p < hi, else -1."""
        x = np.asarray(x, np.int64); hi = np.asarray(hi, np.int64)
        if self.a.size == 0:
            return np.full(x.shape, -1, np.int64)
        j = np.searchsorted(self.b, x, side="right")     # first interval with b > x
        jj = np.minimum(j, self.a.size - 1)
        p = np.maximum(x, self.a[jj])
        ok = (j < self.a.size) & (p < hi)
        return np.where(ok, p, -1)


def expected(w, records=None):
    """Expected verdict fields (flags, first_bad, undef, avail) as numpy arrays."""
    host, dev = w.host, w.dev
    rec = w.records if records is None else records
    assert np.asarray(host.pattern).size == 1
    hb, hl = int(host.base), int(host.length)
    kind = rec["kind"].astype(np.int64)
    src = rec["src"].astype(np.int64)
    dst = rec["dst"].astype(np.int64)
    n = rec["n"].astype(np.int64)
    T = n.size

    # host undefined set (region offsets) and holes
    bg = int(np.asarray(host.pattern)[0])
    if bg:
        hu_a, hu_b = np.array([0]), np.array([hl])
    else:
        r = np.asarray(host.runs, np.int64).reshape(-1, 3)
        p = np.asarray(host.points, np.int64).reshape(-1, 2)
        r = r[r[:, 2] != 0]; p = p[p[:, 1] != 0]
        hu_a = np.concatenate([r[:, 0], p[:, 0]]); hu_b = np.concatenate([r[:, 0] + r[:, 1], p[:, 0] + 1])
    holes = np.asarray(host.holes, np.int64).reshape(-1, 2)
    H = IntervalSet(holes[:, 0], holes[:, 0] + holes[:, 1])
    HU = IntervalSet(hu_a, hu_b)
    HUa, HUb = subtract(HU.a, HU.b, H.a, H.b)
    D_host = IntervalSet(HUa, HUb)              # undefined and addressable

    # device: live allocations sorted, undefined set in absolute addresses
    live = dev.live_idx
    lb = dev.base[live].astype(np.int64); ls = dev.size[live].astype(np.int64)
    o = np.argsort(lb); lb, ls = lb[o], ls[o]
    li = live[o]
    ua, ub = [], []
    init_ff = dev.init[li] != 0
    ua.append(lb[init_ff]); ub.append(lb[init_ff] + ls[init_ff])
    rr = np.asarray(dev.runs, np.int64).reshape(-1, 4)
    rr = rr[(rr[:, 3] != 0) & dev.live[rr[:, 0]]]
    ua.append(dev.base[rr[:, 0]].astype(np.int64) + rr[:, 1])
    ub.append(dev.base[rr[:, 0]].astype(np.int64) + rr[:, 1] + rr[:, 2])
    D_dev = IntervalSet(np.concatenate(ua), np.concatenate(ub))

    def lookup(p):
        j = np.searchsorted(lb, p, side="right") - 1
        jj = np.maximum(j, 0)
        inside = (j >= 0) & (p < lb[jj] + ls[jj])
        avail = np.where(inside, lb[jj] + ls[jj] - p, 0)
        return inside, avail

    def region_clip(p):
        off = p - hb
        lo = np.clip(-off, 0, n)
        hi = np.clip(hl - off, 0, n)
        hi = np.maximum(hi, lo)
        return off, lo, hi

    flags = np.zeros(T, np.int64)
    big = np.int64(1) << 62
    first = np.full(T, big, np.int64)
    undef = np.zeros(T, np.int64)
    avail = np.zeros(T, np.int64)

    # --- source side
    hs = kind == 0
    off, lo, hi = region_clip(src)
    unaddr_first = np.where(lo > 0, 0, np.where(hi < n, hi, big))
    hole_first = H.first_at_or_after(off + lo, off + hi)
    hole_first = np.where(hole_first >= 0, hole_first - off, big)
    f_un = np.minimum(unaddr_first, hole_first)
    und_h = D_host.measure(off + lo, off + hi)
    fu_h = D_host.first_at_or_after(off + lo, off + hi)
    fu_h = np.where(fu_h >= 0, fu_h - off, big)
    flags |= np.where(hs & (f_un < big), SRC_UNADDR, 0)
    first = np.where(hs, np.minimum(first, np.minimum(f_un, fu_h)), first)
    undef = np.where(hs, und_h, undef)

    ds = ~hs
    ins, av_s = lookup(src)
    lim = np.minimum(n, av_s)
    und_d = D_dev.measure(src, src + lim)
    fu_d = D_dev.first_at_or_after(src, src + lim)
    fu_d = np.where(fu_d >= 0, fu_d - src, big)
    flags |= np.where(ds & ~ins, SRC_UNALLOC, 0)
    flags |= np.where(ds & ins & (n > av_s), SRC_OVERRUN, 0)
    first = np.where(ds, np.minimum(first, np.minimum(np.where(av_s < n, av_s, big), fu_d)), first)
    undef = np.where(ds, und_d, undef)

    # --- destination side
    hd = kind == 1
    offd, lod, hid = region_clip(dst)
    unaddr_d = np.where(lod > 0, 0, np.where(hid < n, hid, big))
    hole_d = H.first_at_or_after(offd + lod, offd + hid)
    hole_d = np.where(hole_d >= 0, hole_d - offd, big)
    f_und = np.minimum(unaddr_d, hole_d)
    flags |= np.where(hd & (f_und < big), DST_UNADDR, 0)
    first = np.where(hd, np.minimum(first, f_und), first)
    dd = ~hd
    insd, av_d = lookup(dst)
    flags |= np.where(dd & ~insd, DST_UNALLOC, 0)
    flags |= np.where(dd & insd & (n > av_d), DST_OVERRUN, 0)
    first = np.where(dd, np.minimum(first, np.where(av_d < n, av_d, big)), first)

    flags |= np.where(undef > 0, SRC_UNDEF, 0)
    d2d = kind == 2
    ov = d2d & (src < dst + n) & (dst < src + n)
    flags |= np.where(ov, OVERLAP, 0)
    avail = np.where(kind == 0, av_d, np.where(kind == 1, av_s, np.minimum(av_s, av_d)))

    bad_kind = (kind < 0) | (kind > 2)
    zero = n == 0
    flags = np.where(bad_kind, BAD_KIND, np.where(zero, 0, flags))
    undef = np.where(bad_kind | zero, 0, undef)
    avail = np.where(bad_kind | zero, 0, avail)
    fb = np.where(first >= big, NONE, first.astype(np.uint64))
    fb = np.where(bad_kind | zero, NONE, fb)
    return flags.astype(np.uint32), fb.astype(np.uint64), undef.astype(np.uint64), avail.astype(np.uint64)


def piece_closed_form(w, stage):
    """Undefined bytes and first undefined offset of each piece [a, b) of the
    2 GiB region (pieces cut at the same offsets in every stage): the padding
    bytes 13..15 of every 16-byte record, plus the one payload byte of each
    payload record, counted by arithmetic rather than by a byte loop."""
    a = (stage["src"] - stage["src"][0]).astype(np.int64)
    b = a + stage["n"].astype(np.int64)
    pad = lambda x: 3 * (x // 16) + np.maximum(0, x % 16 - 13)     # padding bytes in [0, x)
    pos = np.sort(16 * np.asarray(w.payload_records, np.int64) + np.asarray(w.payload_byte, np.int64))
    lo, hi = np.searchsorted(pos, a), np.searchsorted(pos, b)
    und = (pad(b) - pad(a) + (hi - lo)).astype(np.uint64)
    first_pad = np.where(a % 16 <= 13, 13 - a % 16, 0)
    first_pay = np.where(hi > lo, pos[np.minimum(lo, pos.size - 1)] - a, np.iinfo(np.int64).max)
    first = np.minimum(first_pad, first_pay)
    first = np.where(first < b - a, first, -1).astype(np.int64).astype(np.uint64)   # -1: none (~0)
    return und, first
