"""Shared helpers of the test suite (no GPU needed to import)."""
from __future__ import annotations

import numpy as np

from oracle.oracle import OracleState
from paper_1310_0901_amd import workloads as W

FIELDS = ("flags", "first_bad", "undef_bytes", "avail")


def oracle_for(w, host_arrays=None):
    dev = w.dev
    live = dev.live_idx
    hv, ha = host_arrays if host_arrays is not None else (W.host_v(w.host), W.host_a(w.host))
    return OracleState(w.host.base, w.host.length, hv.copy(), ha, dev.base[live], dev.size[live],
                       [W.alloc_v(dev, j) for j in live])


def assert_verdicts_equal(got, want, what=""):
    assert got.shape == want.shape, what
    for f in FIELDS:
        bad = np.flatnonzero(got[f] != want[f])
        if bad.size:
            i = int(bad[0])
            raise AssertionError(
                f"{what}: field {f} differs at {bad.size} records; first record {i}: "
                f"got {tuple(int(got[x][i]) for x in FIELDS)} want {tuple(int(want[x][i]) for x in FIELDS)}")


def workload_from_arrays(hb, hv, a_bits, bases, sizes, vs, records, live=None):
    """A Workload holding explicit small arrays (tiny universes, random worlds)."""
    hv = np.asarray(hv, np.uint8)
    a_bits = np.asarray(a_bits, np.uint8)
    nzv = np.flatnonzero(hv)
    points = np.stack([nzv, hv[nzv].astype(np.int64)], 1) if nzv.size else np.zeros((0, 2), np.int64)
    z = np.flatnonzero(a_bits == 0)
    holes = np.stack([z, np.ones(z.size, np.int64)], 1) if z.size else np.zeros((0, 2), np.int64)
    host = W.HostSpec(int(hb), int(hv.size), points=points.astype(np.int64), holes=holes.astype(np.int64))
    bases = np.asarray(bases, np.uint64)
    sizes = np.asarray(sizes, np.uint64)
    live = np.ones(bases.size, bool) if live is None else np.asarray(live, bool)
    runs = []
    for j, v in enumerate(vs):
        v = np.asarray(v, np.uint8)
        for x in np.flatnonzero(v):
            runs.append((j, int(x), 1, int(v[x])))
    dev = W.DeviceSpec(bases, sizes, live, np.zeros(bases.size, np.uint8),
                       np.array(runs, np.int64).reshape(-1, 4))
    return W.Workload("arrays", host, dev, np.ascontiguousarray(records, W.RECORD_DTYPE),
                      np.zeros(len(records), np.int64))


def random_world(rng, hl=None, nalloc=None, max_size=None, dens=None):
    """Random host region and allocations (ascending, with gaps and adjacency)."""
    hl = hl or int(rng.integers(1000, 300_000))
    nalloc = nalloc or int(rng.integers(1, 12))
    max_size = max_size or int(rng.choice([100, 5000, 200_000]))
    dens = dens if dens is not None else float(rng.choice([0.0, 1e-4, 0.01, 0.3]))
    hv = np.where(rng.random(hl) < dens, rng.integers(1, 256, hl), 0).astype(np.uint8)
    a = (rng.random(hl) > float(rng.choice([0.0, 1e-4, 0.01]))).astype(np.uint8)
    sizes = rng.integers(1, max_size, size=nalloc)
    gaps = rng.integers(0, 2, size=nalloc) * rng.integers(1, 300, size=nalloc)
    bases = W.DEV_BASE + np.cumsum(np.concatenate([[0], sizes[:-1]])) + np.cumsum(gaps) + int(rng.integers(0, 16))
    vs = [np.where(rng.random(int(s)) < dens, rng.integers(1, 256, int(s)), 0).astype(np.uint8) for s in sizes]
    return hl, hv, a, bases.astype(np.uint64), sizes.astype(np.uint64), vs


def random_records(rng, hb, hl, bases, sizes, count, max_n=None, kinds=(0, 1, 2)):
    rows = []
    for _ in range(count):
        kind = int(rng.choice(kinds))
        n = int(rng.integers(0, max_n or 60_000))

        def hostp():
            if rng.random() < 0.1:
                return hb + int(rng.integers(-n - 50, hl + 50))
            return hb + int(rng.integers(0, max(1, hl - n + 1)))

        def devp():
            j = int(rng.integers(0, bases.size))
            if rng.random() < 0.1:
                return int(bases[j]) + int(rng.integers(-20, int(sizes[j]) + 20))
            return int(bases[j]) + int(rng.integers(0, max(1, int(sizes[j]) - n + 1)))
        s = hostp() if kind == 0 else devp()
        d = hostp() if kind == 1 else devp()
        rows.append((s, d, n, kind, 0))
    return np.array(rows, W.RECORD_DTYPE)


def shadow_intervals(rec, hb, hl, bases, sizes):
    """Shadow byte intervals a record reads and writes, in a unified space
    (host region offsets below 2^62, allocation j at (j+1) << 48)."""
    src, dst, n, kind = int(rec["src"]), int(rec["dst"]), int(rec["n"]), int(rec["kind"])

    def host_iv(p):
        lo, hi = max(p, hb), min(p + n, hb + hl)
        return (lo - hb, hi - hb) if hi > lo else None

    def dev_iv(p):
        for j, (b, s) in enumerate(zip(bases, sizes)):
            b, s = int(b), int(s)
            if b <= p < b + s:
                return ((j + 1) << 48) + p - b, ((j + 1) << 48) + p - b + min(n, b + s - p)
        return None
    if kind > 2 or n == 0:
        return None, None
    r = host_iv(src) if kind == 0 else dev_iv(src)
    w = host_iv(dst) if kind == 1 else dev_iv(dst)
    if kind == 2 and (src < dst + n and dst < src + n):
        w = None
    return r, w


def conflict_free(recs, hb, hl, bases, sizes):
    """Greedy subset of records whose written shadow meets no other record's shadow."""
    keep, reads, writes = [], [], []

    def meets(iv, lst):
        return iv is not None and any(iv[0] < b and a < iv[1] for a, b in lst)
    for i in range(len(recs)):
        r, w = shadow_intervals(recs[i], hb, hl, bases, sizes)
        if meets(w, reads) or meets(w, writes) or meets(r, writes):
            continue
        if w is not None and r is not None and w[0] < r[1] and r[0] < w[1]:
            continue
        keep.append(i)
        if r is not None:
            reads.append(r)
        if w is not None:
            writes.append(w)
    return recs[keep]


def oracle_subset(w, records, hv, ha):
    """Oracle state holding only the live allocations that the device pointers
    of `records` lie in (a verdict depends only on the allocation holding the
    pointer), for full-size workloads whose whole device shadow is too large."""
    live = w.dev.live_idx
    lb = w.dev.base[live].astype(np.int64)
    ls = w.dev.size[live].astype(np.int64)
    ptrs = np.concatenate([records["src"][records["kind"] != 0],
                           records["dst"][records["kind"] != 1]]).astype(np.int64)
    j = np.searchsorted(lb, ptrs, side="right") - 1
    inside = (j >= 0) & (ptrs < lb[np.maximum(j, 0)] + ls[np.maximum(j, 0)])
    idx = np.unique(live[j[inside]])
    return OracleState(w.host.base, w.host.length, hv, ha, w.dev.base[idx], w.dev.size[idx],
                       [W.alloc_v(w.dev, int(x)) for x in idx])
