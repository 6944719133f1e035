"""Seeded synthetic workloads for the transfer checker.

This module only *describes* inputs: a host region (its V bytes and A
bitmap), a set of device allocations with their initial shadow contents, and
a list of transfer records with the labels the generator injected.  It holds
none of the checking arithmetic.  Both the CPU oracle (through the numpy
materialisers below) and the GPU path (through the library's own
allocation / shadow-set calls plus a plain upload of the host arrays) build
their state from the same description.

Shapes follow the workloads of the method: host-to-device, device-to-host and
device-to-device copies (Summary, Sec. 5), checked against a per-context list
of linear device allocations (Sec. 2, Fig. 2 caption) and against host
addressability / definedness shadow with one V byte per data byte where a set
bit means "undefined" and one A bit per byte where 1 means "addressable"
(Sec. 1.1).  Sizes, densities and mixes are those of the five benchmark
configurations; where those are silent the reading is stated next to the code.

Conventions
-----------
* A bitmap: the byte at region offset x is bit (x & 63) of little-endian u64
  word x >> 6.
* Record kinds: 0 = host->device, 1 = device->host, 2 = device->device.
* Labels: 0 clean, 1 overrun injected, 2 use-after-free injected.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

HOST_BASE = 0x7F00_0000_0000
DEV_BASE = 0x7000_0000_0000
KIND_H2D, KIND_D2H, KIND_D2D = 0, 1, 2
SEED0 = 13100900
KiB, MiB, GiB = 1 << 10, 1 << 20, 1 << 30

LABEL_CLEAN, LABEL_OVERRUN, LABEL_UAF = 0, 1, 2

# numpy layout of one transfer record and one verdict (32 bytes each)
RECORD_DTYPE = np.dtype([("src", "<u8"), ("dst", "<u8"), ("n", "<u8"),
                         ("kind", "<u4"), ("reserved", "<u4")])
VERDICT_DTYPE = np.dtype([("flags", "<u4"), ("reserved", "<u4"),
                          ("first_bad", "<u8"), ("undef_bytes", "<u8"),
                          ("avail", "<u8")])
# serving event log entry (48 bytes) and per-request result (72 bytes)
EV_CHECK, EV_ALLOC, EV_FREE = 0, 1, 2
# one pitched 2D copy (cg_transfer2d)
RECORD2D_DTYPE = np.dtype([("src", "<u8"), ("dst", "<u8"), ("width", "<u8"), ("rows", "<u8"), ("spitch", "<u8"),
                           ("dpitch", "<u8"), ("kind", "<u4"), ("reserved", "<u4", (3,))])
# one result of the pointer check (cg_ptr_check)
PTR_DTYPE = np.dtype([("flags", "<u4"), ("reserved", "<u4"), ("base", "<u8"), ("avail", "<u8")])
# one result of the concurrent-access join (cg_race)
RACE_DTYPE = np.dtype([("flags", "<u4"), ("reserved", "<u4"), ("partner", "<u8")])
SERVE_EVENT_DTYPE = np.dtype([("t", "<f8"), ("type", "<u4"), ("reserved", "<u4"),
                              ("src", "<u8"), ("dst", "<u8"), ("n", "<u8"), ("kind", "<u4"), ("rsv", "<u4")])
SERVE_RESULT_DTYPE = np.dtype([("flags", "<u4"), ("reserved", "<u4"), ("first_bad", "<u8"),
                               ("undef_bytes", "<u8"), ("avail", "<u8"), ("t_arrive", "<f8"),
                               ("t_admit", "<f8"), ("t_done", "<f8"), ("epoch", "<u8"),
                               ("batch", "<u4"), ("slot", "<u4")])


@dataclass
class HostSpec:
    """Host region [base, base+length) with its V bytes and A bitmap.

    V = tile(pattern) then runs (start, len, value) then points (index, value);
    A = all ones except holes (start, len).
    """
    base: int
    length: int
    pattern: np.ndarray = field(default_factory=lambda: np.zeros(1, np.uint8))
    runs: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), np.int64))
    points: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int64))
    holes: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int64))


@dataclass
class DeviceSpec:
    """Device allocations (ascending base); only `live` ones are registered.

    A live allocation's shadow starts at `init[j]` (0xFF = nothing defined
    yet, 0 = fully written), then runs (alloc, offset, len, value) are set.
    """
    base: np.ndarray
    size: np.ndarray
    live: np.ndarray
    init: np.ndarray
    runs: np.ndarray = field(default_factory=lambda: np.zeros((0, 4), np.int64))

    @property
    def live_idx(self) -> np.ndarray:
        return np.flatnonzero(self.live)

    @property
    def freed_idx(self) -> np.ndarray:
        return np.flatnonzero(~self.live)


@dataclass
class Workload:
    name: str
    host: HostSpec
    dev: DeviceSpec
    records: np.ndarray            # RECORD_DTYPE
    label: np.ndarray              # per record
    propagate: bool = False
    stages: list = field(default_factory=list)  # extra record batches (chains)
    note: str = ""

    @property
    def count(self) -> int:
        return int(self.records.shape[0])


# ---------------------------------------------------------------------------
# materialisers (plain data construction, used by the oracle side and for the
# upload of the host region to device memory)
# ---------------------------------------------------------------------------

def host_v(spec: HostSpec) -> np.ndarray:
    p = np.asarray(spec.pattern, np.uint8)
    if p.size == 1:
        v = np.full(spec.length, p[0], np.uint8) if p[0] else np.zeros(spec.length, np.uint8)
    else:
        reps = -(-spec.length // p.size)
        v = np.tile(p, reps)[: spec.length].copy()
    for s, ln, val in np.asarray(spec.runs, np.int64).reshape(-1, 3):
        v[s:s + ln] = val
    pts = np.asarray(spec.points, np.int64).reshape(-1, 2)
    if pts.shape[0]:
        v[pts[:, 0]] = pts[:, 1].astype(np.uint8)
    return v


def host_a(spec: HostSpec) -> np.ndarray:
    """A bitmap as little-endian u64 words (padded with zero bits)."""
    nwords = -(-spec.length // 64)
    a = np.full(nwords, np.uint64(0xFFFF_FFFF_FFFF_FFFF), np.uint64)
    tail = spec.length & 63
    if tail:
        a[-1] = np.uint64((1 << tail) - 1)
    full = np.uint64(0xFFFF_FFFF_FFFF_FFFF)
    for s, ln in np.asarray(spec.holes, np.int64).reshape(-1, 2):
        e = min(int(s + ln), spec.length)
        s = int(s)
        while s < e:
            w, b = s >> 6, s & 63
            take = min(64 - b, e - s)
            m = full if take == 64 else np.uint64(((1 << take) - 1) << b)
            if take == 64 and b == 0:
                # clear whole words in one slice
                wend = e >> 6
                a[w:wend] = 0
                s = wend << 6
                continue
            a[w] &= ~m
            s += take
    return a


def alloc_v(dev: DeviceSpec, j: int) -> np.ndarray:
    v = np.full(int(dev.size[j]), np.uint8(dev.init[j]), np.uint8)
    r = np.asarray(dev.runs, np.int64).reshape(-1, 4)
    for _, off, ln, val in r[r[:, 0] == j]:
        v[off:off + ln] = val
    return v


def make_records(kind, src, dst, n) -> np.ndarray:
    r = np.zeros(len(n), RECORD_DTYPE)
    r["src"], r["dst"], r["n"], r["kind"] = src, dst, n, kind
    return r


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def _round_up(x, a):
    return (x + a - 1) // a * a


def place_allocations(rng, sizes, align=256, gap_units=16) -> np.ndarray:
    """Ascending bases: each base = round_up(prev_end, align) + align*U{0..gap_units}."""
    sizes = np.asarray(sizes, np.int64)
    gaps = rng.integers(0, gap_units + 1, size=sizes.size) * align
    bases = np.empty(sizes.size, np.int64)
    cur = 0
    for j in range(sizes.size):
        cur = _round_up(cur, align) + int(gaps[j])
        bases[j] = cur
        cur += int(sizes[j])
    return (bases + DEV_BASE).astype(np.uint64)


def log_uniform_int(rng, lo, hi, size) -> np.ndarray:
    """floor(exp(U(ln lo, ln hi))), as int64 in [lo, hi)."""
    x = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))).astype(np.int64)
    return np.clip(x, lo, hi - 1)


def zipf_weights(m, s):
    w = np.arange(1, m + 1, dtype=np.float64) ** (-s)
    return w / w.sum()


class ConditionalZipf:
    """Draw an allocation by Zipf(s) rank over a seeded permutation, conditioned
    on its size being >= a required length.

    This is the same law as re-drawing until the size fits, computed directly
    by restricting the cumulative Zipf mass to the allocations that fit."""

    def __init__(self, rng, sizes, s):
        m = sizes.size
        perm = rng.permutation(m)           # rank r -> allocation perm[r]
        w = np.empty(m)
        w[perm] = zipf_weights(m, s)        # weight of each allocation
        order = np.argsort(-sizes, kind="stable")   # largest first
        self.order = order
        self.sorted_sizes_desc = sizes[order]
        self.cum = np.cumsum(w[order])

    def draw(self, rng, need) -> np.ndarray:
        need = np.asarray(need, np.int64)
        # number of allocations with size >= need (prefix of the descending order)
        m = np.searchsorted(-self.sorted_sizes_desc, -need, side="right")
        if np.any(m == 0):
            raise ValueError("no allocation large enough")
        u = rng.uniform(0.0, 1.0, size=need.size) * self.cum[m - 1]
        k = np.minimum(np.searchsorted(self.cum, u, side="right"), m - 1)
        return self.order[k]


def _sparse_runs(rng, total, density, max_len=64):
    """Undefined runs at a byte density: count = round(density*total/mean_len),
    run length U{1..max_len}."""
    mean_len = (1 + max_len) / 2.0
    cnt = int(round(density * total / mean_len))
    lens = rng.integers(1, max_len + 1, size=cnt)
    return cnt, lens


# ---------------------------------------------------------------------------
# configuration 1: plain, tiny
# ---------------------------------------------------------------------------

def config1(seed=SEED0 + 1, n_transfers=64, host_len=1 * MiB, n_alloc=20,
            n_freed=4, max_n=64 * KiB) -> Workload:
    rng = np.random.default_rng(seed)
    hl = host_len
    n_undef = int(round(1e-4 * hl))
    pos = rng.choice(hl, size=n_undef, replace=False)
    host = HostSpec(HOST_BASE, hl,
                    points=np.stack([np.sort(pos), np.full(n_undef, 0xFF)], 1).astype(np.int64))
    sizes = rng.integers(4 * KiB, 256 * KiB + 1, size=n_alloc)
    bases = place_allocations(rng, sizes)
    live = np.ones(n_alloc, bool)
    live[rng.choice(n_alloc, size=n_freed, replace=False)] = False
    dev = DeviceSpec(bases, sizes.astype(np.uint64), live, np.full(n_alloc, 0xFF, np.uint8))

    T = n_transfers
    n_over, n_uaf = int(round(0.10 * T)), int(round(0.05 * T))
    cls = np.zeros(T, np.int64)
    p = rng.permutation(T)
    cls[p[:n_over]] = LABEL_OVERRUN
    cls[p[n_over:n_over + n_uaf]] = LABEL_UAF
    liv, fre = dev.live_idx, dev.freed_idx
    src = np.zeros(T, np.uint64); dst = np.zeros(T, np.uint64); n = np.zeros(T, np.uint64)
    for t in range(T):
        if cls[t] == LABEL_OVERRUN:
            d = int(rng.integers(1, 65))
            nn = int(rng.integers(d + 1, max_n + 1))
            cand = liv[sizes[liv] >= nn - d]
            j = int(rng.choice(cand))
            o = int(sizes[j]) - (nn - d)
        elif cls[t] == LABEL_UAF:
            nn = int(rng.integers(1, max_n + 1))
            cand = fre[sizes[fre] >= nn]
            j = int(rng.choice(cand if cand.size else fre))
            o = int(rng.integers(0, max(int(sizes[j]) - nn, 0) + 1))
        else:
            nn = int(rng.integers(1, max_n + 1))
            cand = liv[sizes[liv] >= nn]
            j = int(rng.choice(cand))
            o = int(rng.integers(0, int(sizes[j]) - nn + 1))
        n[t] = nn
        dst[t] = int(bases[j]) + o
        src[t] = HOST_BASE + int(rng.integers(0, hl - nn + 1))
    rec = make_records(np.full(T, KIND_H2D), src, dst, n)
    return Workload("plain-tiny", host, dev, rec, cls,
                    note="64 H2D over a 1 MiB host region, 16 live allocations")


# ---------------------------------------------------------------------------
# configuration 2: plain at scale
# ---------------------------------------------------------------------------

def config2(seed=SEED0 + 2, host_len=4 * GiB, n_alloc=4096, min_size=256,
            max_size=64 * MiB, density=1e-6, hole_p=1e-5) -> Workload:
    rng = np.random.default_rng(seed)
    hl = host_len
    cnt, lens = _sparse_runs(rng, hl, density)
    starts = rng.integers(0, hl - lens + 1)
    runs = np.stack([starts, lens, np.full(cnt, 0xFF)], 1).astype(np.int64)
    npages = hl // 4096
    hole_pages = np.flatnonzero(rng.random(npages) < hole_p) if npages < (1 << 22) else \
        np.unique(rng.integers(0, npages, size=rng.binomial(npages, hole_p)))
    holes = np.stack([hole_pages * 4096, np.full(hole_pages.size, 4096)], 1).astype(np.int64)
    host = HostSpec(HOST_BASE, hl, runs=runs, holes=holes)
    sizes = log_uniform_int(rng, min_size, max_size, n_alloc)
    bases = place_allocations(rng, sizes)
    dev = DeviceSpec(bases, sizes.astype(np.uint64), np.ones(n_alloc, bool),
                     np.full(n_alloc, 0xFF, np.uint8))
    n = sizes.astype(np.uint64)
    src = (HOST_BASE + rng.integers(0, hl - sizes + 1)).astype(np.uint64)
    rec = make_records(np.full(n_alloc, KIND_H2D), src, bases, n)
    return Workload("plain-at-scale", host, dev, rec, np.zeros(n_alloc, np.int64),
                    note="one full-size H2D per allocation")


# ---------------------------------------------------------------------------
# configuration 3: batched, Zipf over live allocations, mixed kinds
# ---------------------------------------------------------------------------

def config3(seed=SEED0 + 3, n_transfers=1_000_000, n_alloc=65536,
            host_len=4 * GiB, min_size=8, max_size=16 * MiB,
            zipf_s=1.1, p_over=0.02, p_uaf=0.01, density=1e-6,
            hole_p=1e-5, freed_frac=0.01) -> Workload:
    rng = np.random.default_rng(seed)
    hl = host_len
    # host region as in configuration 2
    cnt, lens = _sparse_runs(rng, hl, density)
    starts = rng.integers(0, hl - lens + 1)
    runs = np.stack([starts, lens, np.full(cnt, 0xFF)], 1).astype(np.int64)
    npages = hl // 4096
    nh = rng.binomial(npages, hole_p)
    hole_pages = np.unique(rng.integers(0, npages, size=nh))
    holes = np.stack([hole_pages * 4096, np.full(hole_pages.size, 4096)], 1).astype(np.int64)
    host = HostSpec(HOST_BASE, hl, runs=runs, holes=holes)

    # device: live + freed allocations, interleaved in address order
    n_freed = max(1, int(round(freed_frac * n_alloc)))
    n_all = n_alloc + n_freed
    sizes_all = log_uniform_int(rng, min_size, max_size, n_all)
    bases = place_allocations(rng, sizes_all)
    live = np.ones(n_all, bool)
    live[rng.choice(n_all, size=n_freed, replace=False)] = False
    init = np.zeros(n_all, np.uint8)           # device data written (defined)
    liv = np.flatnonzero(live)
    fre = np.flatnonzero(~live)
    live_sizes = sizes_all[liv]
    # undefined runs over the concatenated live shadow, at the byte density
    tot = int(live_sizes.sum())
    rcnt, rlens = _sparse_runs(rng, tot, density)
    which = rng.choice(liv.size, size=rcnt, p=live_sizes / tot)
    rl = np.minimum(rlens, live_sizes[which])
    roff = (rng.random(rcnt) * (live_sizes[which] - rl + 1)).astype(np.int64)
    druns = np.stack([liv[which], roff, rl, np.full(rcnt, 0xFF)], 1).astype(np.int64)
    dev = DeviceSpec(bases, sizes_all.astype(np.uint64), live, init, druns)

    T = n_transfers
    kind = rng.choice(3, size=T, p=[0.6, 0.1, 0.3]).astype(np.int64)  # H2D, D2H, D2D
    n = log_uniform_int(rng, min_size, max_size, T)
    # transfers longer than the largest live allocation cannot be placed: redraw
    # (device->device needs two distinct allocations that fit: second largest)
    srt = np.sort(live_sizes)
    mx = np.where(kind == KIND_D2D, int(srt[-2]), int(srt[-1]))
    bad = n > mx
    while bad.any():
        n[bad] = log_uniform_int(rng, min_size, max_size, int(bad.sum()))
        bad = n > mx
    u = rng.random(T)
    label = np.where(u < p_over, LABEL_OVERRUN, np.where(u < p_over + p_uaf, LABEL_UAF, LABEL_CLEAN))
    delta = rng.integers(1, 65, size=T)
    # overruns need n > delta
    label[(label == LABEL_OVERRUN) & (n <= delta)] = LABEL_CLEAN

    cz = ConditionalZipf(rng, live_sizes, zipf_s)
    need = np.where(label == LABEL_OVERRUN, n - delta, n)
    # the "device side" that carries an injection: dst for H2D/D2D, src for D2H
    inj = liv[cz.draw(rng, need)]
    o_inj = np.where(label == LABEL_OVERRUN, sizes_all[inj] - (n - delta),
                     (rng.random(T) * (sizes_all[inj] - n + 1)).astype(np.int64))
    # use-after-free: into a freed allocation
    uaf = np.flatnonzero(label == LABEL_UAF)
    fj = fre[rng.integers(0, fre.size, size=uaf.size)]
    inj[uaf] = fj
    o_inj[uaf] = (rng.random(uaf.size) * np.maximum(sizes_all[fj] - n[uaf] + 1, 1)).astype(np.int64)
    side_inj = bases[inj].astype(np.int64) + o_inj

    # the other device side of D2D (a clean draw, different allocation)
    d2d = np.flatnonzero(kind == KIND_D2D)
    other = liv[cz.draw(rng, n[d2d])]
    same = other == inj[d2d]
    while same.any():
        other[same] = liv[cz.draw(rng, n[d2d][same])]
        same = other == inj[d2d]
    o_oth = (rng.random(d2d.size) * (sizes_all[other] - n[d2d] + 1)).astype(np.int64)
    host_off = (rng.random(T) * (hl - n + 1)).astype(np.int64)
    hostp = HOST_BASE + host_off

    src = np.where(kind == KIND_H2D, hostp, side_inj)
    dst = np.where(kind == KIND_D2H, hostp, side_inj)
    src[d2d] = bases[other].astype(np.int64) + o_oth
    rec = make_records(kind, src.astype(np.uint64), dst.astype(np.uint64), n.astype(np.uint64))
    return Workload("batched-1M", host, dev, rec, label,
                    note="Zipf(1.1) device sides, 60/30/10 H2D/D2D/D2H, 2% overrun, 1% UAF")


# ---------------------------------------------------------------------------
# configuration 4: partial definedness (16-byte records) plus propagation
# ---------------------------------------------------------------------------

def config4(seed=SEED0 + 4, host_len=2 * GiB, pieces=1, hops=4) -> Workload:
    rng = np.random.default_rng(seed)
    hl = host_len
    R = hl // 16
    pattern = np.array([0] * 13 + [0xFF] * 3, np.uint8)
    P = int(math.floor(0.01 * R))
    recs = np.sort(rng.choice(R, size=P, replace=False))
    b = rng.integers(0, 13, size=P)
    k = rng.integers(0, 8, size=P)
    points = np.stack([recs * 16 + b, (1 << k)], 1).astype(np.int64)
    host = HostSpec(HOST_BASE, hl, pattern=pattern, points=points)
    nA = hops + 1
    sizes = np.full(nA, hl, np.int64)
    bases = place_allocations(rng, sizes)
    dev = DeviceSpec(bases, sizes.astype(np.uint64), np.ones(nA, bool), np.full(nA, 0xFF, np.uint8))

    def cuts():
        if pieces == 1:
            return np.array([0, hl], np.int64)
        c = np.sort(rng.choice(np.arange(1, hl), size=pieces - 1, replace=False))
        return np.concatenate([[0], c, [hl]]).astype(np.int64)

    stages = []
    c = cuts()
    off, ln = c[:-1], np.diff(c)
    stages.append(make_records(np.full(off.size, KIND_H2D), (HOST_BASE + off).astype(np.uint64),
                               (bases[0].astype(np.int64) + off).astype(np.uint64), ln.astype(np.uint64)))
    for h in range(1, nA):
        c = cuts()
        off, ln = c[:-1], np.diff(c)
        stages.append(make_records(np.full(off.size, KIND_D2D),
                                   (int(bases[h - 1]) + off).astype(np.uint64),
                                   (int(bases[h]) + off).astype(np.uint64), ln.astype(np.uint64)))
    w = Workload("partial-definedness", host, dev, stages[0], np.zeros(stages[0].size, np.int64),
                 propagate=True, stages=stages,
                 note=f"{R} 16-byte records, 3 padding bytes each, {P} payload bits; H2D then {hops} D2D hops")
    w.R, w.P = R, P
    w.payload_records, w.payload_byte, w.payload_bit = recs, b, k
    return w


# ---------------------------------------------------------------------------
# configuration 5: serving -- Poisson requests interleaved with allocation events
# ---------------------------------------------------------------------------

def _mixture(rng, size, weights, comps):
    """Log-uniform sizes from a mixture of [lo, hi) components."""
    which = rng.choice(len(comps), size=size, p=weights)
    out = np.empty(size, np.int64)
    for k, (lo, hi) in enumerate(comps):
        m = which == k
        out[m] = log_uniform_int(rng, lo, hi, int(m.sum()))
    return out


REQ_COMPONENTS = [(64, 4 * KiB), (4 * KiB, 1 * MiB), (1 * MiB, 64 * MiB)]


@dataclass
class ServeWorkload:
    name: str
    host: HostSpec
    dev: DeviceSpec              # the initial state (live allocations at t = 0)
    events: np.ndarray           # SERVE_EVENT_DTYPE, ordered by t
    label: np.ndarray            # per check request
    rate: float
    note: str = ""

    @property
    def requests(self) -> np.ndarray:
        return self.events[self.events["type"] == EV_CHECK]


def config5(seed=SEED0 + 5, rate=50_000.0, duration=10.0, n_alloc=975_000, host_len=4 * GiB,
            event_ratio=10, p_over=0.02, p_uaf=0.01, p_new=0.1, zipf_s=1.1, density=1e-6,
            req_weights=(0.90, 0.09, 0.01), alloc_weights=(0.99, 0.009, 0.001)) -> ServeWorkload:
    """Poisson check requests at `rate` for `duration` seconds; one
    allocation or free event (p = 1/2 each) per `event_ratio` requests.

    Readings where the configuration is silent: request and allocation sizes
    are log-uniform within each mixture component; the initial allocations
    are fully written (V = 0) except sparse undefined runs at `density`;
    allocations made during the run are fresh (V = 0xFF) at new addresses;
    frees pick a live allocation uniformly; requests pick their device side
    by Zipf(1.1) over the initial allocations that fit (so a request may hit
    one freed before it arrives), or with probability p_new an allocation made
    during the run; kinds 60/30/10 H2D/D2D/D2H; 2 % overruns and 1 %
    pointers into freed allocations as in configuration 3."""
    rng = np.random.default_rng(seed)
    hl = host_len
    cnt, lens = _sparse_runs(rng, hl, density)
    starts = rng.integers(0, hl - lens + 1)
    host = HostSpec(HOST_BASE, hl, runs=np.stack([starts, lens, np.full(cnt, 0xFF)], 1).astype(np.int64))
    sizes0 = _mixture(rng, n_alloc, list(alloc_weights), REQ_COMPONENTS)
    bases0 = place_allocations(rng, sizes0).astype(np.int64)
    tot = int(sizes0.sum())
    rcnt, rlens = _sparse_runs(rng, tot, density)
    which = rng.choice(n_alloc, size=rcnt, p=sizes0 / tot)
    rl = np.minimum(rlens, sizes0[which])
    roff = (rng.random(rcnt) * (sizes0[which] - rl + 1)).astype(np.int64)
    dev = DeviceSpec(bases0.astype(np.uint64), sizes0.astype(np.uint64), np.ones(n_alloc, bool),
                     np.zeros(n_alloc, np.uint8),
                     np.stack([which, roff, rl, np.full(rcnt, 0xFF)], 1).astype(np.int64))

    # arrivals: one Poisson stream of requests and events
    total_rate = rate * (1 + 1 / event_ratio)
    n_arr = int(rng.poisson(total_rate * duration))
    t = np.sort(rng.uniform(0, duration, size=n_arr))
    is_ev = rng.random(n_arr) < (1 / (event_ratio + 1))
    ev_t = t[is_ev]
    rq_t = t[~is_ev]
    n_ev, n_rq = ev_t.size, rq_t.size

    # allocation events, simulated in order (frees pick a live allocation)
    ev_type = np.where(rng.random(n_ev) < 0.5, EV_ALLOC, EV_FREE)
    new_sizes = _mixture(rng, n_ev, list(alloc_weights), REQ_COMPONENTS)
    next_base = int(bases0[-1] + sizes0[-1]) + (1 << 20)
    live = list(range(n_alloc))           # ids into all_base / all_size
    pos = np.arange(n_alloc)              # id -> index in `live` (or -1)
    all_base = list(bases0)
    all_size = list(sizes0)
    ev_addr = np.zeros(n_ev, np.int64)
    ev_size = np.zeros(n_ev, np.int64)
    born = [0.0] * n_alloc                # creation time of every id
    died = [np.inf] * n_alloc
    pos = list(pos)
    pick = rng.random(n_ev)
    for k in range(n_ev):
        if ev_type[k] == EV_ALLOC or len(live) < 2:
            ev_type[k] = EV_ALLOC
            sz = int(new_sizes[k])
            i = len(all_base)
            all_base.append(next_base)
            all_size.append(sz)
            born.append(ev_t[k])
            died.append(np.inf)
            pos.append(len(live))
            live.append(i)
            ev_addr[k], ev_size[k] = next_base, sz
            next_base += (sz + 255) // 256 * 256 + 256
        else:
            j = int(pick[k] * len(live))
            i = live[j]
            last = live[-1]
            live[j] = last
            pos[last] = j
            live.pop()
            pos[i] = -1
            died[i] = ev_t[k]
            ev_addr[k] = all_base[i]
    all_base = np.array(all_base, np.int64)
    all_size = np.array(all_size, np.int64)
    born = np.array(born)
    died = np.array(died)

    # requests
    kind = rng.choice(3, size=n_rq, p=[0.6, 0.1, 0.3]).astype(np.int64)
    n = _mixture(rng, n_rq, list(req_weights), REQ_COMPONENTS)
    srt = np.sort(sizes0)
    mx = np.where(kind == KIND_D2D, int(srt[-2]), int(srt[-1]))
    bad = n > mx
    while bad.any():
        n[bad] = _mixture(rng, int(bad.sum()), list(req_weights), REQ_COMPONENTS)
        bad = n > mx
    u = rng.random(n_rq)
    label = np.where(u < p_over, LABEL_OVERRUN, np.where(u < p_over + p_uaf, LABEL_UAF, LABEL_CLEAN))
    delta = rng.integers(1, 65, size=n_rq)
    label[(label == LABEL_OVERRUN) & (n <= delta)] = LABEL_CLEAN
    cz = ConditionalZipf(rng, sizes0, zipf_s)
    need = np.where(label == LABEL_OVERRUN, n - delta, n)
    inj = cz.draw(rng, need)
    # requests to allocations made during the run (clipped to fit)
    n_new_before = np.searchsorted(born[n_alloc:], rq_t, side="right")
    to_new = (rng.random(n_rq) < p_new) & (n_new_before > 0) & (label == LABEL_CLEAN)
    ni = n_alloc + (rng.random(n_rq) * np.maximum(n_new_before, 1)).astype(np.int64)
    inj = np.where(to_new, ni, inj)
    n = np.where(to_new, np.minimum(n, all_size[inj]), n)
    L = all_size[inj]
    o_inj = np.where(label == LABEL_OVERRUN, L - (n - delta), (rng.random(n_rq) * (L - n + 1)).astype(np.int64))
    side_inj = all_base[inj] + o_inj
    # pointers into allocations freed before the request (else past the end)
    uaf = np.flatnonzero(label == LABEL_UAF)
    dead_t = np.where(np.isfinite(died), died, np.inf)
    order = np.argsort(dead_t)
    dead_sorted = dead_t[order]
    for r in uaf:
        k = int(np.searchsorted(dead_sorted, rq_t[r], side="left"))
        if k > 0:
            i = int(order[int(rng.integers(0, k))])
            side_inj[r] = all_base[i] + int(rng.integers(0, all_size[i]))
        else:
            side_inj[r] = next_base + int(rng.integers(0, 1 << 20))
    d2d = np.flatnonzero(kind == KIND_D2D)
    other = cz.draw(rng, n[d2d])
    same = other == inj[d2d]
    while same.any():
        other[same] = cz.draw(rng, n[d2d][same])
        same = other == inj[d2d]
    o_oth = (rng.random(d2d.size) * (sizes0[other] - n[d2d] + 1)).astype(np.int64)
    hostp = HOST_BASE + (rng.random(n_rq) * (hl - n + 1)).astype(np.int64)
    src = np.where(kind == KIND_H2D, hostp, side_inj)
    dst = np.where(kind == KIND_D2H, hostp, side_inj)
    src[d2d] = bases0[other] + o_oth

    events = np.zeros(n_arr, SERVE_EVENT_DTYPE)
    events["t"] = t
    ie = np.flatnonzero(is_ev)
    ir = np.flatnonzero(~is_ev)
    events["type"][ie] = ev_type
    events["dst"][ie] = ev_addr.astype(np.uint64)
    events["n"][ie] = ev_size.astype(np.uint64)
    events["type"][ir] = EV_CHECK
    events["src"][ir] = src.astype(np.uint64)
    events["dst"][ir] = dst.astype(np.uint64)
    events["n"][ir] = n.astype(np.uint64)
    events["kind"][ir] = kind
    return ServeWorkload("serving", host, dev, events, label, rate,
                         note=f"Poisson {rate:.0f} req/s for {duration:g} s, one alloc/free per "
                              f"{event_ratio} requests, {n_alloc} initial allocations")


def small_serve(seed=SEED0 + 5, duration=0.15) -> ServeWorkload:
    return config5(seed=seed, duration=duration, n_alloc=2000, host_len=64 * MiB, density=2e-4,
                   req_weights=(0.95, 0.048, 0.002), alloc_weights=(0.95, 0.045, 0.005))


# sizes used by the parity tests: several tiles and a ragged tail, oracle in seconds
def small_config(k: int) -> Workload:
    if k == 1:
        return config1()
    if k == 2:
        return config2(host_len=64 * MiB + 4093, n_alloc=96, max_size=2 * MiB,
                       density=2e-4, hole_p=2e-3)
    if k == 3:
        return config3(n_transfers=6000, n_alloc=2048, host_len=96 * MiB + 77,
                       max_size=1 * MiB, density=2e-5, hole_p=1e-3)
    if k == 4:
        return config4(host_len=4 * MiB, pieces=37, hops=4)
    raise ValueError(k)


def full_config(k: int) -> Workload:
    return {1: config1, 2: config2, 3: config3, 4: config4}[k]()


# ---- concurrent-access batches ------------------------------------------------

@dataclass
class RaceBatch:
    """Records with the stream each was issued on and its epoch (synchronising
    calls before it)."""
    records: np.ndarray      # RECORD_DTYPE
    streams: np.ndarray      # uint32
    epochs: np.ndarray       # uint32
    desc: str = ""


def race_from_records(records, seed=SEED0 + 6, streams=8, epoch_len=4096, desc="") -> RaceBatch:
    """A multi-stream program's copies: each record on one of `streams`
    streams (uniform), with a synchronisation after every `epoch_len` copies."""
    rng = np.random.default_rng(seed)
    T = records.size
    st = rng.integers(0, streams, size=T).astype(np.uint32)
    ep = (np.arange(T, dtype=np.int64) // epoch_len).astype(np.uint32)
    return RaceBatch(np.ascontiguousarray(records, RECORD_DTYPE), st, ep, desc)


def race_config(seed=SEED0 + 6, streams=8, epoch_len=4096) -> RaceBatch:
    """The 1,000,000 transfers of configuration 3 issued from `streams`
    streams, synchronised every `epoch_len` copies."""
    w = config3()
    return race_from_records(w.records, seed, streams, epoch_len,
                             f"race-1M: configuration 3's {w.records.size} transfers on {streams} streams, "
                             f"a synchronisation every {epoch_len} copies")


def small_race(seed=SEED0 + 7, count=20_000, window=1 << 16, streams=8, epochs=4,
               p_bad_kind=0.01, p_empty=0.02) -> RaceBatch:
    """Dense overlaps: records over a 64 KiB device window and a 64 KiB host
    window, log-uniform sizes 1..4096, a few bad kinds and empty records."""
    rng = np.random.default_rng(seed)
    kind = rng.choice(3, size=count, p=[0.4, 0.3, 0.3]).astype(np.int64)
    n = log_uniform_int(rng, 1, 4096, count)
    n[rng.random(count) < p_empty] = 0
    dev = lambda: DEV_BASE + rng.integers(0, window, size=count)
    host = HOST_BASE + rng.integers(0, window, size=count)
    d1, d2 = dev(), dev()
    src = np.where(kind == KIND_H2D, host, d1)
    dst = np.where(kind == KIND_D2H, host, np.where(kind == KIND_D2D, d2, d1))
    kind[rng.random(count) < p_bad_kind] = 3
    recs = make_records(kind, src, dst, n)
    st = rng.integers(0, streams, size=count).astype(np.uint32)
    ep = rng.integers(0, epochs, size=count).astype(np.uint32)
    return RaceBatch(recs, st, ep, f"small-race: {count} records, {streams} streams, {epochs} epochs")



# ---- kernel-argument pointers -------------------------------------------------

@dataclass
class PointerBatch:
    """Live allocations (sorted bases and sizes), allocations freed since, and
    pointers to look up among the live ones."""
    bases: np.ndarray
    sizes: np.ndarray
    freed: np.ndarray        # indices into bases/sizes of allocations to free before the lookup
    ptrs: np.ndarray
    desc: str = ""


def pointer_batch(seed=SEED0 + 8, n_alloc=975_000, n_ptrs=1_000_000, min_size=64, max_size=4096,
                  freed_frac=0.01) -> PointerBatch:
    """Kernel-argument pointers against a table the size of configuration 5's:
    a third each inside allocations (uniform offset), one past an allocation's
    end, and uniform over the whole address span (mostly in gaps); 1 % of the
    allocations are freed before the lookup."""
    rng = np.random.default_rng(seed)
    sizes = log_uniform_int(rng, min_size, max_size, n_alloc)
    bases = place_allocations(rng, sizes).astype(np.int64)
    freed = np.sort(rng.choice(n_alloc, size=int(freed_frac * n_alloc), replace=False))
    k = n_ptrs // 3
    j = rng.integers(0, n_alloc, size=k)
    inside = bases[j] + (rng.random(k) * sizes[j]).astype(np.int64)
    j2 = rng.integers(0, n_alloc, size=k)
    past = bases[j2] + sizes[j2]
    lo, hi = int(bases[0]) - 4096, int(bases[-1] + sizes[-1]) + 4096
    anywhere = rng.integers(lo, hi, size=n_ptrs - 2 * k)
    ptrs = rng.permutation(np.concatenate([inside, past, anywhere])).astype(np.uint64)
    return PointerBatch(bases.astype(np.uint64), sizes.astype(np.uint64), freed, ptrs,
                        f"pointers: {n_ptrs} lookups among {n_alloc - freed.size} live allocations")
