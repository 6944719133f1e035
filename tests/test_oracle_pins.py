"""Pins of the CPU oracle against things other than itself (no GPU).

* brute force: an independent set formulation, compared over every small case;
* the worked example printed in the paper (Sec. 4, Listings 2 and 6);
* the error classes of Sec. 2 reduced to closed-form verdicts;
* special cases that reduce to numpy / bisect routines;
* algebraic laws the definition implies (split, permutation, round trip,
  monotonicity) and snapshot == sequential replay under the no-conflict rule.
"""
import bisect
import itertools
import json
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

from oracle import brute
from oracle.oracle import (OracleState, REC, NONE, SRC_UNADDR, SRC_UNDEF, SRC_UNALLOC,
                           SRC_OVERRUN, DST_UNADDR, DST_UNALLOC, DST_OVERRUN, OVERLAP, BAD_KIND)
from tests.tiny import Tiny, recs, as_tuples, oracle_world, brute_world, bits_to_words

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# a tiny universe with every feature: A holes, V bytes with single bits,
# adjacent allocations, a gap, a freed range
# ---------------------------------------------------------------------------
HB = 0x1000
HL = 32
HV = [0] * HL
for x, v in [(3, 0xFF), (10, 0x01), (11, 0x80), (25, 0x10), (31, 0xFF)]:
    HV[x] = v
HA = [1] * HL
for x in (5, 17, 18, 19, 28):
    HA[x] = 0
DB = 0x100000
ALLOCS = {
    DB: [0, 0, 0xFF, 0, 0, 0, 0, 0x04, 0, 0],                 # [DB, DB+10)
    DB + 10: [0] * 6 + [0xFF] * 2 + [0] * 6,                  # adjacent [DB+10, DB+24)
    DB + 48: [0x20] + [0] * 14 + [0x01],                      # [DB+48, DB+64)
}
FREED = DB + 80


def tiny():
    return Tiny(HB, HV, HA, ALLOCS)


def positions_host():
    return [HB + d for d in (-3, -1, 0, 1, 4, 5, 9, 16, 20, 29, 30, 31, 32, 35)] + [0, 2 ** 64 - 8]


def positions_dev():
    out = [FREED, FREED + 3, DB - 1, DB + 30, 2 ** 64 - 4]
    for b, v in ALLOCS.items():
        L = len(v)
        out += [b, b + 1, b + L // 2, b + L - 1]
    return out


LENGTHS = [0, 1, 2, 3, 5, 8, 13, 16, 17, 31, 33, 40]


def all_records():
    rows = []
    for kind in (0, 1, 2, 5):
        sp = positions_host() if kind == 0 else positions_dev()
        dp = positions_host() if kind == 1 else positions_dev()
        for s, d, n in itertools.product(sp, dp, LENGTHS):
            rows.append((kind, s, d, n))
    return rows


def test_brute_force_matches_oracle_everywhere():
    rows = all_records()
    t = tiny()
    got = as_tuples(t.oracle().run(recs(rows)))
    want, _ = brute.run_snapshot(t.world(), rows)
    assert len(rows) > 5000
    bad = [(r, g, w) for r, g, w in zip(rows, got, want) if g != w]
    assert not bad, bad[:5]


def test_brute_force_matches_oracle_propagation():
    """Every record alone (one-record batches), with propagation: identical shadow afterwards."""
    rows = all_records()[::3]
    for row in rows:
        t = tiny()
        o = t.oracle()
        v = as_tuples(o.run(recs([row]), propagate=True))
        want, after = brute.run_snapshot(t.world(), [row], propagate=True)
        assert v == want, row
        assert oracle_world(o) == brute_world(after, HB, HL), row


def test_bitmap_padding_bits_are_ignored():
    """Bits of the last A word beyond the region length carry no meaning."""
    rows = [r for r in all_records() if r[0] in (0, 1)]
    t = tiny()
    o = t.oracle()
    clean = as_tuples(o.run(recs(rows)))
    o.ha[-1] |= np.uint64(0xFFFF_FFFF_0000_0000)
    assert as_tuples(o.run(recs(rows))) == clean


def test_snapshot_equals_sequential_without_conflicts():
    """Disjoint sources and destinations: batch snapshot == one-by-one replay."""
    rows = [(0, HB + 0, DB + 48, 8), (2, DB + 1, DB + 12, 6), (1, DB + 56, HB + 20, 8),
            (0, HB + 9, DB + 20, 4)]
    w1, a1 = brute.run_snapshot(tiny().world(), rows, propagate=True)
    w2, a2 = brute.run_sequential(tiny().world(), rows, propagate=True)
    assert w1 == w2 and brute_world(a1, HB, HL) == brute_world(a2, HB, HL)
    o = tiny().oracle()
    assert as_tuples(o.run(recs(rows), propagate=True)) == w1
    assert oracle_world(o) == brute_world(a1, HB, HL)


# ---------------------------------------------------------------------------
# PIN-1: the worked example of Sec. 4 (Listing 2) and the report of Listing 6
# ---------------------------------------------------------------------------

def worked_example_state(fx):
    c_host = 0x7F00_0000_0000
    n_host = fx["copy_bytes"]
    c = 0x7000_0000_0000
    a = c + fx["c_alloc_bytes"]          # placed right after c: one-allocation rule
    b = a + fx["a_alloc_bytes"] + 256
    st_ = OracleState(c_host, n_host, np.full(n_host, 0xFF, np.uint8),
                      bits_to_words(np.ones(n_host, np.uint8)),
                      np.array([c, a, b], np.uint64),
                      np.array([fx["c_alloc_bytes"], fx["a_alloc_bytes"], fx["b_alloc_bytes"]], np.uint64),
                      [np.zeros(fx["c_alloc_bytes"], np.uint8),      # the kernel wrote all of c
                       np.full(fx["a_alloc_bytes"], 0xFF, np.uint8),
                       np.full(fx["b_alloc_bytes"], 0xFF, np.uint8)])
    return st_, c, c_host


def test_pin1_worked_example():
    fx = json.load(open(os.path.join(GOLDEN, "pin1_worked_example.json")))
    assert fx["c_alloc_bytes"] == fx["elements"] * fx["sizeof_float"]
    assert fx["copy_bytes"] == fx["elements"] * fx["sizeof_double"]
    st_, c, c_host = worked_example_state(fx)
    v = st_.run(recs([(1, c, c_host, fx["copy_bytes"])]))[0]
    assert int(v["flags"]) == SRC_OVERRUN
    assert int(v["avail"]) == fx["found_bytes"]
    assert int(v["first_bad"]) == fx["found_bytes"]
    assert int(v["undef_bytes"]) == 0
    # what the report calls "expected" is the size of the copy
    assert fx["expected_bytes"] == fx["copy_bytes"]


# ---------------------------------------------------------------------------
# PIN-7: the error classes of Sec. 2 (plus struct padding) as closed forms
# ---------------------------------------------------------------------------

def test_pin7_uninitialised_host_source():
    n = 4096
    st_ = OracleState(HB, n, np.full(n, 0xFF, np.uint8), bits_to_words(np.ones(n)),
                      np.array([DB], np.uint64), np.array([n], np.uint64), [np.zeros(n, np.uint8)])
    v = st_.run(recs([(0, HB, DB, n)]))[0]
    assert (int(v["flags"]), int(v["first_bad"]), int(v["undef_bytes"]), int(v["avail"])) == \
        (SRC_UNDEF, 0, n, n)


@pytest.mark.parametrize("L,delta", [(1000, 1), (4096, 64), (77, 13)])
def test_pin7_overrun(L, delta):
    st_ = OracleState(HB, 2 * L, np.zeros(2 * L, np.uint8), bits_to_words(np.ones(2 * L)),
                      np.array([DB, DB + L], np.uint64), np.array([L, L], np.uint64),
                      [np.zeros(L, np.uint8), np.zeros(L, np.uint8)])
    v = st_.run(recs([(0, HB, DB, L + delta)]))[0]
    assert (int(v["flags"]), int(v["first_bad"]), int(v["undef_bytes"]), int(v["avail"])) == \
        (DST_OVERRUN, L, 0, L)


def test_pin7_copy_into_freed_region():
    n = 300
    st_ = OracleState(HB, n, np.zeros(n, np.uint8), bits_to_words(np.ones(n)),
                      np.array([DB], np.uint64), np.array([n], np.uint64), [np.zeros(n, np.uint8)])
    # DB + 4096 was freed: it is not in the live list
    v = st_.run(recs([(0, HB, DB + 4096, n)]))[0]
    assert (int(v["flags"]), int(v["first_bad"]), int(v["undef_bytes"]), int(v["avail"])) == \
        (DST_UNALLOC, 0, 0, 0)


def test_pin7_struct_padding():
    R = 257
    hv = np.tile(np.array([0] * 13 + [0xFF] * 3, np.uint8), R)
    st_ = OracleState(HB, 16 * R, hv, bits_to_words(np.ones(16 * R)),
                      np.array([DB], np.uint64), np.array([16 * R], np.uint64),
                      [np.full(16 * R, 0xFF, np.uint8)])
    v = st_.run(recs([(0, HB, DB, 16 * R)]), propagate=True)[0]
    assert (int(v["flags"]), int(v["first_bad"]), int(v["undef_bytes"])) == (SRC_UNDEF, 13, 3 * R)
    assert np.array_equal(st_.vs[0], hv)


def test_bad_kind_and_zero_length():
    t = tiny().oracle()
    v = as_tuples(t.run(recs([(3, HB, DB, 4), (0, HB, DB, 0), (2, DB, DB, 0)])))
    assert v == [(BAD_KIND, NONE, 0, 0), (0, NONE, 0, 0), (0, NONE, 0, 0)]


# ---------------------------------------------------------------------------
# PIN-4: special cases that reduce to library routines
# ---------------------------------------------------------------------------

@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2 ** 31))
def test_pin4_numpy_reductions(seed):
    rng = np.random.default_rng(seed)
    hl = int(rng.integers(64, 5000))
    hv = np.where(rng.random(hl) < rng.choice([0.0, 0.01, 0.3]), rng.integers(1, 256, hl), 0).astype(np.uint8)
    sizes = rng.integers(1, 3000, size=int(rng.integers(1, 8)))
    bases = DB + np.cumsum(np.concatenate([[0], sizes[:-1]])) + rng.integers(0, 64, sizes.size).cumsum()
    vs = [rng.integers(0, 256, int(s)).astype(np.uint8) * (rng.random(int(s)) < 0.2) for s in sizes]
    vs = [v.astype(np.uint8) for v in vs]
    st_ = OracleState(HB, hl, hv, bits_to_words(np.ones(hl)), bases.astype(np.uint64),
                      sizes.astype(np.uint64), vs)
    j = int(rng.integers(0, sizes.size))
    L = int(sizes[j])
    n = int(rng.integers(1, min(L, hl) + 1))
    o = int(rng.integers(0, L - n + 1))
    s = int(rng.integers(0, hl - n + 1))
    dst = int(bases[j]) + o
    v = st_.run(recs([(0, HB + s, dst, n)]))[0]
    win = hv[s:s + n]
    nz = np.flatnonzero(win)
    assert int(v["undef_bytes"]) == np.count_nonzero(win)
    assert int(v["first_bad"]) == (int(nz[0]) if nz.size else NONE)
    # the lookup is bisect over the sorted bases
    k = bisect.bisect_right(list(map(int, bases)), dst) - 1
    assert k == j and int(v["avail"]) == int(bases[k]) + L - dst
    # device->host of the same bytes reads the allocation slice
    v2 = st_.run(recs([(1, dst, HB + s, n)]))[0]
    sl = vs[j][o:o + n]
    nz2 = np.flatnonzero(sl)
    assert int(v2["undef_bytes"]) == np.count_nonzero(sl)
    assert int(v2["first_bad"]) == (int(nz2[0]) if nz2.size else NONE)
    # propagation equals a slice copy
    before = [x.copy() for x in st_.vs]
    st_.run(recs([(0, HB + s, dst, n)]), propagate=True)
    exp = before[j].copy()
    exp[o:o + n] = win
    assert np.array_equal(st_.vs[j], exp)


# ---------------------------------------------------------------------------
# PIN-6: laws of the definition
# ---------------------------------------------------------------------------

def random_world(rng, hl=600):
    hv = np.where(rng.random(hl) < 0.05, rng.integers(1, 256, hl), 0).astype(np.uint8)
    a = (rng.random(hl) > 0.03).astype(np.uint8)
    sizes = rng.integers(1, 400, size=5)
    gaps = rng.integers(0, 3, size=5) * rng.integers(1, 40, size=5)
    bases = DB + np.cumsum(np.concatenate([[0], sizes[:-1]])) + np.cumsum(gaps)
    vs = [np.where(rng.random(int(s)) < 0.05, rng.integers(1, 256, int(s)), 0).astype(np.uint8) for s in sizes]
    return Tiny(HB, hv, a, dict(zip(map(int, bases), vs))), bases, sizes


def random_record(rng, bases, sizes, hl=600):
    kind = int(rng.integers(0, 3))
    n = int(rng.integers(1, 300))

    def hostp():
        return HB + int(rng.integers(-20, hl + 10))

    def devp():
        j = int(rng.integers(0, bases.size))
        return int(bases[j]) + int(rng.integers(-5, int(sizes[j]) + 5))
    s = hostp() if kind == 0 else devp()
    d = hostp() if kind == 1 else devp()
    return kind, s, d, n


@settings(max_examples=80, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2 ** 31))
def test_pin6_split_law(seed):
    """Splitting a record at k: counts add, first_bad = min(f1, k + f2), flags OR
    (overrun/unalloc of the tail re-based onto its own avail)."""
    rng = np.random.default_rng(seed)
    t, bases, sizes = random_world(rng)
    o = t.oracle()
    kind, s, d, n = random_record(rng, bases, sizes)
    av = int(o.run(recs([(kind, s, d, n)]))[0]["avail"])
    # the tail's pointer must stay inside the same allocation on device sides
    kmax = n if av >= n else max(av - 1, 0)
    k = int(rng.integers(0, kmax + 1))
    whole, a, b = as_tuples(o.run(recs([(kind, s, d, n), (kind, s, d, k), (kind, s + k, d + k, n - k)])))
    fa = a[1] if k > 0 else NONE
    fb = (k + b[1]) if (n - k > 0 and b[1] != NONE) else NONE
    assert whole[2] == a[2] + b[2]
    assert whole[1] == min(fa, fb)
    mask = SRC_UNADDR | SRC_UNDEF | DST_UNADDR
    assert whole[0] & mask == (a[0] | b[0]) & mask


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2 ** 31))
def test_pin6_permutation_invariance(seed):
    rng = np.random.default_rng(seed)
    t, bases, sizes = random_world(rng)
    rows = [random_record(rng, bases, sizes) for _ in range(40)]
    v = as_tuples(t.oracle().run(recs(rows)))
    p = rng.permutation(len(rows))
    vp = as_tuples(t.oracle().run(recs([rows[i] for i in p])))
    assert [v[i] for i in p] == vp


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2 ** 31))
def test_pin6_round_trip(seed):
    """Propagate host->device, then check the destination as a device source:
    same undefined count and same first undefined byte where the source was
    addressable throughout."""
    rng = np.random.default_rng(seed)
    t, bases, sizes = random_world(rng)
    t.a[:] = 1
    o = t.oracle()
    j = int(rng.integers(0, bases.size))
    L = int(sizes[j])
    n = int(rng.integers(1, L + 1))
    s = HB + int(rng.integers(0, 600 - n + 1)) if n <= 600 else HB
    n = min(n, 600)
    v1 = o.run(recs([(0, s, int(bases[j]), n)]), propagate=True)[0]
    v2 = o.run(recs([(2, int(bases[j]), DB - 10_000, n)]))[0]
    assert int(v1["undef_bytes"]) == int(v2["undef_bytes"])
    f1 = int(v1["first_bad"]) if int(v1["undef_bytes"]) else NONE
    first_undef2 = np.flatnonzero(o.vs[j][:n])
    assert f1 == (int(first_undef2[0]) if first_undef2.size else NONE)


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(seed=st.integers(0, 2 ** 31))
def test_pin6_growing_an_allocation_adds_no_fault(seed):
    rng = np.random.default_rng(seed)
    L = int(rng.integers(1, 200))
    grow = int(rng.integers(1, 50))
    n = int(rng.integers(1, 300))
    hv = np.where(rng.random(400) < 0.02, 0xFF, 0).astype(np.uint8)
    base_v = np.zeros(L + grow, np.uint8)
    small = OracleState(HB, 400, hv, bits_to_words(np.ones(400)), np.array([DB], np.uint64),
                        np.array([L], np.uint64), [base_v[:L].copy()])
    big = OracleState(HB, 400, hv, bits_to_words(np.ones(400)), np.array([DB], np.uint64),
                      np.array([L + grow], np.uint64), [base_v.copy()])
    r = recs([(0, HB, DB, min(n, 400))])
    a, b = small.run(r)[0], big.run(r)[0]
    assert int(b["flags"]) & ~int(a["flags"]) == 0
    assert int(b["first_bad"]) >= int(a["first_bad"]) or int(b["first_bad"]) == NONE
    assert int(b["avail"]) == int(a["avail"]) + grow
