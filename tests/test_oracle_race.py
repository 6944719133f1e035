"""Pins of the oracle's concurrent-access join (Sec. 2's concurrent accesses,
read as stated in oracle/oracle.c): hand-derived cases, the byte-set brute
force of oracle/brute.py on random tiny batches, and invariants (record
permutation, stream relabelling, epoch splitting, the pair predicate)."""
import numpy as np
import pytest

from oracle import brute, oracle
from tests.tiny import recs

D = 0x7000_0000_0000      # a device address
H = 0x5000_0000           # a host address
H2D, D2H, D2D = 0, 1, 2
L48 = 1 << 48
TOP = 1 << 64       # one past the last address

# (rows (kind, src, dst, n), streams, epochs, expected flags); flags derived by hand
PINS = [
    # two uploads on different streams writing overlapping device bytes
    ([(H2D, H, D, 100), (H2D, H + 1000, D + 50, 100)], [1, 2], [0, 0], [2, 2]),
    # ... on one stream: ordered
    ([(H2D, H, D, 100), (H2D, H + 1000, D + 50, 100)], [1, 1], [0, 0], [0, 0]),
    # ... in different epochs: ordered
    ([(H2D, H, D, 100), (H2D, H + 1000, D + 50, 100)], [1, 2], [0, 1], [0, 0]),
    # two downloads of the same device bytes: reads never conflict
    ([(D2H, D, H, 100), (D2H, D, H + 200, 100)], [1, 2], [0, 0], [0, 0]),
    # an upload writes what a download reads (last byte shared)
    ([(H2D, H, D, 100), (D2H, D + 99, H + 500, 100)], [1, 2], [0, 0], [2, 1]),
    # adjacent ranges share no byte
    ([(H2D, H, D, 100), (D2H, D + 100, H + 500, 100)], [1, 2], [0, 0], [0, 0]),
    # two device copies swapping buffers: each reads what the other writes
    ([(D2D, D, D + 1000, 100), (D2D, D + 1000, D, 100)], [1, 2], [0, 0], [3, 3]),
    # two writers on one stream, one reader on another
    ([(H2D, H, D, 64), (H2D, H + 64, D, 64), (D2H, D + 10, H + 1000, 5)], [1, 1, 2], [0, 0, 0], [2, 2, 1]),
    # a download into host bytes another stream uploads from
    ([(D2H, D, H, 50), (H2D, H + 25, D + 5000, 50)], [3, 4], [7, 7], [2, 1]),
    # bad kind: not checked, and meets nothing
    ([(3, H, D, 100), (H2D, H + 1000, D, 100)], [1, 2], [0, 0], [4, 0]),
    # any address: ranges ending at, crossing and lying above 2^48 meet as integers do
    ([(H2D, H, L48 - 100, 100), (H2D, H + 200, L48 - 50, 50)], [1, 2], [0, 0], [2, 2]),
    ([(H2D, H, L48 - 50, 100), (H2D, H + 200, L48 - 100, 100)], [1, 2], [0, 0], [2, 2]),
    ([(H2D, H, L48 - 50, 50), (D2H, L48, H + 500, 10)], [1, 2], [0, 0], [0, 0]),
    ([(D2D, 3 * L48, 5 * L48, 64), (D2H, 5 * L48 + 63, H, 1), (H2D, H + 900, 3 * L48 + 64, 8)],
     [1, 2, 3], [0, 0, 0], [2, 1, 0]),
    # any 32-bit epoch: only equality matters
    ([(H2D, H, D, 8), (H2D, H + 8, D, 8)], [1, 2], [(1 << 15) - 1] * 2, [2, 2]),
    ([(H2D, H, D, 8), (H2D, H + 8, D, 8)], [1, 2], [1 << 15, 1 << 15], [2, 2]),
    ([(H2D, H, D, 8), (H2D, H + 8, D, 8)], [1, 2], [(1 << 32) - 1, (1 << 32) - 2], [0, 0]),
    ([(H2D, H, D, 8), (H2D, H + 8, D, 8)], [1, 2], [5, 5 + (1 << 15)], [0, 0]),
    ([(H2D, H, D, 8), (H2D, H + 8, D, 8)], [1, 2], [7, 7 + (1 << 31)], [0, 0]),
    ([(H2D, H, D, 8), (H2D, H + 8, D, 8), (D2H, D + 4, H + 100, 2)], [1, 2, 3],
     [(1 << 32) - 1, (1 << 32) - 1, 1 << 16], [2, 2, 0]),
    # ranges that run past 2^64 are integer ranges: they meet the top bytes, never address 0
    ([(D2D, TOP - 300, TOP - 10, 100), (H2D, H, TOP - 1, 1), (H2D, H + 500, 0, 50)], [1, 2, 3], [0, 0, 0],
     [2, 2, 0]),
    ([(H2D, H, TOP - 1, TOP - 1), (D2H, TOP - 1, H + 100, 1), (D2H, 0, H + 300, 100)], [1, 2, 3], [0, 0, 0],
     [3, 3, 2]),
    # zero-length records touch nothing
    ([(H2D, H, D, 0), (H2D, H + 8, D, 8)], [1, 2], [0, 0], [0, 0]),
    # one device copy overlapping itself is no race
    ([(D2D, D, D + 10, 100)], [1], [0], [0]),
    # one-byte overlap at the first byte
    ([(D2D, D, D + 500, 10), (H2D, H, D + 509, 1)], [1, 2], [0, 0], [2, 2]),
]


def run_oracle(rows, streams, epochs, lib=None, which=None):
    return [int(x) for x in oracle.race(recs(rows), streams, epochs, which=which, lib=lib)]


def check_pins(lib=None):
    """Every pin; raises AssertionError naming the first that fails."""
    for i, (rows, st, ep, want) in enumerate(PINS):
        got = run_oracle(rows, st, ep, lib=lib)
        assert got == want, f"race pin {i}: {got} != {want}"
        assert brute.race_flags(rows, st, ep) == want, f"race pin {i} (brute)"
    for seed in range(40):
        rows, st, ep = random_batch(np.random.default_rng(seed), 12)
        assert run_oracle(rows, st, ep, lib=lib) == brute.race_flags(rows, st, ep), f"race brute seed {seed}"
    for seed in range(12):
        rows, st, ep = random_batch(np.random.default_rng(seed), 12, **HIGH[seed % len(HIGH)])
        assert run_oracle(rows, st, ep, lib=lib) == brute.race_flags(rows, st, ep), f"race brute high seed {seed}"


def random_batch(rng, count, universe=160, streams=3, epochs=2, dbase=D, hbase=H, epoch0=0):
    """Tiny batch over two small address windows (device at dbase, host at
    hbase) with many overlaps, some bad kinds and zero lengths; epochs are
    epoch0 + 0 .. epochs - 1."""
    D, H = dbase, hbase
    rows = []
    for _ in range(count):
        kind = int(rng.choice([0, 1, 2, 3], p=[0.35, 0.3, 0.3, 0.05]))
        n = int(rng.integers(0, 24)) if rng.random() > 0.1 else 0
        d_off, h_off = int(rng.integers(0, universe)), int(rng.integers(0, universe))
        dev2 = D + int(rng.integers(0, universe))
        if kind == H2D:
            rows.append((kind, H + h_off, D + d_off, n))
        elif kind == D2H:
            rows.append((kind, D + d_off, H + h_off, n))
        elif kind == D2D:
            rows.append((kind, D + d_off, dev2, n))
        else:
            rows.append((kind, H + h_off, D + d_off, n))
    st = [int(x) for x in rng.integers(0, streams, count)]
    ep = [epoch0 + int(x) for x in rng.integers(0, epochs, count)]
    return rows, st, ep


# windows at the top of the key space: device bytes around 2^48 and up to the
# last address (ranges there run past 2^64), epochs just below 2^32
HIGH = [dict(dbase=L48 - 80, hbase=H, epoch0=(1 << 15) - 1),
        dict(dbase=TOP - 200, hbase=L48 - 100, epoch0=(1 << 32) - 3),
        dict(dbase=TOP - 161, hbase=TOP - 330, epoch0=1 << 31)]


@pytest.mark.parametrize("i", range(len(PINS)))
def test_pin(i):
    rows, st, ep, want = PINS[i]
    assert run_oracle(rows, st, ep) == want
    assert brute.race_flags(rows, st, ep) == want


@pytest.mark.parametrize("seed", range(60))
def test_oracle_matches_byte_sets(seed):
    rng = np.random.default_rng(1000 + seed)
    rows, st, ep = random_batch(rng, int(rng.integers(1, 20)))
    assert run_oracle(rows, st, ep) == brute.race_flags(rows, st, ep)


@pytest.mark.parametrize("seed", range(30))
def test_oracle_matches_byte_sets_high(seed):
    rng = np.random.default_rng(3000 + seed)
    rows, st, ep = random_batch(rng, int(rng.integers(1, 20)), epochs=3, **HIGH[seed % len(HIGH)])
    assert run_oracle(rows, st, ep) == brute.race_flags(rows, st, ep)


def test_invariants():
    rng = np.random.default_rng(7)
    for _ in range(20):
        rows, st, ep = random_batch(rng, 30, universe=400, streams=4, epochs=3)
        base = run_oracle(rows, st, ep)
        # permuting records permutes the flags
        p = rng.permutation(len(rows))
        got = run_oracle([rows[i] for i in p], [st[i] for i in p], [ep[i] for i in p])
        assert got == [base[i] for i in p]
        # an injective relabelling of streams changes nothing
        relabel = {s: 1000 + 7 * s for s in set(st)}
        assert run_oracle(rows, [relabel[s] for s in st], ep) == base
        # epochs are independent: each epoch alone gives the same flags
        for e in set(ep):
            idx = [i for i in range(len(rows)) if ep[i] == e]
            sub = run_oracle([rows[i] for i in idx], [st[i] for i in idx], [ep[i] for i in idx])
            assert sub == [base[i] for i in idx]
        # a subset of records evaluated against the whole batch
        which = np.array(sorted(rng.choice(len(rows), 7, replace=False)), np.uint64)
        assert run_oracle(rows, st, ep, which=which) == [base[int(i)] for i in which]
        # the flags are the OR of the pair predicate over all other records
        r = recs(rows)
        for a in range(len(rows)):
            if base[a] & oracle.RACE_UNCHECKED:
                continue
            f = 0
            for b in range(len(rows)):
                if b != a:
                    dh, sh = oracle.conflict(r[a], r[b], st[a], st[b], ep[a], ep[b])
                    f |= (2 if dh else 0) | (1 if sh else 0)
            assert f == base[a]


def test_threads_and_no_epochs():
    rng = np.random.default_rng(3)
    rows, st, _ = random_batch(rng, 200, universe=3000, streams=5, epochs=1)
    one = oracle.race(recs(rows), st)
    four = oracle.race(recs(rows), st, np.zeros(len(rows), np.uint32), threads=4)
    assert np.array_equal(one, four)
    assert [int(x) for x in one] == brute.race_flags(rows, st)
