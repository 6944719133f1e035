"""Pins of the oracle's pointer check (kernel arguments, Sec. 5.1, read as
stated in oracle/oracle.c): hand-derived cases and the address-set brute
force of oracle/brute.py on random tiny tables."""
import numpy as np
import pytest

from oracle import brute, oracle

# A = [1000, 1100) and B = [1100, 1200) adjacent, C = [5000, 5010)
ALLOCS = {1000: 100, 1100: 100, 5000: 10}
# pointer -> (flags, base, avail), derived by hand
PINS = {
    1000: (0, 1000, 100),      # first byte of A
    1099: (0, 1000, 1),        # last byte of A
    1100: (0, 1100, 100),      # held by B; also one past A: holding wins
    1200: (0, 1100, 0),        # one past the end of B
    1201: (1, 0, 0),
    999: (1, 0, 0),
    0: (1, 0, 0),
    5009: (0, 5000, 1),
    5010: (0, 5000, 0),
    5011: (1, 0, 0),
    4999: (1, 0, 0),
    (1 << 64) - 1: (1, 0, 0),
}


def run(allocs, ptrs, lib=None, reverse=False):
    bases = sorted(allocs, reverse=reverse)
    o = oracle.pointers(bases, [allocs[b] for b in bases], ptrs, lib=lib)
    return [(int(f), int(b), int(a)) for f, b, a in zip(o["flags"], o["base"], o["avail"])]


def check_pins(lib=None):
    ptrs = list(PINS)
    assert run(ALLOCS, ptrs, lib) == [PINS[p] for p in ptrs], "pointer pins"
    # the answer does not depend on the order of the allocation list
    assert run(ALLOCS, ptrs, lib, reverse=True) == [PINS[p] for p in ptrs], "pointer pins (list reversed)"
    assert brute.pointer_checks(ALLOCS, ptrs) == [PINS[p] for p in ptrs], "pointer pins (brute)"
    for seed in range(30):
        allocs, ptrs = random_table(np.random.default_rng(seed))
        assert run(allocs, ptrs, lib) == brute.pointer_checks(allocs, ptrs), f"pointer brute seed {seed}"


def random_table(rng, universe=400, n=8):
    """Disjoint allocations (some adjacent) in a small universe, and pointers
    over the whole universe and its edges."""
    allocs, x = {}, int(rng.integers(1, 20))
    for _ in range(n):
        z = int(rng.integers(1, 40))
        if x + z >= universe:
            break
        allocs[x] = z
        x += z + (0 if rng.random() < 0.4 else int(rng.integers(1, 30)))
    ptrs = [int(p) for p in rng.integers(0, universe, 60)] + [b + z for b, z in allocs.items()] + list(allocs)
    return allocs, ptrs


def test_pins():
    ptrs = list(PINS)
    assert run(ALLOCS, ptrs) == [PINS[p] for p in ptrs]
    assert run(ALLOCS, ptrs, reverse=True) == [PINS[p] for p in ptrs]
    assert brute.pointer_checks(ALLOCS, ptrs) == [PINS[p] for p in ptrs]


@pytest.mark.parametrize("seed", range(40))
def test_matches_address_sets(seed):
    allocs, ptrs = random_table(np.random.default_rng(100 + seed))
    assert run(allocs, ptrs) == brute.pointer_checks(allocs, ptrs)


def test_no_allocations_and_order():
    assert run({}, [0, 5, 1 << 40]) == [(1, 0, 0)] * 3
    # the order of the allocation list does not matter
    rng = np.random.default_rng(9)
    allocs, ptrs = random_table(rng)
    bases = list(allocs)
    rng.shuffle(bases)
    o = oracle.pointers(bases, [allocs[b] for b in bases], ptrs)
    assert [(int(f), int(b), int(a)) for f, b, a in zip(o["flags"], o["base"], o["avail"])] == run(allocs, ptrs)
