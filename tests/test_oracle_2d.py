"""Pins of the oracle's pitched 2D copies (the strided copies of the footnote
to Sec. 2's error list): hand-derived closed forms for the worked example's
pitched case, an undefined byte inside and outside the copied rows, rows that
leave the allocation, and identities with the 1D check."""
import numpy as np
import pytest

from oracle import oracle

HB, D = 0x7F00_0000_0000, 0x7000_0000_0000
NONE = oracle.NONE
H2D, D2H, D2D = 0, 1, 2


def state(hl, undef_at=(), allocs=((D, 25600),), alloc_v=0):
    hv = np.zeros(hl, np.uint8)
    for x in undef_at:
        hv[x] = 0xFF
    ha = np.full((hl + 63) // 64, ~np.uint64(0), np.uint64)
    bases = np.array([b for b, _ in allocs], np.uint64)
    sizes = np.array([z for _, z in allocs], np.uint64)
    return oracle.OracleState(HB, hl, hv, ha, bases, sizes, [np.full(int(z), alloc_v, np.uint8) for _, z in allocs])


def rec2d(src, dst, width, rows, spitch, dpitch, kind):
    r = np.zeros(1, oracle.REC2D)
    r[0] = (src, dst, width, rows, spitch, dpitch, kind, (0, 0, 0))
    return r


def tup(v):
    return int(v["flags"]), int(v["first_bad"]), int(v["undef_bytes"]), int(v["avail"])


def pins():
    """(state, 2D record, expected verdict), derived by hand."""
    P = []
    # the worked example's pitched copy: 100 rows of 300 bytes into a 256-byte pitch
    # (25,600 bytes): row 99 starts at 25,344 and finds 256 bytes
    P.append((state(30000), rec2d(HB, D, 300, 100, 300, 256, H2D),
              (oracle.DST_OVERRUN, 99 * 300 + 256, 0, 25600)))
    # the same rows 256 bytes wide fit
    P.append((state(30000), rec2d(HB, D, 256, 100, 300, 256, H2D), (0, NONE, 0, 25600)))
    # an undefined host byte at 5 is copied (row 0); the one at 700 lies between rows 1 and 2
    P.append((state(2000, undef_at=(5, 700)), rec2d(HB, D, 100, 3, 400, 100, H2D), (oracle.SRC_UNDEF, 5, 1, 25600)))
    # ... and at 450 it is byte 50 of row 1: index 100 + 50
    P.append((state(2000, undef_at=(450,)), rec2d(HB, D, 100, 3, 400, 100, H2D), (oracle.SRC_UNDEF, 150, 1, 25600)))
    # device rows of 300 at pitch 400 from a 1,000-byte allocation: row 2 finds 200 bytes,
    # row 3 starts past the end
    P.append((state(4096, allocs=((D, 1000),)), rec2d(D, HB, 300, 4, 400, 300, D2H),
              (oracle.SRC_OVERRUN | oracle.SRC_UNALLOC, 2 * 300 + 200, 0, 1000)))
    # no rows, or rows of no bytes
    P.append((state(100), rec2d(HB, D, 10, 0, 10, 10, H2D), (0, NONE, 0, 0)))
    P.append((state(100), rec2d(HB, D, 0, 5, 10, 10, H2D), (0, NONE, 0, 0)))
    # a bad kind
    P.append((state(100), rec2d(HB, D, 10, 2, 10, 10, 7), (oracle.BAD_KIND, NONE, 0, 0)))
    return P


def check_pins(lib=None):
    for i, (st, r, want) in enumerate(pins()):
        if lib is not None:
            st.lib = lib
        assert tup(st.run2d(r)[0]) == want, f"2D pin {i}: {tup(st.run2d(r)[0])} != {want}"


def test_pins():
    check_pins()


@pytest.mark.parametrize("seed", range(10))
def test_identities_with_1d(seed):
    rng = np.random.default_rng(seed)
    hl = 8192
    st = state(hl, undef_at=tuple(int(x) for x in rng.integers(0, hl, 20)), allocs=((D, 8192), (D + 16384, 4096)))
    for _ in range(20):
        width, rows = int(rng.integers(1, 200)), int(rng.integers(1, 20))
        n = width * rows
        off = int(rng.integers(0, hl - n)) if n < hl else 0
        doff = int(rng.integers(0, 8192 - n)) if n < 8192 else 0
        # one row is the 1D record
        one = st.run2d(rec2d(HB + off, D + doff, width, 1, 0, 0, H2D))[0]
        assert tup(one) == tup(st.run(np.array([(HB + off, D + doff, width, H2D, 0)], oracle.REC))[0])
        # contiguous rows inside the allocation are the 1D record of rows * width bytes
        if n <= 8192 - doff and n <= hl - off:
            two = st.run2d(rec2d(HB + off, D + doff, width, rows, width, width, H2D))[0]
            assert tup(two) == tup(st.run(np.array([(HB + off, D + doff, n, H2D, 0)], oracle.REC))[0])
