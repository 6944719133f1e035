"""A quick battery of the oracle's pins, runnable against any build of the
oracle library (used by the mutation test: a planted mistake must fail it).

    python -m tests.pin_battery /path/to/liboracle_variant.so
exits 0 when every pin holds.
"""
import json
import os
import sys

import numpy as np


def main(path):
    from oracle import oracle, brute
    from tests import test_oracle_pins as P
    from tests.tiny import recs, as_tuples, oracle_world, brute_world, bits_to_words
    lib = oracle.load(path)

    def state(t):
        bases = sorted(t.allocs)
        return oracle.OracleState(t.hb, t.hv.size, t.hv.copy(), bits_to_words(t.a),
                                  np.array(bases, np.uint64),
                                  np.array([t.allocs[b].size for b in bases], np.uint64),
                                  [t.allocs[b].copy() for b in bases], lib=lib)

    rows = P.all_records()
    t = P.tiny()
    got = as_tuples(state(t).run(recs(rows)))
    want, _ = brute.run_snapshot(t.world(), rows)
    assert got == want, "brute force (check)"
    for row in rows[::7]:
        o = state(P.tiny())
        v = as_tuples(o.run(recs([row]), propagate=True))
        w2, after = brute.run_snapshot(P.tiny().world(), [row], propagate=True)
        assert v == w2 and oracle_world(o) == brute_world(after, P.HB, P.HL), ("brute force (propagate)", row)
    # the bitmap's padding bits beyond the region are ignored
    o = state(P.tiny())
    o.ha[-1] |= np.uint64(0xFFFF_FFFF_0000_0000)
    edge = [r for r in rows if r[0] in (0, 1)]
    assert as_tuples(o.run(recs(edge))) == [w for r, w in zip(rows, want) if r[0] in (0, 1)], "padding bits"
    # worked example
    fx = json.load(open(os.path.join(P.GOLDEN, "pin1_worked_example.json")))
    c_host, c = 0x7F00_0000_0000, 0x7000_0000_0000
    n = fx["copy_bytes"]
    a = c + fx["c_alloc_bytes"]
    st = oracle.OracleState(c_host, n, np.full(n, 0xFF, np.uint8), bits_to_words(np.ones(n, np.uint8)),
                            np.array([c, a], np.uint64),
                            np.array([fx["c_alloc_bytes"], fx["a_alloc_bytes"]], np.uint64),
                            [np.zeros(fx["c_alloc_bytes"], np.uint8),
                             np.full(fx["a_alloc_bytes"], 0xFF, np.uint8)], lib=lib)
    v = st.run(recs([(1, c, c_host, n)]))[0]
    assert (int(v["flags"]), int(v["first_bad"]), int(v["avail"])) == \
        (oracle.SRC_OVERRUN, fx["found_bytes"], fx["found_bytes"]), "worked example"
    # the concurrent-access join
    from tests.test_oracle_race import check_pins
    check_pins(lib)
    # the pointer check
    from tests.test_oracle_pointers import check_pins as check_pointer_pins
    check_pointer_pins(lib)
    # pitched 2D copies
    from tests.test_oracle_2d import check_pins as check_2d_pins
    check_2d_pins(lib)
    return 0


if __name__ == "__main__":
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    try:
        sys.exit(main(sys.argv[1]))
    except AssertionError as e:
        print("pin failed:", e)
        sys.exit(3)
