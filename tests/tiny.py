"""Tiny hand-built universes shared by the oracle pin tests (test-only)."""
from __future__ import annotations

import numpy as np

from oracle.brute import World
from oracle.oracle import OracleState, REC


def bits_to_words(bits):
    bits = np.asarray(bits, np.uint8)
    pad = (-bits.size) % 64
    b = np.concatenate([bits, np.zeros(pad, np.uint8)])
    return np.packbits(b, bitorder="little").view(np.uint64).copy()


class Tiny:
    """hb, hv (list), a (list of 0/1), allocs {base: V list} -> oracle state + brute world."""

    def __init__(self, hb, hv, a, allocs):
        self.hb, self.hv, self.a = hb, np.asarray(hv, np.uint8), np.asarray(a, np.uint8)
        self.allocs = {int(k): np.asarray(v, np.uint8) for k, v in allocs.items()}

    def oracle(self):
        bases = sorted(self.allocs)
        return OracleState(self.hb, self.hv.size, self.hv.copy(), bits_to_words(self.a),
                           np.array(bases, np.uint64),
                           np.array([self.allocs[b].size for b in bases], np.uint64),
                           [self.allocs[b].copy() for b in bases])

    def world(self):
        return World(self.hb, self.hv.tolist(), self.a.tolist(), {b: v.tolist() for b, v in self.allocs.items()})


def recs(rows):
    r = np.zeros(len(rows), REC)
    for i, (k, s, d, n) in enumerate(rows):
        r[i] = (s, d, n, k, 0)
    return r


def as_tuples(v):
    return [(int(a), int(b), int(c), int(d)) for a, b, c, d in
            zip(v["flags"], v["first_bad"], v["undef_bytes"], v["avail"])]


def oracle_world(st: OracleState):
    """Snapshot of an oracle state as comparable python structures."""
    return st.hv.tolist(), {int(b): v.tolist() for b, v in zip(st.bases, st.vs)}


def brute_world(w: World, hb, hl):
    return [w.hv[hb + x] for x in range(hl)], {b: list(v) for b, v in w.allocs.items()}
