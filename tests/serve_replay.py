"""Sequential oracle replay of a serving event log (test-only): the events are
applied one after another and every check request is evaluated by the CPU
oracle against the allocation table as it stands at its arrival."""
from __future__ import annotations

import numpy as np

from oracle.oracle import OracleState
from paper_1310_0901_amd import workloads as W


def replay(sw: W.ServeWorkload) -> np.ndarray:
    hv, ha = W.host_v(sw.host), W.host_a(sw.host)
    live = {int(sw.dev.base[j]): W.alloc_v(sw.dev, int(j)) for j in sw.dev.live_idx}
    ev = sw.events
    out = np.zeros(int((ev["type"] == W.EV_CHECK).sum()), W.VERDICT_DTYPE)
    k = 0
    i = 0
    n = ev.size
    while i < n:
        if ev["type"][i] == W.EV_ALLOC:
            live[int(ev["dst"][i])] = np.full(int(ev["n"][i]), 0xFF, np.uint8)
            i += 1
            continue
        if ev["type"][i] == W.EV_FREE:
            del live[int(ev["dst"][i])]
            i += 1
            continue
        j = i
        while j < n and ev["type"][j] == W.EV_CHECK:
            j += 1
        recs = W.make_records(ev["kind"][i:j], ev["src"][i:j], ev["dst"][i:j], ev["n"][i:j])
        bases = np.array(sorted(live), np.uint64)
        st = OracleState(sw.host.base, sw.host.length, hv, ha, bases,
                         np.array([live[int(b)].size for b in bases], np.uint64), [live[int(b)] for b in bases])
        out[k:k + (j - i)] = st.run(recs)
        k += j - i
        i = j
    return out


def replay_sampled(sw: W.ServeWorkload, which, hv, ha) -> np.ndarray:
    """Oracle verdicts of the check requests listed in `which` (indices among
    the requests), each against the allocation table as it stands at its
    arrival, for logs whose whole device shadow is too large to hold: the live
    set is tracked as (creation, free) event indices of every allocation the
    log ever holds, and V is materialised only for the allocations a sampled
    request's device pointers lie in (a verdict depends only on those).
    Allocations made by the log are at fresh addresses, above the initial ones
    and never reused, so every pointer lies in at most one of them."""
    ev = sw.events
    d = sw.dev
    req_ev = np.flatnonzero(ev["type"] == W.EV_CHECK)
    made = np.flatnonzero(ev["type"] == W.EV_ALLOC)
    init = d.live_idx
    bases = np.concatenate([d.base[init].astype(np.int64), ev["dst"][made].astype(np.int64)])
    sizes = np.concatenate([d.size[init].astype(np.int64), ev["n"][made].astype(np.int64)])
    assert (np.diff(bases) > 0).all() and (bases[:-1] + sizes[:-1] <= bases[1:]).all()
    born = np.concatenate([np.full(init.size, -1, np.int64), made])
    died = np.full(bases.size, np.iinfo(np.int64).max, np.int64)
    freed = np.flatnonzero(ev["type"] == W.EV_FREE)
    fid = np.searchsorted(bases, ev["dst"][freed].astype(np.int64))
    assert (bases[fid] == ev["dst"][freed].astype(np.int64)).all()
    assert (died[fid] == np.iinfo(np.int64).max).all()   # each allocation is freed once
    died[fid] = freed
    which = np.asarray(which, np.int64)
    out = np.zeros(which.size, W.VERDICT_DTYPE)
    for o, q in enumerate(which):
        i = int(req_ev[q])
        rec = W.make_records(ev["kind"][i:i + 1], ev["src"][i:i + 1], ev["dst"][i:i + 1], ev["n"][i:i + 1])
        ptrs = [int(rec["src"][0])] if rec["kind"][0] != W.KIND_H2D else []
        ptrs += [int(rec["dst"][0])] if rec["kind"][0] != W.KIND_D2H else []
        ids = set()
        for p in ptrs:
            j = int(np.searchsorted(bases, p, side="right")) - 1
            if j >= 0 and p < bases[j] + sizes[j] and born[j] < i < died[j]:
                ids.add(j)
        ids = sorted(ids)
        vs = [W.alloc_v(d, int(init[j])) if j < init.size else np.full(int(sizes[j]), 0xFF, np.uint8) for j in ids]
        st = OracleState(sw.host.base, sw.host.length, hv, ha, bases[ids].astype(np.uint64),
                         sizes[ids].astype(np.uint64), vs)
        out[o] = st.run(rec)[0]
    return out
