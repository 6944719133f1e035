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
