"""Serving on the GPU: continuous batching with interleaved allocation events.
Every verdict is the same alone and in the mix, and equals a sequential oracle
replay of the event log (tolerance 0: integer results)."""
import numpy as np
import pytest

from paper_1310_0901_amd import workloads as W
from tests import util
from tests.serve_replay import replay, replay_sampled

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def S():
    from paper_1310_0901_amd import serving, xfercheck
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    xfercheck.lib()
    return serving


def verdicts(res):
    v = np.zeros(res.size, W.VERDICT_DTYPE)
    for f in util.FIELDS:
        v[f] = res[f]
    return v


def test_serving_mix_alone_and_oracle(S):
    sw = W.small_serve()
    want = replay(sw)
    runs = {}
    for name, cfg in (("mix", S.config(streams=4, max_batch=256)),
                      ("mix-graphs", S.config(streams=4, max_batch=512)),
                      ("alone", S.config(streams=1, max_batch=1)),
                      ("closed", S.config(streams=3, max_batch=64, open_loop=False)),
                      ("plain", S.config(plain=True)),
                      ("capped", S.config(streams=4, max_batch=256, mem_cap=4 << 20))):
        dw = S.serve_world(sw)
        try:
            res, summ = S.run(dw, sw, cfg)
        finally:
            dw.close()
        print(name, summ, flush=True)
        util.assert_verdicts_equal(verdicts(res), want, f"serving {name}")
        runs[name] = (res, summ)
    # epochs: the number of allocation events before each request
    ev = sw.events
    nev_before = np.cumsum(ev["type"] != W.EV_CHECK)[ev["type"] == W.EV_CHECK]
    assert np.array_equal(runs["mix"][0]["epoch"], nev_before)
    # the admission cap bounds the bytes in flight (a single request may exceed it alone)
    big = float(np.max(sw.requests["n"]) * 1.125)
    assert runs["capped"][1]["max_inflight_GB"] * 1e9 <= max(4 << 20, big) + 1
    assert runs["mix"][1]["mean_batch"] >= 1.0
    # latencies of the open-loop runs, several in this process: a completion
    # never comes before its scheduled arrival (the device clock starts no
    # later than the host clock)
    for name in ("mix", "alone", "plain", "capped"):
        res = runs[name][0]
        lat = res["t_done"] - res["t_arrive"]
        assert np.isfinite(lat).all() and (lat >= 0).all(), name


@pytest.mark.slow
def test_serving_full_log_sampled(S):
    """The full serving configuration (500k requests at 50k/s, 975k initial
    allocations, one alloc/free per 10 requests, so the device table is
    re-merged tens of thousands of times) against a host replay of the log on
    a sample: every 500th request, and the 20 requests after each of 200 table
    events spread over the log."""
    sw = W.config5()
    hv, ha = W.host_v(sw.host), W.host_a(sw.host)
    dw = S.serve_world(sw, host_arrays=(hv, ha))
    try:
        res, summ = S.run(dw, sw, S.config(streams=4, max_batch=64))
    finally:
        dw.close()
    print(summ, flush=True)
    assert summ["table_versions"] > 10_000
    ev = sw.events
    is_req = ev["type"] == W.EV_CHECK
    req_before = np.cumsum(is_req) - is_req            # requests before each event
    table_ev = np.flatnonzero(~is_req)
    picks = table_ev[np.linspace(0, table_ev.size - 1, 200).astype(np.int64)]
    after = (req_before[picks][:, None] + np.arange(20)[None, :]).ravel()
    n_req = int(is_req.sum())
    which = np.unique(np.concatenate([np.arange(0, n_req, 500), after[after < n_req]]))
    want = replay_sampled(sw, which, hv, ha)
    util.assert_verdicts_equal(verdicts(res)[which], want, "serving full log, sampled")
    # the sample holds clean requests and requests into unallocated memory
    assert (want["flags"] == 0).any() and (want["flags"] & (0x4 | 0x20)).any()
