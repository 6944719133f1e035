"""Serving on the GPU: continuous batching with interleaved allocation events.
Every verdict is the same alone and in the mix, and equals a sequential oracle
replay of the event log (tolerance 0: integer results)."""
import numpy as np
import pytest

from paper_1310_0901_amd import workloads as W
from tests import util
from tests.serve_replay import replay

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
