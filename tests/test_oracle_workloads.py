"""The oracle on the benchmark workloads (reduced sizes), pinned by interval
arithmetic over the generators' sparse descriptions, by the injected labels,
and by configuration 4's closed form (no GPU)."""
import numpy as np
import pytest

from oracle.oracle import OracleState, NONE, SRC_UNDEF, SRC_UNALLOC, SRC_OVERRUN, \
    DST_UNALLOC, DST_OVERRUN
from paper_1310_0901_amd import workloads as W
from tests import intervals


def oracle_for(w):
    dev = w.dev
    live = dev.live_idx
    return OracleState(w.host.base, w.host.length, W.host_v(w.host), W.host_a(w.host),
                       dev.base[live], dev.size[live], [W.alloc_v(dev, j) for j in live])


@pytest.mark.parametrize("k", [1, 2, 3])
def test_pin5_interval_arithmetic_matches_oracle(k):
    w = W.small_config(k)
    got = oracle_for(w).run(w.records)
    f, fb, u, a = intervals.expected(w)
    assert np.array_equal(got["flags"], f)
    assert np.array_equal(got["first_bad"], fb)
    assert np.array_equal(got["undef_bytes"], u)
    assert np.array_equal(got["avail"], a)


@pytest.mark.parametrize("k", [1, 3])
def test_pin5_injected_labels(k):
    w = W.small_config(k)
    v = oracle_for(w).run(w.records)
    kind = w.records["kind"]
    n = w.records["n"].astype(np.int64)
    over = w.label == W.LABEL_OVERRUN
    uaf = w.label == W.LABEL_UAF
    assert over.sum() > 0 and uaf.sum() > 0
    # the injected side: source for device->host, destination otherwise
    of = np.where(kind == W.KIND_D2H, SRC_OVERRUN, DST_OVERRUN)
    uf = np.where(kind == W.KIND_D2H, SRC_UNALLOC, DST_UNALLOC)
    assert np.all(v["flags"][over] & of[over])
    assert np.all(v["first_bad"][over].astype(np.int64) <= v["avail"][over].astype(np.int64))
    assert np.all(v["avail"][over].astype(np.int64) < n[over])
    assert np.all(v["flags"][uaf] & uf[uaf])
    assert np.all(v["first_bad"][uaf] == 0) and np.all(v["avail"][uaf] == 0)
    clean = w.label == W.LABEL_CLEAN
    assert not np.any(v["flags"][clean] & (SRC_OVERRUN | DST_OVERRUN | SRC_UNALLOC | DST_UNALLOC))


def test_pin2_closed_form_config4_small():
    """16-byte records with 3 padding bytes each and 1% single payload bits:
    every hop reports 3R + P undefined bytes, first at min(13, payload byte of
    record 0); after the chain the last allocation's shadow equals host V."""
    w = W.config4(host_len=1 << 20, pieces=1, hops=4)
    o = oracle_for(w)
    R, P = w.R, w.P
    assert P == int(0.01 * R)
    b0 = [int(b) for r, b in zip(w.payload_records, w.payload_byte) if r == 0]
    want_first = min([13] + b0)
    for stage in w.stages:
        v = o.run(stage, propagate=True)
        assert int(v["flags"][0]) == SRC_UNDEF
        assert int(v["undef_bytes"][0]) == 3 * R + P
        assert int(v["first_bad"][0]) == want_first
    hv = W.host_v(w.host)
    for j in range(len(w.stages)):
        assert np.array_equal(o.vs[j], hv)


def test_pin2_closed_form_config4_pieces():
    w = W.config4(host_len=1 << 20, pieces=37, hops=2)
    o = oracle_for(w)
    R, P = w.R, w.P
    for stage in w.stages:
        v = o.run(stage, propagate=True)
        assert int(v["undef_bytes"].sum()) == 3 * R + P
    assert np.array_equal(o.vs[-1], W.host_v(w.host))


def test_generators_are_seeded_and_shaped():
    a, b = W.small_config(3), W.small_config(3)
    assert np.array_equal(a.records, b.records)
    w = W.config3(n_transfers=20000, n_alloc=4096, host_len=64 << 20)
    kinds = np.bincount(w.records["kind"], minlength=3) / w.count
    assert abs(kinds[0] - 0.6) < 0.02 and abs(kinds[1] - 0.1) < 0.02 and abs(kinds[2] - 0.3) < 0.02
    assert abs((w.label == W.LABEL_OVERRUN).mean() - 0.02) < 0.005
    assert abs((w.label == W.LABEL_UAF).mean() - 0.01) < 0.004
    n = w.records["n"].astype(np.float64)
    # log-uniform sizes: median near sqrt(8 * 16 MiB)
    assert 0.8 < np.median(n) / np.sqrt(8 * 16 * 2 ** 20) < 1.25


def test_sampled_serving_replay_equals_full_replay():
    """The sampled replay (live set tracked by event index, V materialised
    only for the allocations each request touches) gives the full sequential
    replay's verdicts on a small log, for every request."""
    from tests.serve_replay import replay, replay_sampled
    sw = W.small_serve()
    want = replay(sw)
    n = want.size
    which = np.arange(n)
    got = replay_sampled(sw, which, W.host_v(sw.host), W.host_a(sw.host))
    for f in ("flags", "first_bad", "undef_bytes", "avail"):
        assert np.array_equal(got[f], want[f]), f
    # the log makes and frees allocations that requests then hit
    assert (want["flags"] & (DST_UNALLOC | SRC_UNALLOC)).any()


@pytest.mark.parametrize("pieces", [1, 7, 64])
def test_config4_piece_closed_form_matches_oracle(pieces):
    """The per-piece closed form used at full size (padding bytes by
    arithmetic, payload bytes by search) equals the oracle on a 1 MiB region
    cut into pieces, on the first stage and on a device-to-device hop."""
    w = W.config4(host_len=1 << 20, pieces=pieces)
    st = oracle_for(w)
    for h in (0, 1):
        stage = w.stages[h]
        if h == 1:
            st.run(w.stages[0], check=False, propagate=True)
        got = st.run(stage)
        und, first = intervals.piece_closed_form(w, stage)
        assert np.array_equal(got["undef_bytes"], und)
        assert np.array_equal(got["first_bad"], first)
