"""GPU parity: the HIP path against the CPU oracle, element by element, on
seeded inputs (needs an MI355X; run with -m gpu)."""
import numpy as np
import pytest

from paper_1310_0901_amd import workloads as W
from tests import util
from tests.test_oracle_pins import all_records, HB, HV, HA, ALLOCS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def X():
    from paper_1310_0901_amd import xfercheck
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    xfercheck.lib()
    return xfercheck


@pytest.fixture(scope="module")
def H(X):
    from paper_1310_0901_amd import harness
    return harness


@pytest.fixture(params=["one-launch", "multi-kernel"])
def batch_path(request, monkeypatch):
    """Batches worked by the one-launch kernel (any batch of up to 2^20
    records) or by the classify / scan / persistent-kernel chain (no batch):
    the limit is read when a context is created."""
    monkeypatch.setenv("XC_SMALL_MAX", str(1 << 20) if request.param == "one-launch" else "0")
    return request.param


@pytest.fixture(params=["host-index", "host-index-overflow", "host-lds", "host-lds-after", "scan-only"])
def host_lds(request, monkeypatch):
    """Check-only batches worked as segments: host-to-device records answered
    from the host index (built for every such batch; and with lists of 4
    entries, which these worlds overflow, so that the index stays invalid and
    the records are scanned), or with their host-source segments staged in
    LDS by the scan kernel's own blocks or by a kernel of their own after it,
    or all of them in the persistent scan kernel."""
    p = request.param
    monkeypatch.setenv("XC_SHADOW_INDEX", "2" if p.startswith("host-index") else "0")
    if p == "host-index-overflow":
        monkeypatch.setenv("XC_SIDX_CAP", "4")
    monkeypatch.setenv("XC_HOST_LDS", {"host-lds-after": "2", "scan-only": "0"}.get(p, "1"))
    return p


def modes(X):
    return [("graph", X.CG_CHECK), ("eager", X.CG_CHECK | X.CG_EAGER), ("plain", X.CG_CHECK | X.CG_PLAIN)]


def tiny_workload(records):
    bases = sorted(ALLOCS)
    return util.workload_from_arrays(HB, HV, HA, bases, [len(ALLOCS[b]) for b in bases],
                                     [ALLOCS[b] for b in bases], records)


def test_tiny_universe_every_case(X, H, batch_path):
    rows = all_records()
    recs = np.array([(s, d, n, k, 0) for k, s, d, n in rows], W.RECORD_DTYPE)
    w = tiny_workload(recs)
    want = util.oracle_for(w).run(recs)
    dw = H.DeviceWorld(w)
    try:
        for name, mode in modes(X):
            util.assert_verdicts_equal(dw.check(recs, mode), want, name)
    finally:
        dw.close()


def test_tiny_universe_segmented(X, H, host_lds, monkeypatch):
    """Every classification case of the tiny universe (bad kinds, empty
    records, unallocated and unaddressable sides, overruns, overlapping
    D2D) in one batch worked as source-block segments of 16 bytes and up,
    on the graph and eager paths."""
    monkeypatch.setenv("XC_REORDER_MIN", "1")
    monkeypatch.setenv("XC_SEG_MIN_LOG2", "4")
    rows = all_records()
    recs = np.array([(s, d, n, k, 0) for k, s, d, n in rows], W.RECORD_DTYPE)
    w = tiny_workload(recs)
    want = util.oracle_for(w).run(recs)
    dw = H.DeviceWorld(w)
    try:
        for name, mode in modes(X)[:2]:
            util.assert_verdicts_equal(dw.check(recs, mode), want, f"segmented {name}")
    finally:
        dw.close()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_small_config_parity(X, H, batch_path, k):
    w = W.small_config(k)
    want = util.oracle_for(w).run(w.records)
    dw = H.DeviceWorld(w)
    try:
        for name, mode in modes(X):
            util.assert_verdicts_equal(dw.check(w.records, mode), want, f"config {k} {name}")
    finally:
        dw.close()


def test_small_tiles_and_ragged_tails(X, H):
    """Minimum tile size, so that records straddle many tiles and every
    tile / wave boundary; random alignments and ragged lengths."""
    rng = np.random.default_rng(7)
    hl, hv, a, bases, sizes, vs = util.random_world(rng, hl=400_000, nalloc=9, max_size=300_000, dens=0.003)
    recs = util.random_records(rng, W.HOST_BASE, hl, bases, sizes, 400, max_n=200_000)
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, recs)
    want = util.oracle_for(w).run(recs)
    dw = H.DeviceWorld(w)
    try:
        for unroll in (1, 2, 4, 8):
            t = X.cg_get_tuning(dw.ctx)
            t.tile_units, t.unroll = 4096, unroll
            X.cg_set_tuning(dw.ctx, t)
            for name, mode in modes(X):
                util.assert_verdicts_equal(dw.check(recs, mode), want, f"unroll {unroll} {name}")
    finally:
        dw.close()


@pytest.mark.parametrize("seed", [11, 12, 13, 14, 15])
def test_random_worlds_check(X, H, batch_path, seed):
    rng = np.random.default_rng(seed)
    hl, hv, a, bases, sizes, vs = util.random_world(rng)
    recs = util.random_records(rng, W.HOST_BASE, hl, bases, sizes, 300)
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, recs)
    want = util.oracle_for(w).run(recs)
    dw = H.DeviceWorld(w)
    try:
        for name, mode in modes(X):
            util.assert_verdicts_equal(dw.check(recs, mode), want, f"seed {seed} {name}")
    finally:
        dw.close()


@pytest.mark.parametrize("seed", [21, 22, 23, 24])
@pytest.mark.parametrize("path", ["graph", "plain"])
def test_random_worlds_propagation(X, H, batch_path, seed, path):
    """Check + propagate on conflict-free batches: verdicts and every shadow
    byte (device allocations and host region) equal the oracle's."""
    rng = np.random.default_rng(seed)
    hl, hv, a, bases, sizes, vs = util.random_world(rng, dens=0.02)
    recs = util.random_records(rng, W.HOST_BASE, hl, bases, sizes, 200, max_n=30_000)
    recs = util.conflict_free(recs, W.HOST_BASE, hl, bases, sizes)
    assert len(recs) >= 3
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, recs)
    o = util.oracle_for(w)
    want = o.run(recs, propagate=True)
    dw = H.DeviceWorld(w)
    try:
        mode = X.CG_CHECK | X.CG_PROPAGATE | X.CG_DEBUG_CONFLICTS
        if path == "plain":
            mode |= X.CG_PLAIN
        util.assert_verdicts_equal(dw.check(recs, mode), want, f"seed {seed}")
        for j in range(bases.size):
            assert np.array_equal(dw.alloc_shadow(bases[j], sizes[j]), o.vs[j]), f"allocation {j}"
        assert np.array_equal(dw.host_shadow(), o.hv), "host region shadow"
    finally:
        dw.close()


def test_config4_small_chain(X, H, batch_path):
    """Struct padding and single payload bits, H2D then D2D hops with
    propagation: verdicts and shadows bit-exact after every hop."""
    w = W.small_config(4)
    o = util.oracle_for(w)
    dw = H.DeviceWorld(w)
    live = w.dev.live_idx
    try:
        for h, stage in enumerate(w.stages):
            want = o.run(stage, propagate=True)
            got = dw.check(stage, X.CG_CHECK | X.CG_PROPAGATE | X.CG_DEBUG_CONFLICTS)
            util.assert_verdicts_equal(got, want, f"hop {h}")
            for k, j in enumerate(live):
                assert np.array_equal(dw.alloc_shadow(w.dev.base[j], w.dev.size[j]), o.vs[k]), (h, k)
    finally:
        dw.close()


def test_conflicting_batch_is_refused(X, H):
    w = tiny_workload(np.zeros(0, W.RECORD_DTYPE))
    dw = H.DeviceWorld(w)
    try:
        b = sorted(ALLOCS)
        recs = np.array([(HB, b[0], 4, 0, 0), (HB + 8, b[0] + 2, 4, 0, 0)], W.RECORD_DTYPE)
        with pytest.raises(X.CgError) as e:
            dw.check(recs, X.CG_CHECK | X.CG_PROPAGATE | X.CG_DEBUG_CONFLICTS)
        assert e.value.status == X.CG_ECONFLICT
    finally:
        dw.close()


@pytest.mark.parametrize("seg_log2", ["20", "4"])
@pytest.mark.parametrize("seed", [31, 32, 33])
def test_reordered_batches(X, H, seed, seg_log2, host_lds, monkeypatch):
    """Batches worked as source-block segments (forced here for small
    batches; with a 16-byte floor on the block size, records are cut into
    several segments each): verdicts and every shadow byte equal the
    oracle's, and equal the verdicts of the same batch in its given order."""
    monkeypatch.setenv("XC_REORDER_MIN", "1")
    monkeypatch.setenv("XC_SEG_MIN_LOG2", seg_log2)
    rng = np.random.default_rng(seed)
    hl, hv, a, bases, sizes, vs = util.random_world(rng, dens=0.02)
    recs = util.random_records(rng, W.HOST_BASE, hl, bases, sizes, 600, max_n=30_000)
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, recs)
    want = util.oracle_for(w).run(recs)
    dw = H.DeviceWorld(w)
    try:
        for mode in (X.CG_CHECK, X.CG_CHECK | X.CG_EAGER, X.CG_CHECK | X.CG_KEEP_ORDER):
            util.assert_verdicts_equal(dw.check(recs, mode), want, f"seed {seed} mode {mode}")
    finally:
        dw.close()
    # check + propagate on a conflict-free subset
    cf = util.conflict_free(recs, W.HOST_BASE, hl, bases, sizes)
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, cf)
    o = util.oracle_for(w)
    want = o.run(cf, propagate=True)
    dw = H.DeviceWorld(w)
    try:
        util.assert_verdicts_equal(dw.check(cf, X.CG_CHECK | X.CG_PROPAGATE), want, f"seed {seed} propagate")
        for j in range(bases.size):
            assert np.array_equal(dw.alloc_shadow(bases[j], sizes[j]), o.vs[j]), f"allocation {j}"
        assert np.array_equal(dw.host_shadow(), o.hv), "host region shadow"
    finally:
        dw.close()


@pytest.mark.parametrize("seed", [41, 42])
def test_segments_of_large_records(X, H, seed, host_lds, monkeypatch):
    """Records of up to 3 MB beside small ones, worked as segments: the block
    size follows the mean record size, so large records are cut into many
    segments (some of them in blocks other records also read), and single
    records or a few units straddle block ends.  Check, and check +
    propagate on a conflict-free subset with every shadow byte compared."""
    monkeypatch.setenv("XC_REORDER_MIN", "1")
    monkeypatch.setenv("XC_SEG_MIN_LOG2", "4")
    rng = np.random.default_rng(seed)
    hl, hv, a, bases, sizes, vs = util.random_world(rng, hl=6 << 20, nalloc=8, max_size=4 << 20, dens=1e-4)
    big = util.random_records(rng, W.HOST_BASE, hl, bases, sizes, 12, max_n=3 << 20)
    small = util.random_records(rng, W.HOST_BASE, hl, bases, sizes, 400, max_n=2000)
    recs = np.concatenate([small[:200], big, small[200:]])
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, recs)
    want = util.oracle_for(w).run(recs)
    dw = H.DeviceWorld(w)
    try:
        for mode in (X.CG_CHECK, X.CG_CHECK | X.CG_EAGER, X.CG_CHECK | X.CG_KEEP_ORDER):
            util.assert_verdicts_equal(dw.check(recs, mode), want, f"seed {seed} mode {mode}")
    finally:
        dw.close()
    cf = util.conflict_free(recs, W.HOST_BASE, hl, bases, sizes)
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, cf)
    o = util.oracle_for(w)
    want = o.run(cf, propagate=True)
    dw = H.DeviceWorld(w)
    try:
        util.assert_verdicts_equal(dw.check(cf, X.CG_CHECK | X.CG_PROPAGATE), want, f"seed {seed} propagate")
        for j in range(bases.size):
            assert np.array_equal(dw.alloc_shadow(bases[j], sizes[j]), o.vs[j]), f"allocation {j}"
        assert np.array_equal(dw.host_shadow(), o.hv), "host region shadow"
    finally:
        dw.close()


def test_segmented_graph_replays(X, H, host_lds, monkeypatch):
    """A segmented batch checked through its captured graph several times on
    the same buffers, with the verdicts overwritten, eager checks and host
    synchronisation between the replays: every replay equals the oracle."""
    monkeypatch.setenv("XC_REORDER_MIN", "1")
    monkeypatch.setenv("XC_SEG_MIN_LOG2", "4")
    rng = np.random.default_rng(51)
    hl, hv, a, bases, sizes, vs = util.random_world(rng, hl=1 << 20, nalloc=10, max_size=200_000, dens=1e-3)
    recs = util.random_records(rng, W.HOST_BASE, hl, bases, sizes, 500, max_n=40_000)
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, recs)
    want = util.oracle_for(w).run(recs)
    dw = H.DeviceWorld(w)
    try:
        rt = H.records_tensor(recs)
        out = H.verdicts_tensor(recs.size)
        s = torch.cuda.current_stream()
        for rep in range(4):
            out.fill_(0xAB)
            X.check_transfers(dw.ctx, rt.data_ptr(), recs.size, out.data_ptr(), X.CG_CHECK, s.cuda_stream)
            s.synchronize()
            util.assert_verdicts_equal(H.verdicts_np(out, recs.size), want, f"replay {rep}")
            # eager work on the same stream between the replays
            util.assert_verdicts_equal(dw.check(recs[::3], X.CG_CHECK | X.CG_EAGER), want[::3], f"eager {rep}")
    finally:
        dw.close()


@pytest.mark.parametrize("cap", ["4096", "64"])
def test_host_index_edges(X, H, cap, monkeypatch):
    """Host-to-device records answered from the host index, against the
    oracle: a region whose length is not a multiple of 16, undefined bytes and
    A holes on both edges of chunks and at the region's last bytes, records
    starting below the region, ending past it, lying wholly outside it, empty,
    and starting and ending at every offset of a chunk; the lists hold every
    faulty chunk (cap 4096) or overflow (cap 64: the records are scanned)."""
    monkeypatch.setenv("XC_REORDER_MIN", "1")
    monkeypatch.setenv("XC_SEG_MIN_LOG2", "4")
    monkeypatch.setenv("XC_SHADOW_INDEX", "2")
    monkeypatch.setenv("XC_SIDX_CAP", cap)
    rng = np.random.default_rng(61)
    hl = 4000 + 7
    hv = np.zeros(hl, np.uint8)
    for o in (0, 15, 16, 31, 32, 47, 100, 101, 102, 1000, 2047, 2048, hl - 17, hl - 1):
        hv[o] = 0x40
    hv[rng.integers(0, hl, 60)] = 0xFF
    a = np.ones(hl, np.uint8)
    for o in (17, 40, 41, 42, 43, 44, 45, 46, 47, 63, 64, 1500, hl - 2):
        a[o] = 0
    a[rng.integers(0, hl, 30)] = 0
    bases = np.array([W.DEV_BASE, W.DEV_BASE + 100_000], np.uint64)
    sizes = np.array([90_000, 5_000], np.uint64)
    vs = [np.zeros(int(z), np.uint8) for z in sizes]
    recs = []
    for start in list(range(-40, 80)) + list(range(hl - 80, hl + 20)) + list(rng.integers(-100, hl + 50, 300)):
        for n in (0, 1, 2, 15, 16, 17, 33, 100, 1000, int(rng.integers(1, hl + 200))):
            recs.append((W.HOST_BASE + int(start), int(bases[0]) + int(rng.integers(0, 80_000)), n, 0, 0))
    # a few device-source records in the same batch
    recs += [(int(bases[1]) + 10, int(bases[0]) + 500, 3000, 2, 0), (int(bases[1]), W.HOST_BASE + 5, 4000, 1, 0)]
    recs = np.array(recs, W.RECORD_DTYPE)
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, recs)
    want = util.oracle_for(w).run(recs)
    dw = H.DeviceWorld(w)
    try:
        for mode in (X.CG_CHECK, X.CG_CHECK | X.CG_EAGER):
            util.assert_verdicts_equal(dw.check(recs, mode), want, f"cap {cap} mode {mode}")
    finally:
        dw.close()


def faulty_chunks(hv, a):
    """Chunks of a host region with an undefined byte (V != 0, A = 1), and
    with an unaddressable byte (A = 0)."""
    n = (hv.size + 15) // 16 * 16
    und = np.zeros(n, bool)
    und[:hv.size] = (hv != 0) & (a == 1)
    un = np.zeros(n, bool)
    un[:hv.size] = a == 0
    return int(und.reshape(-1, 16).any(1).sum()), int(un.reshape(-1, 16).any(1).sum())


@pytest.mark.parametrize("world", ["host-fits", "pool-fits", "both-fit"])
def test_shadow_index_dense_worlds(X, H, world, monkeypatch):
    """Worlds with 30 % undefined bytes and 1 % A holes, so that most chunks
    are listed, and list capacities chosen so that only the host region's
    index fits, only the pool's, or both: every record equals the oracle,
    whichever of its spaces are indexed."""
    monkeypatch.setenv("XC_REORDER_MIN", "1")
    monkeypatch.setenv("XC_SHADOW_INDEX", "2")
    rng = np.random.default_rng(62)
    if world == "pool-fits":
        hl, hv, a, bases, sizes, vs = util.random_world(rng, hl=400_003, nalloc=4, max_size=20_000, dens=0.3)
    else:
        hl, hv, a, bases, sizes, vs = util.random_world(rng, hl=100_003, nalloc=6, max_size=200_000, dens=0.3)
    a = (rng.random(hl) > 0.01).astype(np.uint8)
    hu, hn = faulty_chunks(hv, a)
    pool_u = sum(int(((v != 0)[: (v.size // 16) * 16].reshape(-1, 16).any(1)).sum()) for v in vs)
    host = max(hu, hn)
    if world == "host-fits":
        assert pool_u > 2 * host
        cap = (host + pool_u) // 2
    elif world == "pool-fits":
        assert host > 2 * pool_u
        cap = (host + pool_u) // 2
    else:
        cap = 1 << 20
    monkeypatch.setenv("XC_SIDX_CAP", str(cap))
    recs = util.random_records(rng, W.HOST_BASE, hl, bases, sizes, 2000, max_n=50_000)
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, recs)
    want = util.oracle_for(w).run(recs)
    dw = H.DeviceWorld(w)
    try:
        for mode in (X.CG_CHECK, X.CG_CHECK | X.CG_EAGER):
            util.assert_verdicts_equal(dw.check(recs, mode), want, f"{world} mode {mode}")
    finally:
        dw.close()


@pytest.mark.parametrize("order", ["segments", "given-order"])
def test_shadow_index_reads_marked_steps(X, H, order, monkeypatch):
    """The indexes list and read only the 64 KiB steps of V that the batch's
    records read: in a world dense with faults whose records each touch a
    few of its steps, every verdict equals the oracle's, batch after batch
    (each batch's marks are cleared for the next); a batch confined to one
    allocation and one host window reads at most those steps (the byte counts
    of cg_index_ms)."""
    monkeypatch.setenv("XC_REORDER_MIN", "1" if order == "segments" else str(1 << 40))
    monkeypatch.setenv("XC_SHADOW_INDEX", "2")
    rng = np.random.default_rng(64)
    hl, hv, a, bases, sizes, vs = util.random_world(rng, hl=(4 << 20) + 5, nalloc=8, max_size=3 << 20, dens=0.02)
    a = (rng.random(hl) > 1e-3).astype(np.uint8)
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, np.zeros(0, W.RECORD_DTYPE))
    o = util.oracle_for(w)
    step = 1 << 16
    dw = H.DeviceWorld(w)
    try:
        X.cg_index_ms(dw.ctx)
        for k in range(3):
            recs = util.random_records(rng, W.HOST_BASE, hl, bases, sizes, 1500, max_n=20_000)
            util.assert_verdicts_equal(dw.check(recs), o.run(recs), f"{order} batch {k}")
        _, _, (host_read, pool_read) = X.cg_index_ms(dw.ctx)
        assert 0 < pool_read <= 3 * (int(sizes.sum()) + len(sizes) * step)
        assert 0 < host_read <= 3 * (hl + step) * 18 // 16
        # one allocation and one host window of 100 KiB
        j = int(np.argmax(sizes))
        x0 = int(rng.integers(0, hl - 100_000))
        recs = np.zeros(1000, W.RECORD_DTYPE)
        for i in range(recs.size):
            n = int(rng.integers(1, 5000))
            if i % 2:
                recs[i] = (W.HOST_BASE + x0 + int(rng.integers(0, 100_000 - n)), int(bases[j]) +
                           int(rng.integers(0, int(sizes[j]) - n)), n, X.CG_H2D, 0)
            else:
                recs[i] = (int(bases[j]) + int(rng.integers(0, int(sizes[j]) - n)),
                           W.HOST_BASE + x0 + int(rng.integers(0, 100_000 - n)), n, X.CG_D2H, 0)
        util.assert_verdicts_equal(dw.check(recs), o.run(recs), f"{order} confined batch")
        _, _, (host_read, pool_read) = X.cg_index_ms(dw.ctx)
        assert 0 < pool_read <= (int(sizes[j]) // step + 2) * step, (pool_read, int(sizes[j]))
        assert 0 < host_read <= (100_000 // step + 2) * step * 18 // 16, host_read
    finally:
        dw.close()


def test_shadow_index_after_frees(X, H, monkeypatch):
    """The indexes are rebuilt from the shadow as it is at each check: after
    frees, fresh allocations (one in a freed block's pool slot, whose bytes
    past the new size keep the old shadow), and partial writes, a second
    batch (with pointers into freed allocations) equals the oracle on the new
    state, as the first did on the old."""
    monkeypatch.setenv("XC_REORDER_MIN", "1")
    monkeypatch.setenv("XC_SHADOW_INDEX", "2")
    rng = np.random.default_rng(63)
    hl, hv, a, bases, sizes, vs = util.random_world(rng, hl=300_000, nalloc=6, max_size=100_000, dens=0.01)
    recs = util.random_records(rng, W.HOST_BASE, hl, bases, sizes, 600, max_n=40_000)
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, recs)
    dw = H.DeviceWorld(w, pool_slack=1 << 20)
    try:
        util.assert_verdicts_equal(dw.check(recs), util.oracle_for(w).run(recs), "before")
        # free two allocations; allocate one smaller at the first freed base
        # (its pool slot may be the freed one), and one past the last
        freed = [1, 3]
        for j in freed:
            X.shadow_free(dw.ctx, int(bases[j]))
        torch.cuda.synchronize()
        X.cg_sync(dw.ctx)
        nb = [int(bases[1]), int(bases[-1]) + int(sizes[-1]) + 4096]
        ns = [int(sizes[1]) // 2 + 1, 50_000]
        for b, z in zip(nb, ns):
            X.shadow_alloc(dw.ctx, b, z)
        # define the second half of each new allocation
        nv = []
        for b, z in zip(nb, ns):
            X.shadow_set(dw.ctx, b + z // 2, z - z // 2, 0)
            v = np.full(z, 0xFF, np.uint8)
            v[z // 2:] = 0
            nv.append(v)
        keep = [j for j in range(bases.size) if j not in freed]
        b2 = np.array(sorted([int(bases[j]) for j in keep] + nb), np.uint64)
        order = {int(bases[j]): (int(sizes[j]), vs[j]) for j in keep}
        order.update({b: (z, v) for b, z, v in zip(nb, ns, nv)})
        s2 = np.array([order[int(b)][0] for b in b2], np.uint64)
        v2 = [order[int(b)][1] for b in b2]
        recs2 = np.concatenate([util.random_records(rng, W.HOST_BASE, hl, b2, s2, 500, max_n=40_000),
                                util.random_records(rng, W.HOST_BASE, hl, bases[freed], sizes[freed], 100,
                                                    max_n=5_000)])
        w2 = util.workload_from_arrays(W.HOST_BASE, hv, a, b2, s2, v2, recs2)
        util.assert_verdicts_equal(dw.check(recs2), util.oracle_for(w2).run(recs2), "after frees")
    finally:
        dw.close()
