"""check_transfers_2d (pitched 2D copies, the strided copies of the footnote
to Sec. 2's error list) on the GPU against the oracle: the closed-form pins,
random 2D batches through the no-wait path (rows stepped on the device) and
the expanded path (CG_PLAIN), wide rows worked by whole waves, check +
propagate on conflict-free batches with every shadow byte compared, the row
limit, and a captured call replayed."""
import numpy as np
import pytest

from oracle import oracle
from paper_1310_0901_amd import workloads as W
from tests import util
from tests.test_oracle_2d import pins

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def X():
    from paper_1310_0901_amd import xfercheck
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    xfercheck.lib()
    return xfercheck


@pytest.fixture(scope="module")
def H():
    from paper_1310_0901_amd import harness
    return harness


@pytest.fixture(params=["index-when-it-pays", "index-always"])
def index_mode(request, monkeypatch):
    """Shadow indexes for records whose rows follow row 0 (worked as one
    transfer, or row by row from the entries of their span): built when they
    pay (these small batches: rarely), or for every check."""
    monkeypatch.setenv("XC_SHADOW_INDEX", "2" if request.param == "index-always" else "1")
    return request.param


def check2d(X, dw, recs2d, mode):
    r = np.ascontiguousarray(recs2d, W.RECORD2D_DTYPE)
    rt = torch.from_numpy(r.view(np.uint8).copy()).to("cuda:0")
    out = torch.full((r.size * 32,), 0xAB, dtype=torch.uint8, device="cuda:0")
    s = torch.cuda.current_stream()
    X.check_transfers_2d(dw.ctx, rt.data_ptr(), r.size, out.data_ptr(), mode, s.cuda_stream)
    s.synchronize()
    return out.cpu().numpy().view(W.VERDICT_DTYPE).copy()


def random_2d(rng, hb, hl, bases, sizes, count):
    """2D copies whose rows start inside or near the host region and the
    allocations; pitches equal to, above and below the width."""
    out = np.zeros(count, W.RECORD2D_DTYPE)
    for i in range(count):
        kind = int(rng.choice([0, 1, 2, 5], p=[0.4, 0.3, 0.28, 0.02]))
        width = int(rng.integers(0, 3000)) if rng.random() > 0.05 else 0
        rows = int(rng.integers(0, 12))
        pitch = lambda: int(rng.choice([width, width + int(rng.integers(1, 500)), max(0, width - int(rng.integers(1, 50)))]))

        def hostp():
            return hb + int(rng.integers(-100, hl + 100)) if rng.random() < 0.1 else hb + int(rng.integers(0, hl))

        def devp():
            j = int(rng.integers(0, bases.size))
            return int(bases[j]) + int(rng.integers(-20, int(sizes[j]) + 20))
        src = hostp() if kind == 0 else devp()
        dst = hostp() if kind == 1 else devp()
        out[i] = (src, dst, width, rows, pitch(), pitch(), kind, (0, 0, 0))
    return out


def world_from_state(st):
    a = np.ones(st.hl, np.uint8)
    bits = np.unpackbits(st.ha.view(np.uint8), bitorder="little")[:st.hl]
    a[:] = bits
    return util.workload_from_arrays(st.hb, st.hv, a, st.bases, st.sizes, st.vs, np.zeros(0, W.RECORD_DTYPE))


def test_pins(X, H):
    for i, (st, r, want) in enumerate(pins()):
        dw = H.DeviceWorld(world_from_state(st))
        try:
            v = check2d(X, dw, r, X.CG_CHECK)[0]
            assert (int(v["flags"]), int(v["first_bad"]), int(v["undef_bytes"]), int(v["avail"])) == want, i
        finally:
            dw.close()


@pytest.mark.parametrize("seed", range(4))
def test_random_check(X, H, seed, index_mode):
    rng = np.random.default_rng(700 + seed)
    hl, hv, a, bases, sizes, vs = util.random_world(rng, dens=0.01)
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, np.zeros(0, W.RECORD_DTYPE))
    recs = random_2d(rng, W.HOST_BASE, hl, bases, sizes, 300)
    want = util.oracle_for(w).run2d(recs)
    dw = H.DeviceWorld(w)
    try:
        for mode in (X.CG_CHECK, X.CG_CHECK | X.CG_EAGER, X.CG_CHECK | X.CG_PLAIN):
            util.assert_verdicts_equal(check2d(X, dw, recs, mode), want, f"seed {seed} mode {mode}")
        # a smaller batch on the same stream after the larger one, and single records
        util.assert_verdicts_equal(check2d(X, dw, recs[:7], X.CG_CHECK), want[:7], "prefix")
        for k in (0, 5, 299):
            util.assert_verdicts_equal(check2d(X, dw, recs[k:k + 1], X.CG_CHECK), want[k:k + 1], f"record {k}")
    finally:
        dw.close()


@pytest.mark.parametrize("seed", range(3))
def test_random_propagate(X, H, seed):
    """Conflict-free sets (rows of all records together), check + propagate:
    verdicts and every shadow byte equal the oracle's."""
    rng = np.random.default_rng(800 + seed)
    hl, hv, a, bases, sizes, vs = util.random_world(rng, dens=0.02, nalloc=10, max_size=200_000)
    cand = random_2d(rng, W.HOST_BASE, hl, bases, sizes, 200)
    keep = []
    for i in range(cand.size):
        rows, _, _ = oracle.expand_rows(cand[keep + [i]])
        if len(util.conflict_free(rows, W.HOST_BASE, hl, bases, sizes)) == rows.size:
            keep.append(i)
    recs = cand[keep]
    assert recs.size >= 3
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, np.zeros(0, W.RECORD_DTYPE))
    o = util.oracle_for(w)
    want = o.run2d(recs, propagate=True)
    dw = H.DeviceWorld(w)
    try:
        got = check2d(X, dw, recs, X.CG_CHECK | X.CG_PROPAGATE | X.CG_DEBUG_CONFLICTS)
        util.assert_verdicts_equal(got, want, f"seed {seed}")
        for j in range(bases.size):
            assert np.array_equal(dw.alloc_shadow(bases[j], sizes[j]), o.vs[j]), f"allocation {j}"
        assert np.array_equal(dw.host_shadow(), o.hv), "host region shadow"
    finally:
        dw.close()
    # the same through the no-wait path (rows stepped on the device)
    dw = H.DeviceWorld(w)
    try:
        got = check2d(X, dw, recs, X.CG_CHECK | X.CG_PROPAGATE)
        util.assert_verdicts_equal(got, want, f"seed {seed}, rows stepped on the device")
        for j in range(bases.size):
            assert np.array_equal(dw.alloc_shadow(bases[j], sizes[j]), o.vs[j]), f"allocation {j}"
        assert np.array_equal(dw.host_shadow(), o.hv), "host region shadow"
    finally:
        dw.close()


def wide_2d(rng, hb, hl, bases, sizes, count):
    """2D copies of 1-9 KiB rows (whole-wave work per row), most of them with
    every row inside one allocation or the host region (rows that follow row
    0), some running past it, at pitches equal to and above the width."""
    out = np.zeros(count, W.RECORD2D_DTYPE)
    for i in range(count):
        kind = int(rng.choice([0, 1, 2]))
        width = int(rng.integers(1024, 9 * 1024))
        rows = int(rng.integers(1, 40))
        sp, dp = (width + int(rng.choice([0, 0, 16, 37, 512])) for _ in range(2))
        if kind == 2 and rng.random() < 0.5:
            dp = sp
        inside = rng.random() < 0.8

        def place(host, pitch):
            span = (rows - 1) * pitch + width
            if host:
                room = hl - span
                return hb + (int(rng.integers(0, room + 1)) if inside and room >= 0 else int(rng.integers(0, hl)))
            j = int(rng.integers(0, bases.size))
            room = int(sizes[j]) - span
            if inside and room >= 0:
                return int(bases[j]) + int(rng.integers(0, room + 1))
            return int(bases[j]) + int(rng.integers(0, int(sizes[j])))
        out[i] = (place(kind == 0, sp), place(kind == 1, dp), width, rows, sp, dp, kind, (0, 0, 0))
    return out


@pytest.mark.parametrize("seed", range(3))
def test_wide_rows(X, H, seed, index_mode):
    """Rows of 1-9 KiB: check on the no-wait path and the expanded path, both
    against the oracle; then check + propagate of a conflict-free subset on
    the no-wait path with every shadow byte compared."""
    rng = np.random.default_rng(900 + seed)
    hl, hv, a, bases, sizes, vs = util.random_world(rng, hl=2 << 20, nalloc=6, max_size=1 << 20,
                                                     dens=[1e-4, 0.01, 0.0][seed])
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, np.zeros(0, W.RECORD_DTYPE))
    recs = wide_2d(rng, W.HOST_BASE, hl, bases, sizes, 400)
    want = util.oracle_for(w).run2d(recs)
    dw = H.DeviceWorld(w)
    try:
        for mode in (X.CG_CHECK, X.CG_CHECK | X.CG_PLAIN):
            util.assert_verdicts_equal(check2d(X, dw, recs, mode), want, f"seed {seed} mode {mode}")
    finally:
        dw.close()
    keep = []
    for i in range(recs.size):
        rows, _, _ = oracle.expand_rows(recs[keep + [i]])
        if len(util.conflict_free(rows, W.HOST_BASE, hl, bases, sizes)) == rows.size:
            keep.append(i)
    sub = recs[keep]
    assert sub.size >= 10
    o = util.oracle_for(w)
    want = o.run2d(sub, propagate=True)
    dw = H.DeviceWorld(w)
    try:
        util.assert_verdicts_equal(check2d(X, dw, sub, X.CG_CHECK | X.CG_PROPAGATE), want, f"seed {seed} propagate")
        for j in range(bases.size):
            assert np.array_equal(dw.alloc_shadow(bases[j], sizes[j]), o.vs[j]), f"allocation {j}"
        assert np.array_equal(dw.host_shadow(), o.hv), "host region shadow"
    finally:
        dw.close()


def spans_apart(recs):
    """Greedy subset of 2D records (each with pitches at or above its width)
    whose written address span, first row to last, meets no other kept
    record's read or written span, nor its own read span: a conflict-free
    batch, since disjoint addresses have disjoint shadow bytes."""
    keep, reads, writes = [], [], []

    def span(p, pitch, r):
        return (int(r["rows"]) - 1) * pitch + int(r["width"])

    def meets(a, lst):
        return any(a[0] < y and x < a[1] for x, y in lst)
    for i, r in enumerate(recs):
        rs = (int(r["src"]), int(r["src"]) + span(r["src"], int(r["spitch"]), r))
        ws = (int(r["dst"]), int(r["dst"]) + span(r["dst"], int(r["dpitch"]), r))
        if meets(ws, reads) or meets(ws, writes) or meets(rs, writes) or meets(ws, [rs]):
            continue
        keep.append(i)
        reads.append(rs)
        writes.append(ws)
    return recs[keep]


def step_2d(rng, hb, hl, bases, sizes, count):
    """2D copies at pitches that are multiples of 16 (each row keeps row 0's
    16-byte phase), rows of 1 byte to 5 KB, 1-300 rows, nearly all inside one
    allocation or the host region on each side; a third with rows back to
    back (pitch = width, a multiple of 16) on the source side, and on the
    destination side too for half of those."""
    out = np.zeros(count, W.RECORD2D_DTYPE)
    for i in range(count):
        kind = int(rng.choice([0, 1, 2]))
        width = int(rng.choice([int(rng.integers(1, 64)), int(rng.integers(64, 5000))]))
        rows = int(rng.integers(1, 300))
        sp, dp = ((width + 15) // 16 * 16 + 16 * int(rng.choice([0, 0, 1, 5])) for _ in range(2))
        if kind == 2 and rng.random() < 0.5:
            dp = sp
        if rng.random() < 1 / 3:
            width = 16 * int(rng.integers(1, 300))
            sp = width
            dp = width if rng.random() < 0.5 else width + 16 * int(rng.integers(1, 4))

        def place(host, pitch):
            span = (rows - 1) * pitch + width
            if host:
                room = hl - span
                return hb + int(rng.integers(0, room + 1)) if room >= 0 and rng.random() < 0.95 else hb + int(rng.integers(0, hl))
            j = int(rng.integers(0, bases.size))
            room = int(sizes[j]) - span
            if room >= 0 and rng.random() < 0.95:
                return int(bases[j]) + int(rng.integers(0, room + 1))
            return int(bases[j]) + int(rng.integers(0, int(sizes[j])))
        out[i] = (place(kind == 0, sp), place(kind == 1, dp), width, rows, sp, dp, kind, (0, 0, 0))
    return out


@pytest.mark.parametrize("seed", range(3))
def test_step_rows(X, H, seed, index_mode):
    """Rows at pitches that keep the 16-byte phase, worked with several rows
    per wave iteration: check (host A holes included, so device->host rows
    meet unaddressable destination bytes) against the oracle, on the no-wait
    and expanded paths; then check + propagate of a conflict-free subset with
    every shadow byte compared."""
    rng = np.random.default_rng(950 + seed)
    hl, hv, a, bases, sizes, vs = util.random_world(rng, hl=4 << 20, nalloc=8, max_size=2 << 20,
                                                     dens=[1e-4, 0.01, 0.001][seed])
    a = (rng.random(hl) > 2e-4).astype(np.uint8)
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, np.zeros(0, W.RECORD_DTYPE))
    recs = step_2d(rng, W.HOST_BASE, hl, bases, sizes, 300)
    want = util.oracle_for(w).run2d(recs)
    assert (want["flags"] & X.CG_DST_UNADDR).any() and (want["flags"] & X.CG_SRC_UNDEF).any()
    dw = H.DeviceWorld(w)
    try:
        for mode in (X.CG_CHECK, X.CG_CHECK | X.CG_PLAIN):
            util.assert_verdicts_equal(check2d(X, dw, recs, mode), want, f"seed {seed} mode {mode}")
    finally:
        dw.close()
    sub = spans_apart(recs)
    assert sub.size >= 20
    o = util.oracle_for(w)
    want = o.run2d(sub, propagate=True)
    dw = H.DeviceWorld(w)
    try:
        util.assert_verdicts_equal(check2d(X, dw, sub, X.CG_CHECK | X.CG_PROPAGATE), want, f"seed {seed} propagate")
        for j in range(bases.size):
            assert np.array_equal(dw.alloc_shadow(bases[j], sizes[j]), o.vs[j]), f"allocation {j}"
        assert np.array_equal(dw.host_shadow(), o.hv), "host region shadow"
    finally:
        dw.close()


def inside_2d(rng, hb, hl, bases, sizes, count):
    """2D copies whose rows all lie inside one allocation or the host region
    on each side (so their rows follow row 0), at pitches that make rows
    coincide (0), overlap (below the width), sit closer than a chunk (1-15),
    touch (the width) or leave gaps of any phase; widths of 1-200 bytes."""
    out = np.zeros(count, W.RECORD2D_DTYPE)
    i = 0
    while i < count:
        kind = int(rng.choice([0, 1, 2]))
        width = int(rng.integers(1, 200))
        rows = int(rng.integers(1, 150))

        def pitch():
            return int(rng.choice([0, int(rng.integers(1, 16)), max(1, width - int(rng.integers(1, 40))), width,
                                   width + int(rng.integers(1, 40)), 16 * int(rng.integers(1, 20))]))
        sp, dp = pitch(), pitch()
        if kind == 2 and rng.random() < 0.5:
            dp = sp

        def place(host, q):
            span = (rows - 1) * q + width
            if host:
                return hb + int(rng.integers(0, hl - span + 1)) if span <= hl else None
            j = int(rng.integers(0, bases.size))
            return int(bases[j]) + int(rng.integers(0, int(sizes[j]) - span + 1)) if span <= int(sizes[j]) else None
        s_, d_ = place(kind == 0, sp), place(kind == 1, dp)
        if s_ is None or d_ is None:
            continue
        out[i] = (s_, d_, width, rows, sp, dp, kind, (0, 0, 0))
        i += 1
    return out


@pytest.mark.parametrize("seed", range(3))
def test_rows_from_index(X, H, seed, index_mode):
    """Records whose rows follow row 0, in worlds dense with undefined and
    unaddressable bytes: the index maps its entries onto rows that coincide,
    overlap, sit closer than a chunk or leave gaps; every verdict equals the
    oracle's (and the expanded path's)."""
    rng = np.random.default_rng(970 + seed)
    hl, hv, a, bases, sizes, vs = util.random_world(rng, hl=1 << 20, nalloc=8, max_size=1 << 19,
                                                     dens=[0.05, 0.002, 0.3][seed])
    a = (rng.random(hl) > [0.01, 1e-3, 0.05][seed]).astype(np.uint8)
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, np.zeros(0, W.RECORD_DTYPE))
    recs = inside_2d(rng, W.HOST_BASE, hl, bases, sizes, 600)
    want = util.oracle_for(w).run2d(recs)
    for f in (X.CG_SRC_UNDEF, X.CG_SRC_UNADDR, X.CG_DST_UNADDR):
        assert (want["flags"] & f).any(), f
    assert seed == 2 or (want["flags"] == 0).any()
    dw = H.DeviceWorld(w)
    try:
        for mode in (X.CG_CHECK, X.CG_CHECK | X.CG_PLAIN):
            util.assert_verdicts_equal(check2d(X, dw, recs, mode), want, f"seed {seed} mode {mode}")
    finally:
        dw.close()


def test_sparse_rows_from_index(X, H, index_mode):
    """Rows far apart (a pitch of up to 1 MiB for rows of 1-64 bytes): the
    span from the first row to the last is many times the rows' bytes, so
    the index reads every step of the space for them instead of the steps of
    their span; mixed in one batch with records whose spans are marked step
    by step.  Every verdict equals the oracle's."""
    rng = np.random.default_rng(990)
    hl, hv, a, bases, sizes, vs = util.random_world(rng, hl=24 << 20, nalloc=4, max_size=12 << 20, dens=0.002)
    a = (rng.random(hl) > 1e-4).astype(np.uint8)
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, np.zeros(0, W.RECORD_DTYPE))
    recs = np.zeros(400, W.RECORD2D_DTYPE)
    i = 0
    while i < recs.size:
        kind = int(rng.choice([0, 1, 2]))
        width = int(rng.integers(1, 65))
        rows = int(rng.integers(2, 12))
        sp, dp = (int(rng.choice([int(rng.integers(256 << 10, 1 << 20)), width + int(rng.integers(0, 48))]))
                  for _ in range(2))

        def place(host, q):
            span = (rows - 1) * q + width
            if host:
                return W.HOST_BASE + int(rng.integers(0, hl - span + 1)) if span <= hl else None
            j = int(rng.integers(0, bases.size))
            return int(bases[j]) + int(rng.integers(0, int(sizes[j]) - span + 1)) if span <= int(sizes[j]) else None
        s_, d_ = place(kind == 0, sp), place(kind == 1, dp)
        if s_ is None or d_ is None:
            continue
        recs[i] = (s_, d_, width, rows, sp, dp, kind, (0, 0, 0))
        i += 1
    assert ((recs["spitch"] >= 256 << 10) | (recs["dpitch"] >= 256 << 10)).sum() > 100
    want = util.oracle_for(w).run2d(recs)
    assert (want["flags"] != 0).any() and (want["flags"] == 0).any()
    dw = H.DeviceWorld(w)
    try:
        for mode in (X.CG_CHECK, X.CG_CHECK | X.CG_PLAIN):
            util.assert_verdicts_equal(check2d(X, dw, recs, mode), want, f"mode {mode}")
    finally:
        dw.close()


def test_captured_call_replays(X, H):
    """check_transfers_2d captured in a graph (after one call of that size on
    the stream) and replayed several times, with other eager work and
    synchronisations between the replays: every replay equals the eager call."""
    rng = np.random.default_rng(31)
    hl, hv, a, bases, sizes, vs = util.random_world(rng, hl=1 << 20, nalloc=6, max_size=1 << 20, dens=0.01)
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, np.zeros(0, W.RECORD_DTYPE))
    recs = np.concatenate([wide_2d(rng, W.HOST_BASE, hl, bases, sizes, 100),
                           random_2d(rng, W.HOST_BASE, hl, bases, sizes, 200)])
    want = util.oracle_for(w).run2d(recs)
    dw = H.DeviceWorld(w)
    try:
        side = torch.cuda.Stream()
        r = np.ascontiguousarray(recs, W.RECORD2D_DTYPE)
        rt = torch.from_numpy(r.view(np.uint8).copy()).to("cuda:0")
        out = torch.full((r.size * 32,), 0xAB, dtype=torch.uint8, device="cuda:0")
        torch.cuda.synchronize()
        X.check_transfers_2d(dw.ctx, rt.data_ptr(), r.size, out.data_ptr(), X.CG_CHECK, side.cuda_stream)
        side.synchronize()
        util.assert_verdicts_equal(out.cpu().numpy().view(W.VERDICT_DTYPE), want, "eager call")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=side):
            X.check_transfers_2d(dw.ctx, rt.data_ptr(), r.size, out.data_ptr(), X.CG_CHECK, side.cuda_stream)
        other = random_2d(rng, W.HOST_BASE, hl, bases, sizes, 50)
        want_other = util.oracle_for(w).run2d(other)
        for rep in range(3):
            out.fill_(0xAB)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            util.assert_verdicts_equal(out.cpu().numpy().view(W.VERDICT_DTYPE), want, f"replay {rep}")
            util.assert_verdicts_equal(check2d(X, dw, other, X.CG_CHECK), want_other, f"eager between {rep}")
        del g
    finally:
        dw.close()


def test_many_rows(X, H, index_mode):
    """One record of 200,000 rows and many small ones in one batch."""
    rng = np.random.default_rng(9)
    hl, hv, a, bases, sizes, vs = util.random_world(rng, hl=4 << 20, nalloc=4, max_size=3 << 20, dens=1e-4)
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, np.zeros(0, W.RECORD_DTYPE))
    recs = np.zeros(1001, W.RECORD2D_DTYPE)
    recs[0] = (W.HOST_BASE, int(bases[0]), 16, 200_000, 20, 16, 0, (0, 0, 0))
    recs[1:] = random_2d(rng, W.HOST_BASE, hl, bases, sizes, 1000)
    want = util.oracle_for(w).run2d(recs)
    dw = H.DeviceWorld(w)
    try:
        util.assert_verdicts_equal(check2d(X, dw, recs, X.CG_CHECK), want, "many rows")
    finally:
        dw.close()


def test_no_rows_and_errors(X, H):
    hl, hv, a, bases, sizes, vs = util.random_world(np.random.default_rng(1), nalloc=2)
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, np.zeros(0, W.RECORD_DTYPE))
    dw = H.DeviceWorld(w)
    try:
        recs = np.zeros(3, W.RECORD2D_DTYPE)
        recs[0] = (W.HOST_BASE, int(bases[0]), 0, 5, 0, 0, 0, (0, 0, 0))
        recs[1] = (W.HOST_BASE, int(bases[0]), 5, 0, 0, 0, 0, (0, 0, 0))
        recs[2] = (W.HOST_BASE, int(bases[0]), 0, 0, 0, 0, 9, (0, 0, 0))
        got = check2d(X, dw, recs, X.CG_CHECK)
        assert (got["flags"] == 0).all() and (got["first_bad"] == X.CG_NONE).all()
        assert (got["undef_bytes"] == 0).all() and (got["avail"] == 0).all()
        with pytest.raises(X.CgError) as e:
            X.check_transfers_2d(dw.ctx, 0, 1, 16, X.CG_CHECK, 0)
        assert e.value.status == X.CG_EINVAL
        # the expanded path: too many rows, also when the row counts would
        # wrap a 64-bit sum
        for tall in ([(1 << 64) - 1], [1 << 63, 1 << 63], [1 << 33]):
            t = np.zeros(len(tall), W.RECORD2D_DTYPE)
            for i, r in enumerate(tall):
                t[i] = (W.HOST_BASE, int(bases[0]), 1, r, 1, 1, 0, (0, 0, 0))
            tt = torch.from_numpy(t.view(np.uint8).copy()).to("cuda:0")
            vo = torch.zeros(len(tall) * 32, dtype=torch.uint8, device="cuda:0")
            with pytest.raises(X.CgError) as e:
                X.check_transfers_2d(dw.ctx, tt.data_ptr(), len(tall), vo.data_ptr(), X.CG_CHECK | X.CG_PLAIN,
                                     torch.cuda.current_stream().cuda_stream)
            assert e.value.status == X.CG_EINVAL, tall
        with pytest.raises(X.CgError) as e:
            X.check_transfers_2d(dw.ctx, 16, 1, 16, 0, 0)
        assert e.value.status == X.CG_EINVAL
    finally:
        dw.close()


def test_row_limit(X, H, index_mode):
    """The no-wait path works the rows below index 2^32 that start below byte
    2^62 of the copy and flags a record with more rows CG_ROWS_LIMIT; its
    other fields cover the rows worked.  Rows here repeat one row (pitch 0),
    so the expected verdict is that row's (from the oracle) scaled by the rows
    worked; a bogus width costs only what its rows can reach."""
    rng = np.random.default_rng(5)
    hl, hv, a, bases, sizes, vs = util.random_world(rng, hl=5000, nalloc=2, max_size=3000, dens=0.3)
    a[:] = 1
    w = util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, np.zeros(0, W.RECORD_DTYPE))
    o = util.oracle_for(w)
    undef_at = int(np.flatnonzero(hv)[0])
    cases = []
    # 2^33 one-byte rows reading one undefined host byte into one device byte (rows follow row 0)
    one = np.zeros(1, W.RECORD_DTYPE)
    one[0] = (W.HOST_BASE + undef_at, int(bases[0]), 1, 0, 0)
    cases.append(((W.HOST_BASE + undef_at, int(bases[0]), 1, 1 << 33, 0, 0, 0), o.run(one)[0], 1 << 32))
    # every row 2^50 bytes from the host region's start (past the region and the allocation): 2^12 rows worked
    n_eq = max(hl, int(sizes[0])) + 1   # a row of this length has the same verdict
    eq = np.zeros(1, W.RECORD_DTYPE)
    eq[0] = (W.HOST_BASE, int(bases[0]), n_eq, 0, 0)
    cases.append(((W.HOST_BASE, int(bases[0]), 1 << 50, (1 << 64) - 1, 0, 0, 0), o.run(eq)[0], 1 << 12))
    dw = H.DeviceWorld(w)
    try:
        for rec, row, worked in cases:
            r = np.zeros(1, W.RECORD2D_DTYPE)
            r[0] = rec + ((0, 0, 0),)
            v = check2d(X, dw, r, X.CG_CHECK)[0]
            got = (int(v["flags"]), int(v["first_bad"]), int(v["undef_bytes"]), int(v["avail"]))
            assert got == (int(row["flags"]) | X.CG_ROWS_LIMIT, int(row["first_bad"]),
                           worked * int(row["undef_bytes"]), int(row["avail"])), rec
    finally:
        dw.close()
