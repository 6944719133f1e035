"""check_transfers_2d (pitched 2D copies, the strided copies of the footnote
to Sec. 2's error list) on the GPU against the oracle: the closed-form pins,
random 2D batches on the graph, eager and plain paths, and check + propagate
on conflict-free batches with every shadow byte compared."""
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
def test_random_check(X, H, seed):
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


def test_many_rows(X, H):
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
        # too many rows, also when the row counts would wrap a 64-bit sum
        for tall in ([(1 << 64) - 1], [1 << 63, 1 << 63], [1 << 33]):
            t = np.zeros(len(tall), W.RECORD2D_DTYPE)
            for i, r in enumerate(tall):
                t[i] = (W.HOST_BASE, int(bases[0]), 1, r, 1, 1, 0, (0, 0, 0))
            tt = torch.from_numpy(t.view(np.uint8).copy()).to("cuda:0")
            vo = torch.zeros(len(tall) * 32, dtype=torch.uint8, device="cuda:0")
            with pytest.raises(X.CgError) as e:
                X.check_transfers_2d(dw.ctx, tt.data_ptr(), len(tall), vo.data_ptr(), X.CG_CHECK,
                                     torch.cuda.current_stream().cuda_stream)
            assert e.value.status == X.CG_EINVAL, tall
        with pytest.raises(X.CgError) as e:
            X.check_transfers_2d(dw.ctx, 16, 1, 16, 0, 0)
        assert e.value.status == X.CG_EINVAL
    finally:
        dw.close()
