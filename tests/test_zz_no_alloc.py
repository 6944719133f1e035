"""check_transfers_noalloc (the entry point for callers that cannot allocate)
against check_transfers on the same records, through the C ABI: two calls in
a row, the second with fewer records, check-only and check + propagate, and
the argument errors.  Bit-exact: verdicts and destination shadows are
integers."""
import numpy as np
import pytest

from paper_1310_0901_amd import workloads as W
from tests import util

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


def run(X, H, dw, recs, mode, noalloc):
    rt = H.records_tensor(recs, dw.dev)
    out = H.verdicts_tensor(len(recs), dw.dev)
    s = torch.cuda.current_stream(dw.dev).cuda_stream
    f = X.check_transfers_noalloc if noalloc else X.check_transfers
    f(dw.ctx, rt.data_ptr(), len(recs), out.data_ptr(), mode, s)
    torch.cuda.synchronize(dw.dev)
    return H.verdicts_np(out, len(recs))


def world(seed, n, conflict_free=False, **kw):
    rng = np.random.default_rng(seed)
    hl, hv, a, bases, sizes, vs = util.random_world(rng, **kw)
    recs = util.random_records(rng, W.HOST_BASE, hl, bases, sizes, n, max_n=40_000)
    if conflict_free:
        recs = util.conflict_free(recs, W.HOST_BASE, hl, bases, sizes)
    return util.workload_from_arrays(W.HOST_BASE, hv, a, bases, sizes, vs, recs), (hl, bases, sizes)


def test_noalloc_matches_check_transfers(X, H):
    w, _ = world(41, X.CG_NOALLOC_MAX)
    small = w.records[::7][:600].copy()
    want_all = util.oracle_for(w).run(w.records)
    dw = H.DeviceWorld(w)
    try:
        for recs, what in ((w.records, "full"), (small, "smaller, second call")):
            ref = run(X, H, dw, recs, X.CG_CHECK, False)
            got = run(X, H, dw, recs, X.CG_CHECK, True)
            util.assert_verdicts_equal(got, ref, f"noalloc vs check_transfers, {what}")
        util.assert_verdicts_equal(run(X, H, dw, w.records, X.CG_CHECK, True), want_all, "noalloc vs the oracle")
    finally:
        dw.close()


def test_noalloc_propagation_matches(X, H):
    w, (hl, bases, sizes) = world(43, 400, conflict_free=True, dens=0.02)
    cf = w.records
    assert len(cf) >= 3
    mode = X.CG_CHECK | X.CG_PROPAGATE
    shadows = {}
    for noalloc in (False, True):
        dw = H.DeviceWorld(w)
        try:
            v1 = run(X, H, dw, cf, mode, noalloc)
            v2 = run(X, H, dw, cf[: len(cf) // 3], mode, noalloc)   # a second, smaller call
            shadows[noalloc] = ([dw.alloc_shadow(bases[j], sizes[j]) for j in range(bases.size)], dw.host_shadow(),
                                v1, v2)
        finally:
            dw.close()
    ref, got = shadows[False], shadows[True]
    util.assert_verdicts_equal(got[2], ref[2], "propagate, first call")
    util.assert_verdicts_equal(got[3], ref[3], "propagate, second call")
    for j in range(bases.size):
        assert np.array_equal(got[0][j], ref[0][j]), f"allocation {j}"
    assert np.array_equal(got[1], ref[1]), "host region shadow"


def test_noalloc_argument_errors(X, H):
    w, _ = world(45, 8)
    dw = H.DeviceWorld(w)
    try:
        rt = H.records_tensor(w.records, dw.dev)
        out = H.verdicts_tensor(len(w.records), dw.dev)

        def status(count, mode, recs=rt.data_ptr(), o=out.data_ptr()):
            try:
                X.check_transfers_noalloc(dw.ctx, recs, count, o, mode, 0)
            except X.CgError as e:
                return e.status
            return X.CG_OK
        assert status(X.CG_NOALLOC_MAX + 1, X.CG_CHECK) == X.CG_EINVAL
        assert status(len(w.records), X.CG_CHECK | X.CG_PLAIN) == X.CG_EINVAL
        assert status(len(w.records), X.CG_CHECK | X.CG_DEBUG_CONFLICTS) == X.CG_EINVAL
        assert status(len(w.records), 0) == X.CG_EINVAL
        assert status(len(w.records), X.CG_CHECK, recs=0) == X.CG_EINVAL
        assert status(len(w.records), X.CG_CHECK, o=0) == X.CG_EINVAL
        assert status(0, X.CG_CHECK) == X.CG_OK
        torch.cuda.synchronize(dw.dev)
    finally:
        dw.close()
