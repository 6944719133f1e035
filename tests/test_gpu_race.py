"""The concurrent-access join (check_concurrent) on the GPU against the
oracle: flags element by element, and every named partner a record that
really conflicts with the one that names it.  Sizes span several sort and
sweep tiles with ragged tails; the full-size batch is checked on a sample
against the oracle and by properties on every record."""
import numpy as np
import pytest

from oracle import oracle
from paper_1310_0901_amd import workloads as W
from tests.test_oracle_race import PINS, random_batch
from tests.tiny import recs as tiny_recs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
NONE = (1 << 64) - 1


@pytest.fixture(scope="module")
def X():
    from paper_1310_0901_amd import xfercheck
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    xfercheck.lib()
    return xfercheck


@pytest.fixture(scope="module")
def ctx(X):
    c = X.cg_create(0, 1 << 16, 16)
    yield c
    X.cg_destroy(c)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.uint8).copy()).to("cuda:0")


def gpu_join(X, ctx, records, streams, epochs=None, stream=None):
    records = np.ascontiguousarray(records, W.RECORD_DTYPE)
    n = records.size
    if n == 0:
        return np.zeros(0, W.RACE_DTYPE)
    r, s = to_dev(records), to_dev(np.asarray(streams, np.uint32))
    e = None if epochs is None else to_dev(np.asarray(epochs, np.uint32))
    out = torch.full((n * 16,), 0xAB, dtype=torch.uint8, device="cuda:0")
    st = stream if stream is not None else torch.cuda.current_stream()
    X.check_concurrent(ctx, r.data_ptr(), s.data_ptr(), 0 if e is None else e.data_ptr(), n, out.data_ptr(),
                       st.cuda_stream)
    st.synchronize()
    return out.cpu().numpy().view(W.RACE_DTYPE).copy()


def meets(a, na, b, nb):
    return (na > 0) & (nb > 0) & (a < b + nb) & (b < a + na)


def partners_ok(res, records, streams, epochs):
    """Vectorised: every flagged record names a distinct record of another
    stream in its epoch that meets it the way its first flag says (the
    destination flag's partner when both are set); clean records name none."""
    f = res["flags"].astype(np.int64)
    p = res["partner"]
    flagged = (f & 3) != 0
    if not (p[~flagged] == NONE).all():
        return False
    idx = np.flatnonzero(flagged)
    if idx.size == 0:
        return True
    q = p[idx]
    if not (q < records.size).all():
        return False
    q = q.astype(np.int64)
    ep = np.zeros(records.size, np.uint32) if epochs is None else np.asarray(epochs, np.uint32)
    st = np.asarray(streams, np.uint32)
    ra, rb = records[idx], records[q]
    ok = (q != idx) & (st[q] != st[idx]) & (ep[q] == ep[idx]) & (rb["kind"] <= 2)
    A = lambda r, k: r[k].astype(object)
    na, nb = A(ra, "n"), A(rb, "n")
    dst_hit = meets(A(ra, "dst"), na, A(rb, "dst"), nb) | meets(A(ra, "dst"), na, A(rb, "src"), nb)
    src_hit = meets(A(ra, "src"), na, A(rb, "dst"), nb)
    want = np.where((f[idx] & 2) != 0, dst_hit, src_hit).astype(bool)
    return bool((ok & want).all())


def check(res, records, streams, epochs, want):
    assert np.array_equal(res["flags"].astype(np.int64), np.asarray(want, np.int64))
    assert (res["reserved"] == 0).all()
    assert partners_ok(res, records, streams, epochs)


def test_pins(X, ctx):
    for rows, st, ep, want in PINS:
        r = tiny_recs(rows)
        check(gpu_join(X, ctx, r, st, ep), r, st, ep, want)


@pytest.mark.parametrize("seed", range(6))
def test_random_tiny(X, ctx, seed):
    rng = np.random.default_rng(500 + seed)
    for _ in range(8):
        rows, st, ep = random_batch(rng, int(rng.integers(1, 60)), universe=int(rng.integers(20, 400)))
        r = tiny_recs(rows)
        want = oracle.race(r, st, ep)
        res = gpu_join(X, ctx, r, st, ep)
        check(res, r, st, ep, want)
        # the vectorised partner check agrees with the pair predicate of the oracle
        for a in np.flatnonzero(res["flags"] & 3):
            b = int(res["partner"][a])
            dh, sh = oracle.conflict(r[a], r[b], st[a], st[b], ep[a], ep[b])
            assert (dh if res["flags"][a] & 2 else sh)


@pytest.mark.parametrize("count,streams,epochs", [(20_000, 8, 4), (4097, 3, 1), (12_289, 2, 7), (1, 1, 1),
                                                  (2048, 64, 1), (30_000, 1, 3)])
def test_small_race(X, ctx, count, streams, epochs):
    b = W.small_race(count=count, streams=streams, epochs=epochs)
    want = oracle.race(b.records, b.streams, b.epochs, threads=8)
    res = gpu_join(X, ctx, b.records, b.streams, b.epochs)
    check(res, b.records, b.streams, b.epochs, want)
    if streams == 1:
        assert not (res["flags"] & 3).any()


@pytest.mark.parametrize("count,run", [(20_000, 4096), (20_000, 4097), (9000, 1), (12_289, 777), (4096, None),
                                       (4097, None), (30_000, "random"), (10_000, "decreasing")])
def test_epoch_runs(X, ctx, count, run):
    """Epochs that never decrease (a program's synchronisation windows), as
    runs of a fixed length (shifted so that runs cross the 4,096-record
    chunks), of random lengths up to 4,096, none (one epoch), or with one
    decrease: epochs of at most 4,096 records are sorted in LDS, anything
    else takes the radix sort; flags equal the oracle's either way and
    every partner is valid."""
    b = W.small_race(count=count, streams=8, epochs=1, seed=W.SEED0 + 40 + count % 97)
    rng = np.random.default_rng(count)
    if run is None:
        ep = None
    elif run == "random":
        lengths = rng.integers(1, 4097, size=count)
        ep = np.repeat(np.arange(count, dtype=np.uint32), lengths)[:count]
    elif run == "decreasing":
        ep = (np.arange(count) // 1000).astype(np.uint32)
        ep[count // 2:] -= 1
    else:
        ep = ((np.arange(count) + 2000) // run).astype(np.uint32)
    want = oracle.race(b.records, b.streams, ep, threads=8)
    res = gpu_join(X, ctx, b.records, b.streams, ep)
    check(res, b.records, b.streams, ep, want)
    assert (res["flags"] & 3).any() or run == 1


def test_epoch_runs_with_high_epochs(X, ctx):
    """The per-epoch path with epochs at and above 2^15, and up to 2^32 - 1,
    in the second half: every epoch is decided like any other."""
    count = 12_000
    b = W.small_race(count=count, streams=4, epochs=1, seed=W.SEED0 + 77)
    ep = (np.arange(count) // 1000).astype(np.uint32)
    ep[count // 2:] += (1 << 15) - 6
    ep[-1000:] = (1 << 32) - 1
    want = oracle.race(b.records, b.streams, ep, threads=8)
    res = gpu_join(X, ctx, b.records, b.streams, ep)
    check(res, b.records, b.streams, ep, want)
    assert (res["flags"][count // 2:] & 3).any() and (res["flags"][-1000:] & 3).any()
    assert ((res["flags"] & X.CG_RACE_UNCHECKED) != 0).sum() == (b.records["kind"] > 2).sum()


@pytest.mark.parametrize("seed", range(6))
def test_random_tiny_high(X, ctx, seed):
    """Tiny batches at the top of the address space (ranges above 2^48, up to
    the last byte and past 2^64) with epochs near 2^15, 2^31 and 2^32."""
    from tests.test_oracle_race import HIGH
    rng = np.random.default_rng(900 + seed)
    for j in range(8):
        rows, st, ep = random_batch(rng, int(rng.integers(1, 60)), epochs=3, **HIGH[(seed + j) % len(HIGH)])
        r = tiny_recs(rows)
        check(gpu_join(X, ctx, r, st, ep), r, st, ep, oracle.race(r, st, ep))


@pytest.mark.parametrize("shift,run", [(1 << 48, 1000), ((1 << 64) - (1 << 16), "decreasing"),
                                       (1 << 60, None), ((1 << 64) - (1 << 16), 3000)])
def test_high_addresses(X, ctx, shift, run):
    """A dense batch moved above 2^48 or to the top of the address space (its
    device ranges run past 2^64 there), on the per-epoch path (epoch runs
    of 1,000 or 3,000 records near 2^31) and the radix-sort path (decreasing
    epochs, or none at 5,000 records)."""
    count = 9000 if run is not None else 5000
    b = W.small_race(count=count, streams=6, epochs=1, seed=W.SEED0 + 91 + count)
    r = b.records.copy()
    # the host window goes 1 MiB below `shift`, the device window to `shift`
    for f in ("src", "dst"):
        a = r[f].astype(object)
        r[f] = [(x - W.HOST_BASE + shift - (1 << 20)) % (1 << 64) if x >= W.HOST_BASE else x - W.DEV_BASE + shift
                for x in a]
    if run is None:
        ep = None
    elif run == "decreasing":
        ep = ((1 << 32) - 1 - np.arange(count) // 700).astype(np.uint32)
    else:
        ep = ((1 << 31) + np.arange(count) // run).astype(np.uint32)
    want = oracle.race(r, b.streams, ep, threads=8)
    res = gpu_join(X, ctx, r, b.streams, ep)
    check(res, r, b.streams, ep, want)
    assert (res["flags"] & 3).any()


def test_no_epochs_argument(X, ctx):
    b = W.small_race(count=5000, epochs=1)
    want = oracle.race(b.records, b.streams, None, threads=8)
    check(gpu_join(X, ctx, b.records, b.streams, None), b.records, b.streams, None, want)


def test_edges(X, ctx):
    D, L = W.DEV_BASE, 1 << 48
    rng = np.random.default_rng(11)
    # every record writes the same 100 bytes: ties everywhere
    T = 9000
    r = W.make_records(np.zeros(T, np.int64), W.HOST_BASE + 128 * np.arange(T), np.full(T, D), np.full(T, 100))
    st = rng.integers(0, 5, T).astype(np.uint32)
    check(gpu_join(X, ctx, r, st), r, st, None, oracle.race(r, st, threads=8))
    # keys that differ only in their lowest byte: every other sort pass is skipped
    T = 256
    r = W.make_records(np.full(T, 2), D + np.arange(T), D + 1000 + np.arange(T), np.full(T, 3))
    st = (np.arange(T) % 2).astype(np.uint32)
    check(gpu_join(X, ctx, r, st), r, st, None, oracle.race(r, st))
    # ranges ending at and crossing 2^48; epochs 2^15 - 1 and 2^15, and epochs that differ above bit 15
    rows = [(0, W.HOST_BASE, L - 100, 100), (0, W.HOST_BASE + 500, L - 50, 50), (0, W.HOST_BASE, L - 50, 100),
            (2, D, D + 10_000, 64), (2, D + 10_000, D, 64), (1, D, W.HOST_BASE, 0), (7, D, D, 10)]
    r = tiny_recs([(k, s, d, n) for k, s, d, n in rows])
    for ep in ([0] * 7, [(1 << 15) - 1] * 7, [1 << 15] * 7, [300, 300, 300, 40000, 40000, 5, 5],
               [65535, 257, 257, 258, 258, 1, 1], [5, 5 + (1 << 15), 5, 5 + (1 << 16), 5, 5, 5],
               [(1 << 32) - 1] * 3 + [(1 << 31)] * 4):
        st = [1, 2, 3, 1, 2, 3, 4]
        check(gpu_join(X, ctx, r, st, ep), r, st, ep, oracle.race(r, st, ep))


def test_workspace_growth_and_streams(X, ctx):
    s2 = torch.cuda.Stream()
    for count in (100, 70_000, 5000, 70_001):
        b = W.small_race(seed=count, count=count, window=1 << 20)
        want = oracle.race(b.records, b.streams, b.epochs, threads=8)
        for st in (None, s2):
            check(gpu_join(X, ctx, b.records, b.streams, b.epochs, stream=st), b.records, b.streams, b.epochs, want)


def test_argument_errors(X, ctx):
    def status(*a):
        try:
            X.check_concurrent(ctx, *a)
        except X.CgError as e:
            return e.status
        return X.CG_OK
    assert status(0, 0, 0, 0, 0, 0) == X.CG_OK            # nothing to do
    assert status(0, 16, 0, 1, 16, 0) == X.CG_EINVAL      # null records
    assert status(16, 0, 0, 1, 16, 0) == X.CG_EINVAL      # null streams
    assert status(16, 16, 0, 1, 0, 0) == X.CG_EINVAL      # null results
    assert status(16, 16, 0, (1 << 30) + 1, 16, 0) == X.CG_EINVAL


def test_full_size_sampled(X, ctx):
    b = W.race_config()
    res = gpu_join(X, ctx, b.records, b.streams, b.epochs)
    assert partners_ok(res, b.records, b.streams, b.epochs)
    rng = np.random.default_rng(5)
    which = np.sort(rng.choice(b.records.size, 1500, replace=False))
    # flagged records near the end of an epoch and at the start of the next
    which = np.unique(np.concatenate([which, np.arange(4090, 4102), [b.records.size - 1]]))
    want = oracle.race(b.records, b.streams, b.epochs, which=which, threads=16)
    assert np.array_equal(res["flags"][which].astype(np.int64), want.astype(np.int64))
    # a partner's flags are never clean
    f = res["flags"]
    p = res["partner"][(f & 3) != 0].astype(np.int64)
    assert ((f[p] & 3) != 0).all()
    # the same join twice gives the same results (the choice of partner included)
    again = gpu_join(X, ctx, b.records, b.streams, b.epochs)
    assert np.array_equal(again, res)
