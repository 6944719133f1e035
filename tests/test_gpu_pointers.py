"""check_pointers (kernel-argument pointers, Sec. 5.1) on the GPU against the
oracle, bit-exact: the hand-derived pins, random tables with adjacent
allocations, a table changed by frees and new allocations between lookups,
and a 975,000-entry table with 1,000,000 pointers, sampled."""
import numpy as np
import pytest

from oracle import oracle
from paper_1310_0901_amd import workloads as W
from tests.test_oracle_pointers import ALLOCS, PINS, random_table

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def X():
    from paper_1310_0901_amd import xfercheck
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    xfercheck.lib()
    return xfercheck


def make_ctx(X, bases, sizes):
    pool = int(sum((int(z) + 255) // 256 * 256 for z in sizes)) + (1 << 20)
    ctx = X.cg_create(0, pool, len(bases) + 64)
    if len(bases):
        X.shadow_alloc_batch(ctx, bases, sizes)
    return ctx


def gpu_check(X, ctx, ptrs):
    p = np.ascontiguousarray(ptrs, np.uint64)
    if p.size == 0:
        return np.zeros(0, W.PTR_DTYPE)
    d = torch.from_numpy(p.view(np.uint8).copy()).to("cuda:0")
    out = torch.full((p.size * 24,), 0xAB, dtype=torch.uint8, device="cuda:0")
    s = torch.cuda.current_stream()
    X.check_pointers(ctx, d.data_ptr(), p.size, out.data_ptr(), s.cuda_stream)
    s.synchronize()
    return out.cpu().numpy().view(W.PTR_DTYPE).copy()


def same(got, want):
    return all(np.array_equal(got[f].astype(np.uint64), want[f].astype(np.uint64))
               for f in ("flags", "reserved", "base", "avail"))


def test_pins(X):
    # shifted into device address space; the pins' arithmetic is unchanged by the shift
    off = W.DEV_BASE
    bases = [b + off for b in sorted(ALLOCS)]
    sizes = [ALLOCS[b] for b in sorted(ALLOCS)]
    ctx = make_ctx(X, bases, sizes)
    try:
        ptrs = [p + off for p in PINS if p + off < (1 << 64)]
        got = gpu_check(X, ctx, ptrs)
        want = oracle.pointers(bases, sizes, ptrs)
        assert same(got, want)
        for p, g in zip(ptrs, got):
            f, b, a = PINS[p - off]
            assert (int(g["flags"]), int(g["base"]), int(g["avail"])) == (f, b + off if b else 0, a)
    finally:
        X.cg_destroy(ctx)


@pytest.mark.parametrize("seed", range(4))
def test_random_tables(X, seed):
    rng = np.random.default_rng(300 + seed)
    allocs, ptrs = random_table(rng, universe=5000, n=60)
    bases = [W.DEV_BASE + b for b in sorted(allocs)]
    sizes = [allocs[b] for b in sorted(allocs)]
    ptrs = [W.DEV_BASE + p for p in ptrs] + [0, 1, W.DEV_BASE - 1]
    ctx = make_ctx(X, bases, sizes)
    try:
        assert same(gpu_check(X, ctx, ptrs), oracle.pointers(bases, sizes, ptrs))
    finally:
        X.cg_destroy(ctx)


def test_table_changes_between_lookups(X):
    b = W.pointer_batch(n_alloc=20_000, n_ptrs=30_001)
    ctx = make_ctx(X, b.bases, b.sizes)
    try:
        assert same(gpu_check(X, ctx, b.ptrs), oracle.pointers(b.bases, b.sizes, b.ptrs))
        # free 1 %: pointers into them and one past them become unallocated
        X.shadow_free_batch(ctx, b.bases[b.freed])
        live = np.setdiff1d(np.arange(b.bases.size), b.freed)
        assert same(gpu_check(X, ctx, b.ptrs), oracle.pointers(b.bases[live], b.sizes[live], b.ptrs))
        # allocate them again with half the size
        half = np.maximum(b.sizes[b.freed] // 2, 1)
        X.shadow_alloc_batch(ctx, b.bases[b.freed], half)
        sizes = b.sizes.copy()
        sizes[b.freed] = half
        assert same(gpu_check(X, ctx, b.ptrs), oracle.pointers(b.bases, sizes, b.ptrs))
    finally:
        X.cg_destroy(ctx)


def test_empty_table_and_argument_errors(X):
    ctx = make_ctx(X, [], [])
    try:
        got = gpu_check(X, ctx, [0, W.DEV_BASE, (1 << 64) - 1])
        assert (got["flags"] == X.CG_PTR_UNALLOC).all() and (got["base"] == 0).all() and (got["avail"] == 0).all()
        for args in ((0, 1, 16, 0), (16, 1, 0, 0)):
            with pytest.raises(X.CgError) as e:
                X.check_pointers(ctx, *args)
            assert e.value.status == X.CG_EINVAL
        X.check_pointers(ctx, 0, 0, 0, 0)    # nothing to do
    finally:
        X.cg_destroy(ctx)


def test_full_table_sampled(X):
    b = W.pointer_batch()
    ctx = make_ctx(X, b.bases, b.sizes)
    try:
        X.shadow_free_batch(ctx, b.bases[b.freed])
        live = np.setdiff1d(np.arange(b.bases.size), b.freed)
        got = gpu_check(X, ctx, b.ptrs)
        rng = np.random.default_rng(1)
        idx = np.sort(rng.choice(b.ptrs.size, 1500, replace=False))
        assert same(got[idx], oracle.pointers(b.bases[live], b.sizes[live], b.ptrs[idx]))
        # properties on every pointer: a found base is a live allocation's, and avail fits in it
        ok = got["flags"] == 0
        pos = np.searchsorted(b.bases, got["base"][ok])
        assert (b.bases[pos] == got["base"][ok]).all()
        assert not np.isin(pos, b.freed).any()
        assert (got["avail"][ok] <= b.sizes[pos]).all()
        assert (got["base"][ok] + b.sizes[pos] - got["avail"][ok] == b.ptrs[ok]).all()
        assert ((got["base"][~ok] == 0) & (got["avail"][~ok] == 0)).all()
    finally:
        X.cg_destroy(ctx)
