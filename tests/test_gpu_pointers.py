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
        gpu_check(X, ctx, b.ptrs[:16])   # the table is on the device, so the frees below are merged
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


def test_table_merges_at_full_size(X):
    """The device table at 975,000 entries after 30 rounds of frees and new
    allocations, each round made into a new version by the device merge (the
    list is updated on every allocation and free, Sec. 2 / Fig. 2 caption):
    every base, end, shadow offset and top-level entry read back equals the
    host's sorted list, and sampled lookups equal the oracle's."""
    b = W.pointer_batch()
    ctx = make_ctx(X, b.bases, b.sizes)
    rng = np.random.default_rng(77)
    try:
        gpu_check(X, ctx, b.ptrs[:16])                      # first version: a full upload
        full0 = X.cg_table_read(ctx, b.bases.size + 16)["full_uploads"]
        live = {int(x): int(z) for x, z in zip(b.bases, b.sizes)}
        freed = []
        for r in range(30):
            keys = np.array(sorted(live), np.uint64)
            kill = np.sort(rng.choice(keys.size, 2000, replace=False))
            X.shadow_free_batch(ctx, keys[kill])
            for k in keys[kill]:
                freed.append((int(k), live.pop(int(k))))
            # re-allocate earlier freed blocks at their base, with a size no larger
            rng.shuffle(freed)
            take, freed = freed[:1500], freed[1500:]
            nb = np.array([f[0] for f in take], np.uint64)
            ns = np.array([max(1, int(rng.integers(1, f[1] + 1))) for f in take], np.uint64)
            X.shadow_alloc_batch(ctx, nb, ns)
            live.update({int(x): int(z) for x, z in zip(nb, ns)})
            if r % 3 == 2:
                gpu_check(X, ctx, b.ptrs[r * 1000:(r + 1) * 1000])   # a check makes the version
            if r % 10 == 9:
                t = X.cg_table_read(ctx, len(live) + 16)
                keys = np.array(sorted(live), np.uint64)
                sizes = np.array([live[int(k)] for k in keys], np.uint64)
                assert np.array_equal(t["base"], keys), f"round {r}: bases"
                assert np.array_equal(t["end"], keys + sizes), f"round {r}: ends"
                top = t["base"][:: 1 << t["shift"]]
                assert t["top"].size <= 1024 and np.array_equal(t["top"], top), f"round {r}: top level"
                # shadow slots: 256-byte aligned, disjoint, and where shadow_ptr says
                o = t["off"]
                order = np.argsort(o)
                assert (o % 256 == 0).all()
                assert (o[order][:-1] + (sizes[order][:-1] + 255) // 256 * 256 <= o[order][1:]).all()
                for j in rng.choice(keys.size, 3000, replace=False):
                    assert X.shadow_ptr(ctx, int(keys[j])) == t["pool"] + int(o[j])
        # every version after the first was a device merge
        assert t["full_uploads"] == full0 and t["merges"] >= 10, (t["merges"], t["full_uploads"], full0)
        keys = np.array(sorted(live), np.uint64)
        sizes = np.array([live[int(k)] for k in keys], np.uint64)
        idx = np.sort(rng.choice(b.ptrs.size, 3000, replace=False))
        probe = np.concatenate([b.ptrs[idx], keys[:500], keys[:500] + sizes[:500], np.array([f[0] for f in freed[:500]],
                                                                                          np.uint64)])
        assert same(gpu_check(X, ctx, probe), oracle.pointers(keys, sizes, probe))
    finally:
        X.cg_destroy(ctx)
