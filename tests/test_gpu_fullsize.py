"""GPU parity at the benchmark workloads' full sizes, in the launch shape the
benchmark uses: every verdict against interval arithmetic over the sparse
description (or configuration 4's closed form), sampled records against the
byte-by-byte oracle, and the plain path against the batched one."""
import time

import numpy as np
import pytest

from paper_1310_0901_amd import workloads as W
from tests import intervals, util

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

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


def say(*a):
    print("[fullsize]", *a, flush=True)


def expected_all(w):
    f, fb, u, a = intervals.expected(w)
    out = np.zeros(w.count, W.VERDICT_DTYPE)
    out["flags"], out["first_bad"], out["undef_bytes"], out["avail"] = f, fb, u, a
    return out


def sample_idx(w, k, max_n):
    rng = np.random.default_rng(99)
    small = np.flatnonzero(w.records["n"] <= max_n)
    return np.sort(rng.choice(small, size=min(k, small.size), replace=False))


def test_config2_full_plain_and_batched(X, H):
    t0 = time.time()
    w = W.config2()
    hv, ha = W.host_v(w.host), W.host_a(w.host)
    dw = H.DeviceWorld(w, host_arrays=(hv, ha))
    say(f"config 2 set up in {time.time() - t0:.1f} s")
    try:
        want = expected_all(w)
        for name, mode in (("graph", X.CG_CHECK), ("plain", X.CG_CHECK | X.CG_PLAIN)):
            util.assert_verdicts_equal(dw.check(w.records, mode), want, f"config 2 {name}")
        # every record against the byte oracle, 256 records (and their
        # allocations' shadows) at a time, on 8 host threads
        for c0 in range(0, w.count, 256):
            part = w.records[c0:c0 + 256]
            o = util.oracle_subset(w, part, hv, ha)
            util.assert_verdicts_equal(o.run_threads(part, 8), want[c0:c0 + 256], f"config 2 oracle, from {c0}")
            del o
        say(f"config 2: all {w.count} records equal the oracle ({time.time() - t0:.1f} s)")
        idx = sample_idx(w, 40, 1 << 22)
        # propagation: every allocation receives its host source's V bytes,
        # 0xFF where the host byte is not addressable
        got = dw.check(w.records, X.CG_CHECK | X.CG_PROPAGATE)
        util.assert_verdicts_equal(got, want, "config 2 check+propagate")
        abits = np.unpackbits(ha.view(np.uint8), bitorder="little")
        for i in idx[:10]:
            r = w.records[i]
            off, n = int(r["src"]) - W.HOST_BASE, int(r["n"])
            exp = np.where(abits[off:off + n] == 1, hv[off:off + n], 0xFF).astype(np.uint8)
            assert np.array_equal(dw.alloc_shadow(int(r["dst"]), n), exp), i
    finally:
        dw.close()
    say(f"config 2 done in {time.time() - t0:.1f} s")


def test_config3_full_batched_plain_oracle(X, H):
    t0 = time.time()
    w = W.config3()
    hv, ha = W.host_v(w.host), W.host_a(w.host)
    dw = H.DeviceWorld(w, host_arrays=(hv, ha))
    say(f"config 3 set up in {time.time() - t0:.1f} s")
    try:
        import os
        cache = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                             "paper_1310_0901_amd", "tuning_cache.jsonl")
        rt = H.records_tensor(w.records)
        out = H.verdicts_tensor(w.count)
        s = torch.cuda.current_stream().cuda_stream
        X.cg_autotune(dw.ctx, rt.data_ptr(), w.count, out.data_ptr(), X.CG_CHECK, s, cache)
        want = expected_all(w)
        say(f"expected verdicts by interval arithmetic in {time.time() - t0:.1f} s")
        got = dw.check(w.records, X.CG_CHECK)
        util.assert_verdicts_equal(got, want, "config 3 batched")
        gp = dw.check(w.records, X.CG_CHECK | X.CG_PLAIN)
        util.assert_verdicts_equal(gp, want, "config 3 plain")
        say(f"batched and plain equal the interval verdicts ({time.time() - t0:.1f} s)")
        idx = np.arange(3000)
        o = util.oracle_subset(w, w.records[idx], hv, ha)
        util.assert_verdicts_equal(o.run(w.records[idx]), got[idx], "config 3 oracle sample")
        # injected labels
        lab = w.label
        assert np.all(got["flags"][lab == W.LABEL_UAF] & (X.CG_SRC_UNALLOC | X.CG_DST_UNALLOC))
        assert np.all(got["flags"][lab == W.LABEL_OVERRUN] & (X.CG_SRC_OVERRUN | X.CG_DST_OVERRUN))
    finally:
        dw.close()
    say(f"config 3 done in {time.time() - t0:.1f} s")


@pytest.mark.parametrize("pieces", [1, 4096])
def test_config4_full_chain(X, H, pieces):
    t0 = time.time()
    w = W.config4(pieces=pieces)
    hv = W.host_v(w.host)
    dw = H.DeviceWorld(w, host_arrays=(hv, W.host_a(w.host)))
    R, P = w.R, w.P
    b0 = [int(b) for r, b in zip(w.payload_records, w.payload_byte) if r == 0]
    try:
        for h, stage in enumerate(w.stages):
            got = dw.check(stage, X.CG_CHECK | X.CG_PROPAGATE)
            assert int(got["undef_bytes"].sum()) == 3 * R + P, h
            if pieces == 1:
                assert int(got["flags"][0]) == X.CG_SRC_UNDEF
                assert int(got["first_bad"][0]) == min([13] + b0)
            else:
                assert np.all(got["flags"] == X.CG_SRC_UNDEF)
                assert np.all(got["avail"] == stage["n"] + (w.host.length - (stage["src"] - stage["src"][0]) - stage["n"]))
                # each piece [a, b) of the region against its closed form
                und, first = intervals.piece_closed_form(w, stage)
                assert np.array_equal(got["undef_bytes"], und), h
                assert np.array_equal(got["first_bad"], first), h
        last = w.dev.live_idx[-1]
        dv = H.device_view(X.shadow_ptr(dw.ctx, int(w.dev.base[last])), w.host.length)
        assert torch.equal(dv, dw.hv[: w.host.length]), "final shadow differs from host V"
    finally:
        dw.close()
    say(f"config 4 ({pieces} pieces) done in {time.time() - t0:.1f} s")


def rows_and_expected(w, r2):
    """The row records of pitched 2D records (row r reads src + r*spitch and
    writes dst + r*dpitch, width bytes), the rows' verdicts by interval
    arithmetic, and one verdict per 2D record by the row-by-row numbering of
    its bytes (flags OR, smallest r*width + first_bad_r, undefined bytes
    summed, row 0's avail; no rows: {0, NONE, 0, 0})."""
    T = r2.size
    counts = np.where(r2["width"] > 0, r2["rows"], 0).astype(np.int64)
    rec = np.repeat(np.arange(T), counts)
    first = np.concatenate([[0], np.cumsum(counts)[:-1]])
    r = np.arange(int(counts.sum()), dtype=np.int64) - np.repeat(first, counts)
    rows = np.zeros(r.size, W.RECORD_DTYPE)
    rows["src"] = r2["src"][rec] + (r * r2["spitch"][rec].astype(np.int64)).astype(np.uint64)
    rows["dst"] = r2["dst"][rec] + (r * r2["dpitch"][rec].astype(np.int64)).astype(np.uint64)
    rows["n"] = r2["width"][rec]
    rows["kind"] = r2["kind"][rec]
    f, fb, u, a = intervals.expected(w, rows)
    out = np.zeros(T, W.VERDICT_DTYPE)
    flags = np.zeros(T, np.uint32)
    np.bitwise_or.at(flags, rec, f.astype(np.uint32))
    none = np.uint64((1 << 64) - 1)
    cand = np.where(fb != none, (r.astype(np.uint64) * r2["width"][rec]) + fb, none)
    firsts = np.full(T, none, np.uint64)
    np.minimum.at(firsts, rec, cand.astype(np.uint64))
    und = np.zeros(T, np.uint64)
    np.add.at(und, rec, u.astype(np.uint64))
    av = np.zeros(T, np.uint64)
    av[rec[r == 0]] = a[r == 0]
    out["flags"], out["first_bad"], out["undef_bytes"], out["avail"] = flags, firsts, und, av
    return out, rows.size


def test_config2_as_pitched_rows(X, H):
    """Configuration 2's copies as pitched 2D records on the no-wait path, at
    full size: 4 KiB rows back to back (worked as one transfer each), 4,032-byte
    rows at a 4 KiB pitch (row by row), and, for the first 300 copies,
    240-byte rows at a 256-byte pitch (several rows per wave iteration).
    Every record's verdict equals the rows' verdicts by interval arithmetic,
    combined by the row-by-row numbering of its bytes."""
    t0 = time.time()
    w = W.config2()
    hv, ha = W.host_v(w.host), W.host_a(w.host)
    dw = H.DeviceWorld(w, host_arrays=(hv, ha))
    say(f"config 2 set up in {time.time() - t0:.1f} s")
    try:
        base = np.zeros(w.count, W.RECORD2D_DTYPE)
        base["src"], base["dst"], base["kind"] = w.records["src"], w.records["dst"], w.records["kind"]
        for name, width, pitch, k in (("back to back", 4096, 4096, w.count), ("strided", 4032, 4096, w.count),
                                      ("short rows", 240, 256, 300)):
            r2 = base[:k].copy()
            r2["width"], r2["spitch"], r2["dpitch"] = width, pitch, pitch
            r2["rows"] = w.records["n"][:k] // pitch
            want, nrows = rows_and_expected(w, r2)
            rt = torch.from_numpy(np.ascontiguousarray(r2).view(np.uint8).copy()).to(dw.dev)
            out = H.verdicts_tensor(k, dw.dev)
            X.check_transfers_2d(dw.ctx, rt.data_ptr(), k, out.data_ptr(), X.CG_CHECK,
                                 torch.cuda.current_stream(dw.dev).cuda_stream)
            torch.cuda.synchronize(dw.dev)
            util.assert_verdicts_equal(H.verdicts_np(out, k), want, f"config 2 as {name}")
            say(f"config 2 as {name}: {k} records, {nrows} rows equal ({time.time() - t0:.1f} s)")
    finally:
        dw.close()
