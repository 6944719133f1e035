"""The C ABI on the GPU: status codes of the error paths, the paper's worked
example end to end, graph replays, and concurrent streams."""
import json
import os

import numpy as np
import pytest

from paper_1310_0901_amd import workloads as W
from tests import util

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


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


def status(X, fn, *a):
    try:
        fn(*a)
    except X.CgError as e:
        return e.status
    return X.CG_OK


def test_status_codes(X):
    ctx = X.cg_create(0, 1 << 16, 4)
    try:
        B = W.DEV_BASE
        assert status(X, X.shadow_alloc, ctx, B, 0) == X.CG_EINVAL
        assert status(X, X.shadow_alloc, ctx, B, 1000) == X.CG_OK
        assert status(X, X.shadow_alloc, ctx, B + 999, 10) == X.CG_EOVERLAP
        assert status(X, X.shadow_alloc, ctx, B - 5, 6) == X.CG_EOVERLAP
        assert status(X, X.shadow_alloc, ctx, B + 1000, 10) == X.CG_OK          # adjacent
        assert status(X, X.shadow_free, ctx, B + 1) == X.CG_ENOTFOUND          # not a base
        assert status(X, X.shadow_set, ctx, B + 990, 20, 0) == X.CG_EINVAL     # leaves the allocation
        assert status(X, X.shadow_set, ctx, B + 5000, 1, 0) == X.CG_ENOTFOUND
        assert status(X, X.shadow_ptr, ctx, B + 5000) == X.CG_ENOTFOUND
        assert status(X, X.shadow_alloc, ctx, B + 8192, 1 << 20) == X.CG_ENOMEM  # pool is 64 KiB
        assert status(X, X.shadow_alloc, ctx, B + 8192, 100) == X.CG_OK
        assert status(X, X.shadow_alloc, ctx, B + 9000, 100) == X.CG_OK
        assert status(X, X.shadow_alloc, ctx, B + 10000, 100) == X.CG_ECAPACITY  # 4 live max
        assert status(X, X.shadow_free, ctx, B) == X.CG_OK
        assert status(X, X.shadow_free, ctx, B) == X.CG_ENOTFOUND              # double free
        assert status(X, X.check_transfers, ctx, 0, 1, 0, X.CG_CHECK, 0) == X.CG_EINVAL
        assert status(X, X.check_transfers, ctx, 16, 1, 16, 0, 0) == X.CG_EINVAL   # no mode
        assert status(X, X.check_transfers, ctx, 16, 1, 16, 0x100 | X.CG_CHECK, 0) == X.CG_EINVAL
        assert status(X, X.check_transfers, ctx, 0, 0, 0, X.CG_CHECK, 0) == X.CG_OK   # empty batch
        v = torch.zeros(64, dtype=torch.uint8, device="cuda")
        assert status(X, X.cg_host_register, ctx, 0x1000, 16, v.data_ptr() + 1, v.data_ptr()) == X.CG_EINVAL
        assert status(X, X.cg_host_register, ctx, 0x1000, 0, v.data_ptr(), v.data_ptr()) == X.CG_EINVAL
        assert X.cg_stats(ctx)[0] == 3
        assert "live allocation" in X.cg_last_error(ctx) or X.cg_last_error(ctx)
    finally:
        X.cg_destroy(ctx)


def test_pin1_worked_example_on_gpu(X, H):
    """Sec. 4: c holds 1,000,000 floats, the copy back wants 1,000,000
    doubles; a is allocated right after c."""
    fx = json.load(open(os.path.join(ROOT, "tests", "golden", "pin1_worked_example.json")))
    n = fx["copy_bytes"]
    c = W.DEV_BASE
    a = c + fx["c_alloc_bytes"]
    b = a + fx["a_alloc_bytes"] + 256
    ctx = X.cg_create(0, 32 << 20, 16)
    try:
        hv = torch.full((n + 32,), 0xFF, dtype=torch.uint8, device="cuda")
        ha = torch.full(((n + 63) // 64,), -1, dtype=torch.int64, device="cuda")
        X.cg_host_register(ctx, W.HOST_BASE, n, hv.data_ptr(), ha.data_ptr())
        X.shadow_alloc(ctx, c, fx["c_alloc_bytes"])
        X.shadow_alloc(ctx, a, fx["a_alloc_bytes"])
        X.shadow_alloc(ctx, b, fx["b_alloc_bytes"])
        X.shadow_set(ctx, c, fx["c_alloc_bytes"], 0)      # the kernel wrote c
        recs = np.array([(c, W.HOST_BASE, n, X.CG_D2H, 0)], W.RECORD_DTYPE)
        rt = H.records_tensor(recs)
        out = H.verdicts_tensor(1)
        for mode in (X.CG_CHECK, X.CG_CHECK | X.CG_PLAIN, X.CG_CHECK | X.CG_PROPAGATE):
            X.check_transfers(ctx, rt.data_ptr(), 1, out.data_ptr(), mode, torch.cuda.current_stream().cuda_stream)
            v = H.verdicts_np(out, 1)[0]
            assert (int(v["flags"]), int(v["first_bad"]), int(v["undef_bytes"]), int(v["avail"])) == \
                (X.CG_SRC_OVERRUN, fx["found_bytes"], 0, fx["found_bytes"])
        txt = X.cg_format_verdict((c, W.HOST_BASE, n, X.CG_D2H),
                                  (int(v["flags"]), int(v["first_bad"]), int(v["undef_bytes"]), int(v["avail"])))
        assert txt.split("\n") == fx["report_lines"]
        # propagation wrote c's defined bytes into the host shadow and 0xFF beyond
        h = hv[:n].cpu().numpy()
        assert not h[: fx["c_alloc_bytes"]].any() and (h[fx["c_alloc_bytes"]:] == 0xFF).all()
    finally:
        X.cg_destroy(ctx)


def test_graph_replays_match_eager(X, H):
    """A captured check replayed several times, with other eager work and
    synchronisations between the replays: every replay equals the eager run."""
    w = W.small_config(3)
    dw = H.DeviceWorld(w)
    try:
        s = torch.cuda.current_stream().cuda_stream
        rt = H.records_tensor(w.records)
        eager = dw.check(w.records, X.CG_CHECK | X.CG_EAGER)
        other = w.records[::7].copy()
        out = H.verdicts_tensor(w.count)
        for rep in range(4):
            out.fill_(0xAB)
            X.check_transfers(dw.ctx, rt.data_ptr(), w.count, out.data_ptr(), X.CG_CHECK, s)
            torch.cuda.synchronize()
            util.assert_verdicts_equal(H.verdicts_np(out, w.count), eager, f"replay {rep}")
            dw.check(other, X.CG_CHECK | X.CG_EAGER)
            torch.cuda.synchronize()
    finally:
        dw.close()


def test_two_streams_concurrently(X, H):
    """Checks issued on two streams at once use separate workspaces and give
    the same verdicts as alone."""
    w = W.small_config(3)
    dw = H.DeviceWorld(w)
    try:
        half = w.count // 2
        r1, r2 = w.records[:half], w.records[half:]
        alone1, alone2 = dw.check(r1), dw.check(r2)
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        t1, t2 = H.records_tensor(r1), H.records_tensor(r2)
        o1, o2 = H.verdicts_tensor(len(r1)), H.verdicts_tensor(len(r2))
        torch.cuda.synchronize()
        for _ in range(3):
            X.check_transfers(dw.ctx, t1.data_ptr(), len(r1), o1.data_ptr(), X.CG_CHECK, s1.cuda_stream)
            X.check_transfers(dw.ctx, t2.data_ptr(), len(r2), o2.data_ptr(), X.CG_CHECK, s2.cuda_stream)
        torch.cuda.synchronize()
        util.assert_verdicts_equal(H.verdicts_np(o1, len(r1)), alone1, "stream 1")
        util.assert_verdicts_equal(H.verdicts_np(o2, len(r2)), alone2, "stream 2")
    finally:
        dw.close()


def test_shadow_ops_are_ordered_after_checks(X, H):
    """A free + re-allocation + set issued right after a check (no host sync)
    does not change what that check saw."""
    w = W.small_config(1)
    dw = H.DeviceWorld(w)
    try:
        want = dw.check(w.records)
        s = torch.cuda.current_stream().cuda_stream
        rt = H.records_tensor(w.records)
        out = H.verdicts_tensor(w.count)
        X.check_transfers(dw.ctx, rt.data_ptr(), w.count, out.data_ptr(), X.CG_CHECK, s)
        live = w.dev.live_idx
        X.shadow_free(dw.ctx, int(w.dev.base[live[0]]))
        X.shadow_alloc(dw.ctx, int(w.dev.base[live[0]]), int(w.dev.size[live[0]]))
        X.shadow_set(dw.ctx, int(w.dev.base[live[0]]), int(w.dev.size[live[0]]), 0)
        torch.cuda.synchronize()
        util.assert_verdicts_equal(H.verdicts_np(out, w.count), want, "check before the table change")
    finally:
        dw.close()


def test_table_churn_versions_match_oracle(X, H):
    """Frees and allocations between batches with no host synchronisation:
    each batch sees exactly the table of its issue time (device merges and
    full uploads of the version ring), freed shadow blocks are not reused
    while earlier checks may read them."""
    rng = np.random.default_rng(5)
    hl = 1 << 20
    hv = np.where(rng.random(hl) < 0.001, 0xFF, 0).astype(np.uint8)
    n0 = 3000
    sizes = rng.integers(16, 4096, size=n0)
    bases = (W.DEV_BASE + np.cumsum(np.concatenate([[0], sizes[:-1]])) + np.arange(n0) * 256).astype(np.uint64)
    vs = {int(b): np.where(rng.random(int(s)) < 0.002, 0x40, 0).astype(np.uint8) for b, s in zip(bases, sizes)}
    pool = int(((sizes + 255) // 256 * 256).sum()) + (2 << 20)
    ctx = X.cg_create(0, pool, n0 + 4000)
    try:
        hvt = torch.zeros(hl + 32, dtype=torch.uint8, device="cuda")
        hvt[:hl].copy_(torch.from_numpy(hv))
        ha = np.full(hl // 64, np.uint64(0xFFFF_FFFF_FFFF_FFFF), np.uint64)
        hat = torch.from_numpy(ha.view(np.int64)).cuda()
        X.cg_host_register(ctx, W.HOST_BASE, hl, hvt.data_ptr(), hat.data_ptr())
        X.shadow_alloc_batch(ctx, bases, sizes)
        X.shadow_set_batch(ctx, bases, sizes, np.zeros(n0, np.uint8))
        for b, v in vs.items():
            for x in np.flatnonzero(v):
                X.shadow_set(ctx, b + int(x), 1, int(v[x]))
        live = dict(vs)
        next_base = int(bases[-1] + sizes[-1]) + 4096
        s = torch.cuda.current_stream().cuda_stream
        pending = []
        freed = []
        for step in range(40):
            nev = 1200 if step == 20 else int(rng.integers(0, 25))
            for _ in range(nev):
                if rng.random() < 0.5 and len(live) > 100:
                    b = list(live)[int(rng.integers(0, len(live)))]
                    X.shadow_free(ctx, b)
                    freed.append(b)
                    del live[b]
                else:
                    sz = int(rng.integers(16, 4096))
                    X.shadow_alloc(ctx, next_base, sz)
                    live[next_base] = np.full(sz, 0xFF, np.uint8)
                    next_base += sz + 512
            keys = list(live)
            rows = []
            for _ in range(64):
                kind = int(rng.integers(0, 3))
                if rng.random() < 0.1 and freed:
                    b = freed[int(rng.integers(0, len(freed)))]
                    L = 64
                else:
                    b = keys[int(rng.integers(0, len(keys)))]
                    L = live[b].size
                n = int(rng.integers(1, L + 1))
                o = int(rng.integers(0, L - n + 1))
                hp = W.HOST_BASE + int(rng.integers(0, hl - n))
                dp = b + o
                other = keys[int(rng.integers(0, len(keys)))]
                src = hp if kind == 0 else dp
                dst = hp if kind == 1 else (dp if kind == 0 else other)
                rows.append((src, dst, n, kind, 0))
            recs = np.array(rows, W.RECORD_DTYPE)
            rt, out = H.records_tensor(recs), H.verdicts_tensor(len(recs))
            mode = X.CG_CHECK | (X.CG_PLAIN if step % 7 == 3 else 0)
            X.check_transfers(ctx, rt.data_ptr(), len(recs), out.data_ptr(), mode, s)
            snap = {b: v.copy() for b, v in live.items()}
            pending.append((recs, rt, out, snap))
        torch.cuda.synchronize()
        for i, (recs, rt, out, snap) in enumerate(pending):
            bs = np.array(sorted(snap), np.uint64)
            o = util.OracleState(W.HOST_BASE, hl, hv.copy(), ha, bs, np.array([snap[int(b)].size for b in bs], np.uint64),
                                 [snap[int(b)] for b in bs])
            util.assert_verdicts_equal(H.verdicts_np(out, len(recs)), o.run(recs), f"batch {i}")
    finally:
        X.cg_destroy(ctx)


def test_first_version_merged_into_empty_table(X):
    """A few allocations after the empty start: the next table version is a
    device merge of an empty old version with the inserts (no kept entries).
    Verdicts match the oracle, and pointer lookups see the new entries."""
    from oracle import oracle
    B = W.DEV_BASE
    ctx = X.cg_create(0, 1 << 20, 64)
    try:
        X.shadow_alloc(ctx, B, 1000)
        X.shadow_alloc(ctx, B + 4096, 100)
        recs = np.array([(B, B + 4096, 100, 2, 0), (B, B + 4096, 101, 2, 0), (B + 999, B + 4096, 2, 2, 0)],
                        W.RECORD_DTYPE)
        rt = torch.from_numpy(recs.view(np.uint8).copy()).to("cuda:0")
        out = torch.zeros(recs.size * 32, dtype=torch.uint8, device="cuda:0")
        s = torch.cuda.current_stream()
        X.check_transfers(ctx, rt.data_ptr(), recs.size, out.data_ptr(), X.CG_CHECK | X.CG_EAGER, s.cuda_stream)
        s.synchronize()
        got = out.cpu().numpy().view(W.VERDICT_DTYPE)
        st = oracle.OracleState(0x1000, 64, np.zeros(64, np.uint8), np.full(1, ~np.uint64(0), np.uint64),
                                np.array([B, B + 4096], np.uint64), np.array([1000, 100], np.uint64),
                                [np.full(1000, 0xFF, np.uint8), np.full(100, 0xFF, np.uint8)])
        want = st.run(recs)
        for f in ("flags", "first_bad", "undef_bytes", "avail"):
            assert np.array_equal(got[f], want[f]), f
        ptrs = np.array([B, B + 1000, B + 4096 + 50, B + 2000], np.uint64)
        pt = torch.from_numpy(ptrs.view(np.uint8).copy()).to("cuda:0")
        po = torch.zeros(ptrs.size * 24, dtype=torch.uint8, device="cuda:0")
        X.check_pointers(ctx, pt.data_ptr(), ptrs.size, po.data_ptr(), s.cuda_stream)
        s.synchronize()
        pr = po.cpu().numpy().view(W.PTR_DTYPE)
        assert pr["flags"].tolist() == [0, 0, 0, X.CG_PTR_UNALLOC]
        assert pr["base"].tolist() == [B, B, B + 4096, 0] and pr["avail"].tolist() == [1000, 0, 50, 0]
    finally:
        X.cg_destroy(ctx)
