"""Benchmark of the transfer checker on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 3]

Workload (default): the batched configuration -- 1,000,000 transfer records
(sizes log-uniform in 8 B .. 16 MiB, kinds 60/30/10 host->device /
device->device / device->host, device sides drawn Zipf(1.1) over 65,536 live
allocations, 2 % overruns, 1 % use-after-free) against a 4 GiB host region
(V bytes + A bitmap) and ~75 GB of device shadow, all synthetic and seeded.

A step is one check_transfers call over all records: classify + scan + the
persistent scan kernel, replayed as a hipGraph.  Inputs are resident in HBM
before the timed region.  `value` is algorithmic shadow GB/s (1.125 bytes per
host<->device transfer byte: V byte + A bit; 1.0 per device->device byte).
After the timed region the plain path (one kernel launch per record, same
inner loop) runs once on the same records for the batched-vs-plain ratio, and
the CPU oracle is timed on a bounded sample.  One JSON line on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# the sources of the profiled kernels: a profile holds while their sha256 (in this order) is unchanged
KERNEL_SOURCES = ("kernels.hip", "shadowindex.hip")
METRIC = "shadow GB/s checked (% HBM peak) batched vs plain; transfers/s; p50/p99 check latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algo_bytes(recs, propagate=False):
    import numpy as np
    n = recs["n"].astype(np.float64)
    k = recs["kind"]
    f = np.where(k == 2, 1.0, np.where(k <= 1, 1.125, 0.0))
    if propagate:
        f = f + np.where(k <= 2, 1.0, 0.0)
    return float((n * f).sum())


def cpu_baseline(w, hv, ha, got, target_bytes, threads):
    """Oracle on the first records of the workload up to ~target_bytes of
    transfer data, on `threads` host threads; returns (GB/s, sample text, ok, s)."""
    import numpy as np
    from oracle.oracle import OracleState
    from paper_1310_0901_amd import workloads as W
    n = w.records["n"].astype(np.int64)
    m = int(np.searchsorted(np.cumsum(n), target_bytes)) + 1
    m = min(m, w.count)
    sample = w.records[:m]
    # live allocations any device pointer of the sample lies in (a verdict
    # depends only on the allocation holding the pointer)
    live = w.dev.live_idx
    lb = w.dev.base[live].astype(np.int64)
    ls = w.dev.size[live].astype(np.int64)
    ptrs = np.concatenate([sample["src"][sample["kind"] != 0], sample["dst"][sample["kind"] != 1]]).astype(np.int64)
    j = np.searchsorted(lb, ptrs, side="right") - 1
    ok = (j >= 0) & (ptrs < lb[np.maximum(j, 0)] + ls[np.maximum(j, 0)])
    idx = np.unique(live[j[ok]])
    st = OracleState(w.host.base, w.host.length, hv, ha, w.dev.base[idx], w.dev.size[idx],
                     [W.alloc_v(w.dev, int(x)) for x in idx])
    t0 = time.perf_counter()
    v = st.run_threads(sample, threads)
    dt = time.perf_counter() - t0
    same = all(np.array_equal(v[f], got[f][:m]) for f in ("flags", "first_bad", "undef_bytes", "avail"))
    gbs = algo_bytes(sample) / dt / 1e9
    text = (f"first {m} of {w.count} records ({int(n[:m].sum()) / 1e9:.2f} GB of transfers, "
            f"{idx.size} allocations materialised), check-only, {threads} thread(s), {dt:.2f} s wall; "
            f"the rate is per algorithmic byte, so it scales to the whole batch")
    return gbs, text, same, dt


def cpu_cores():
    """Host cores this process may run on, and how many the oracle uses: all
    of them, up to the 16-core share a one-GPU machine gives a process."""
    aff = sorted(os.sched_getaffinity(0))
    return aff, min(len(aff), 16)


def cpu_baseline_legs(w, hv, ha, got, all_bytes, one_bytes):
    """The oracle on one thread and on every allowed core (cpu_cores)."""
    aff, n_all = cpu_cores()
    legs = {}
    for name, threads, b in (("one_thread", 1, one_bytes), ("all_cores", n_all, all_bytes)):
        gbs, text, same, dt = cpu_baseline(w, hv, ha, got, b, threads)
        legs[name] = {"value": round(gbs, 3), "cores": threads, "sample": text, "seconds": round(dt, 2),
                      "verdicts_identical_to_gpu": bool(same)}
        log(f"[bench] oracle {name}: {gbs:.2f} GB/s on {threads} thread(s), identical: {same}")
    top = legs["all_cores"]
    return {"value": top["value"], "unit": "GB/s", "cores": top["cores"], "kind": "oracle", "sample": top["sample"],
            "verdicts_identical_to_gpu": top["verdicts_identical_to_gpu"] and legs["one_thread"]["verdicts_identical_to_gpu"],
            "one_thread": legs["one_thread"], "all_cores": legs["all_cores"],
            "host": {"affinity_cores": len(aff), "affinity": f"{aff[0]}-{aff[-1]}" if aff else "",
                     "os_cpu_count": os.cpu_count(),
                     "note": "all_cores uses every core of the affinity set up to 16, the CPU share of a one-GPU box"}}


def matching_profile(name, tuning, config):
    """A committed rocprofv3 summary (profiles/<name>.json) of a kernel on the
    1M-record workload, if the kernel source and launch shape are the ones
    profiled: (dict, None); else (None, the reason)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name + ".json")
    if config != 3 or not os.path.exists(path):
        return None, "no profile for this workload"
    prof = json.load(open(path))
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1310_0901_amd", "csrc", name), "rb").read())
    if h.hexdigest() != prof.get("kernel_sources_sha256"):
        return None, "kernel changed since the counters were taken"
    if tuning is not None and {k: tuning[k] for k in prof["tuning"]} != prof["tuning"]:
        return None, "launch shape differs from the profiled one"
    return prof, None


def roofline(tun, config, k_avg_ms, i_avg_ms, pass_bytes, bytes_step, l2_probe_GBps):
    """The dominant kernel's roofline.  When the shadow indexes answer the
    check-only records, that is the indexes' counting pass (k_sidx_count, one
    launch over both spaces): it reads once each V byte (and the host
    region's A bits) of the 64 KiB steps the batch's records read (its
    algorithmic bytes: `pass_bytes`, as the library counted them for the
    timed passes), so HBM bounds it; achieved = those bytes over its live
    duration, traffic from its committed counters.  Otherwise it is the scan
    kernel: the bytes the L2 returns to the L1s per launch (L1 -> L2 read
    requests x 128 B, from its counters) over the launch, against the
    L2-resident read probe measured in this run, HBM traffic beside it."""
    if i_avg_ms and i_avg_ms >= k_avg_ms:
        t = i_avg_ms / 1e3
        achieved = pass_bytes / t / 1e9
        out = {"kernel": "k_sidx_count", "kernel_avg_ms": round(i_avg_ms, 3), "bound": "hbm",
               "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
               "algorithmic_bytes_per_launch": int(pass_bytes), "scan_kernel_avg_ms": round(k_avg_ms, 3),
               "note": "the shadow indexes' counting pass reads once each V byte of the 64 KiB steps of the host "
                       "region and of the pool that the batch's records read, and the host region's A bits of "
                       "them (16-byte V loads, 2-byte A loads); achieved = those bytes (counted by the library, "
                       "cg_index_ms) over the pass's live duration (HIP events around it on the check's stream); "
                       "traffic = HBM-side bytes per launch from FETCH_SIZE + WRITE_SIZE, "
                       "profiles/k_sidx_count_batched-1M_counters.md"}
        prof, why = matching_profile("k_sidx_count_batched-1M_counters", None, config)
        if prof is not None:
            tb = int(prof["limits"]["traffic_bytes"])
            out.update(traffic=tb, hbm_traffic_GBps=round(tb / t / 1e9, 1),
                       traffic_over_algorithmic=round(tb / pass_bytes, 4))
        else:
            out["traffic_note"] = why
        return out
    prof, why = matching_profile("k_batched_lds_batched-1M_counters", tun, config)
    t = k_avg_ms / 1e3
    out = {"kernel": "k_batched_lds", "kernel_avg_ms": round(k_avg_ms, 3),
           "effective_algorithmic_GBps": round(bytes_step / t / 1e9, 1),
           "algorithmic_bytes_per_launch": int(bytes_step)}
    if prof is None:
        return dict(out, bound=None, achieved=None, peak=None, unit="GB/s", frac=None, traffic=None, note=why)
    lim = prof["limits"]
    peak = l2_probe_GBps or None
    achieved = lim["l2_to_l1_bytes"] / t / 1e9
    traffic = int(lim["traffic_bytes"])
    return dict(bound=prof["bound"], achieved=round(achieved, 1), peak=round(peak, 1) if peak else None, unit="GB/s",
                frac=round(achieved / peak, 4) if peak else None, traffic=traffic,
                hbm_GBps=round(traffic / t / 1e9, 1), hbm_frac=round(traffic / t / 1e9 / HBM_PEAK_GBS, 4),
                **out,
                note="achieved = bytes the L2 returns to the L1s per launch (counted L1 -> L2 read requests x 128 B, "
                     "profiles/k_batched_lds_batched-1M_counters.md) over this run's kernel time; peak = this run's "
                     "L2-resident read probe (cg_probe_l2). Host-source segments are checked from LDS, so the "
                     "algorithmic bytes exceed what crosses L2; traffic = HBM-side bytes per launch from FETCH_SIZE + "
                     "WRITE_SIZE; effective_algorithmic_GBps counts every byte the check examines",
                limits=dict({k: v for k, v in lim.items() if k not in ("traffic_bytes", "l2_to_l1_bytes")},
                            source="profiles/k_batched_lds_batched-1M_counters.md"))


def given_order_leg(X, ctx, w, recs_t, got, T, stream, dev, bytes_step, steps=2):
    """The same batch worked in the given order (CG_KEEP_ORDER: no source-block
    segments, so almost no byte is re-read from cache): every examined byte
    comes from HBM, and the algorithmic rate is an HBM rate."""
    import numpy as np
    import torch
    from paper_1310_0901_amd.harness import verdicts_tensor, verdicts_np
    mode = X.CG_CHECK | X.CG_KEEP_ORDER
    out = verdicts_tensor(T, dev)
    tun = X.cg_autotune(ctx, recs_t.data_ptr(), T, out.data_ptr(), mode, stream, TUNE_CACHE).as_dict()
    X.check_transfers(ctx, recs_t.data_ptr(), T, out.data_ptr(), mode, stream)   # warm-up
    torch.cuda.synchronize(dev)
    X.cg_kernel_ms(ctx)
    t0 = time.perf_counter()
    for _ in range(steps):
        X.check_transfers(ctx, recs_t.data_ptr(), T, out.data_ptr(), mode, stream)
    torch.cuda.synchronize(dev)
    wall = (time.perf_counter() - t0) / steps
    kms, nk = X.cg_kernel_ms(ctx)
    k = kms / max(nk, 1)
    v = verdicts_np(out, T)
    same = all(np.array_equal(v[f], got[f]) for f in ("flags", "first_bad", "undef_bytes", "avail"))
    o = {"ms_per_step": round(wall * 1e3, 3), "scan_ms": round(k, 3),
         "GBps": round(bytes_step / wall / 1e9, 1), "scan_GBps": round(bytes_step / (k / 1e3) / 1e9, 1),
         "scan_pct_hbm_peak": round(100 * bytes_step / (k / 1e3) / 1e9 / HBM_PEAK_GBS, 2),
         "verdicts_identical_to_batched": bool(same), "tuning": tun,
         "note": "check-only, records in their given order: almost no re-read hits in L2, so this rate is bound "
                 "by HBM"}
    prof, why = matching_profile("k_batched_given-order_batched-1M_counters", tun, 3)
    if prof is not None:
        tb = prof["limits"]["traffic_bytes"]
        o["roofline"] = {"bound": "hbm", "achieved": round(tb / (k / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(tb / (k / 1e3) / 1e9 / HBM_PEAK_GBS, 4), "traffic": tb,
                         "traffic_over_algorithmic": round(tb / bytes_step, 4),
                         "source": "profiles/k_batched_given-order_batched-1M_counters.md"}
    else:
        o["roofline"] = {"note": why}
    log(f"[bench] given order: {o}")
    return o


def probe_l2(X, dev, stream, cus=256):
    """L2-resident read ceiling (cg_probe_l2): 8 slices, one per XCD, each
    re-read by 8 blocks per CU with the scan kernel's cached 16-byte loads;
    the best of three slice sizes that fit the 4 MB L2 of an XCD."""
    import torch
    best, rates = 0.0, {}
    sink = torch.zeros(1, dtype=torch.int64, device=dev)
    for mib in (1, 2, 3):
        sl = mib << 20
        buf = torch.zeros(8 * sl, dtype=torch.uint8, device=dev)
        blocks, passes = 8 * cus, 16
        X.cg_probe_l2(buf.data_ptr(), sl, passes, blocks, sink.data_ptr(), stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            X.cg_probe_l2(buf.data_ptr(), sl, passes, blocks, sink.data_ptr(), stream)
        e1.record()
        torch.cuda.synchronize(dev)
        r = blocks * sl * passes * 3 / (e0.elapsed_time(e1) / 1e3) / 1e9
        rates[f"{mib}MiB"] = round(r, 1)
        best = max(best, r)
        del buf
    return {"GBps": round(best, 1), "by_slice": rates}


TUNE_CACHE = os.environ.get("XC_TUNE_CACHE", os.path.join(ROOT, "paper_1310_0901_amd", "tuning_cache.jsonl"))


def scan_ms(X, ctx):
    ms, n = X.cg_kernel_ms(ctx)
    return ms / max(n, 1)


def plain_tiny_leg():
    """Configuration 1: 64 host->device records on a 1 MiB region; launch-bound,
    so the figure is latency per call (median of 50 synchronous calls)."""
    import numpy as np
    import torch
    from paper_1310_0901_amd import workloads as W, xfercheck as X
    from paper_1310_0901_amd.harness import DeviceWorld, records_tensor, verdicts_tensor, verdicts_np
    w = W.config1()
    dw = DeviceWorld(w)
    out = {"workload": f"{w.name} (configuration 1): {w.note}",
           "path": f"batches of up to 256 records run in one launch (k_small); larger ones as classify, scans and "
                   f"the persistent kernel"}
    try:
        ctx, T, s = dw.ctx, w.count, torch.cuda.current_stream().cuda_stream
        rt, ob = records_tensor(w.records), verdicts_tensor(T)
        res = {}
        for name, mode in (("batched_graph", X.CG_CHECK), ("batched_eager", X.CG_CHECK | X.CG_EAGER),
                           ("plain", X.CG_CHECK | X.CG_PLAIN)):
            ts = []
            for i in range(55):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                X.check_transfers(ctx, rt.data_ptr(), T, ob.data_ptr(), mode, s)
                torch.cuda.synchronize()
                if i >= 5:
                    ts.append(time.perf_counter() - t0)
            res[name] = verdicts_np(ob, T)
            out[name] = {"median_us_per_call": round(float(np.median(ts)) * 1e6, 1)}
            # device time of the check's kernels (events around them on the stream)
            X.cg_timing(ctx, True)
            X.cg_kernel_ms(ctx)
            for _ in range(20):
                X.check_transfers(ctx, rt.data_ptr(), T, ob.data_ptr(), mode, s)
            ms, k = X.cg_kernel_ms(ctx)
            X.cg_timing(ctx, False)
            out[name]["kernel_us_per_call"] = round(ms * 1e3 / 20, 1)
        out["verdicts_identical"] = bool(all(np.array_equal(res["plain"][f], res["batched_graph"][f])
                                             for f in ("flags", "first_bad", "undef_bytes", "avail")))
    finally:
        dw.close()
    log(f"[bench] plain tiny: {out}")
    return out


def plain_at_scale_leg():
    """Configuration 2: 4,096 full-size host->device records, plain (one launch
    per record) against batched, check-only and fused check + propagate."""
    import numpy as np
    import torch
    from paper_1310_0901_amd import workloads as W, xfercheck as X
    from paper_1310_0901_amd.harness import DeviceWorld, records_tensor, verdicts_tensor, verdicts_np
    w = W.config2()
    dw = DeviceWorld(w)
    try:
        ctx, T, s = dw.ctx, w.count, torch.cuda.current_stream().cuda_stream
        rt, ob, op = records_tensor(w.records), verdicts_tensor(T), verdicts_tensor(T)
        b = algo_bytes(w.records)
        tun = {m: X.cg_autotune(ctx, rt.data_ptr(), T, ob.data_ptr(), m, s, TUNE_CACHE).as_dict()
               for m in (X.CG_CHECK, X.CG_CHECK | X.CG_PROPAGATE)}
        X.cg_timing(ctx, True)
        out = {"workload": f"{w.name} (configuration 2): {w.note}, 4 GiB host region, "
                           f"{int(w.records['n'].sum()) / 1e9:.1f} GB of transfers", "algorithmic_bytes": int(b)}
        for name, mode, buf in (("batched", X.CG_CHECK, ob), ("plain", X.CG_CHECK | X.CG_PLAIN, op)):
            X.check_transfers(ctx, rt.data_ptr(), T, buf.data_ptr(), mode, s)   # warm-up
            torch.cuda.synchronize()
            X.cg_kernel_ms(ctx)
            t0 = time.perf_counter()
            reps = 3
            for _ in range(reps):
                X.check_transfers(ctx, rt.data_ptr(), T, buf.data_ptr(), mode, s)
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / reps
            k = scan_ms(X, ctx)
            out[name] = {"ms": round(wall * 1e3, 3), "GBps": round(b / wall / 1e9, 1),
                         "scan_ms": round(k, 3), "scan_GBps": round(b / (k / 1e3) / 1e9, 1),
                         "launches_per_step": 1 if name == "batched" else int((w.records["n"] > 0).sum())}
        same = all(np.array_equal(verdicts_np(ob, T)[f], verdicts_np(op, T)[f])
                   for f in ("flags", "first_bad", "undef_bytes", "avail"))
        out["verdicts_identical"] = bool(same)
        # fused check + propagate (every record writes its own allocation)
        X.cg_kernel_ms(ctx)
        X.check_transfers(ctx, rt.data_ptr(), T, ob.data_ptr(), X.CG_CHECK | X.CG_PROPAGATE, s)
        torch.cuda.synchronize()
        k = scan_ms(X, ctx)
        bp = algo_bytes(w.records, propagate=True)
        out["batched_check_propagate"] = {"scan_ms": round(k, 3), "GBps": round(bp / (k / 1e3) / 1e9, 1),
                                          "algorithmic_bytes": int(bp)}
        out["tuning"] = {"check": tun[X.CG_CHECK], "check_propagate": tun[X.CG_CHECK | X.CG_PROPAGATE]}
        # the same copies as pitched 2D copies of 4 KiB rows (contiguous pitches), one check_transfers_2d call
        r2 = np.zeros(T, W.RECORD2D_DTYPE)
        rows = w.records["n"] // 4096
        r2["src"], r2["dst"], r2["kind"] = w.records["src"], w.records["dst"], w.records["kind"]
        r2["width"], r2["rows"], r2["spitch"], r2["dpitch"] = 4096, rows, 4096, 4096
        b2 = int((rows * 4096).sum()) * 9 // 8
        rt2 = torch.from_numpy(r2.view(np.uint8).copy()).to(rt.device)
        X.cg_timing(ctx, False)
        X.check_transfers_2d(ctx, rt2.data_ptr(), T, ob.data_ptr(), X.CG_CHECK, s)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            X.check_transfers_2d(ctx, rt2.data_ptr(), T, ob.data_ptr(), X.CG_CHECK, s)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / 3
        out["pitched_2d"] = {"records": T, "rows": int(rows.sum()), "ms": round(wall * 1e3, 3),
                             "GBps": round(b2 / wall / 1e9, 1), "algorithmic_bytes": b2}
        # strided: the same rows narrowed to 4,032 bytes at the 4 KiB pitch (a sub-matrix copy)
        r2["width"] = 4032
        b3 = int((rows * 4032).sum()) * 9 // 8
        rt3 = torch.from_numpy(r2.view(np.uint8).copy()).to(rt.device)
        X.check_transfers_2d(ctx, rt3.data_ptr(), T, ob.data_ptr(), X.CG_CHECK, s)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            X.check_transfers_2d(ctx, rt3.data_ptr(), T, ob.data_ptr(), X.CG_CHECK, s)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / 3
        out["pitched_2d_strided"] = {"records": T, "rows": int(rows.sum()), "width": 4032, "pitch": 4096,
                                     "ms": round(wall * 1e3, 3), "GBps": round(b3 / wall / 1e9, 1),
                                     "algorithmic_bytes": b3}
        # short strided rows: 240 bytes at a 256-byte pitch over the same spans
        rows_s = w.records["n"] // 256
        r2["width"], r2["rows"], r2["spitch"], r2["dpitch"] = 240, rows_s, 256, 256
        b4 = int((rows_s * 240).sum()) * 9 // 8
        rt4 = torch.from_numpy(r2.view(np.uint8).copy()).to(rt.device)
        X.check_transfers_2d(ctx, rt4.data_ptr(), T, ob.data_ptr(), X.CG_CHECK, s)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            X.check_transfers_2d(ctx, rt4.data_ptr(), T, ob.data_ptr(), X.CG_CHECK, s)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / 3
        out["pitched_2d_short"] = {"records": T, "rows": int(rows_s.sum()), "width": 240, "pitch": 256,
                                   "ms": round(wall * 1e3, 3), "GBps": round(b4 / wall / 1e9, 1),
                                   "algorithmic_bytes": b4}
    finally:
        dw.close()
    log(f"[bench] plain at scale: {out}")
    return out


def propagation_leg():
    """Configuration 4: 2 GiB of 16-byte records with padding, H2D then four
    D2D hops, fused check + propagate, one batch per hop; verified against the
    closed form and the final shadow against host V on the device."""
    import numpy as np
    import torch
    from paper_1310_0901_amd import workloads as W, xfercheck as X
    from paper_1310_0901_amd.harness import DeviceWorld, records_tensor, verdicts_tensor, verdicts_np, device_view
    res = {}
    for pieces in (1, 4096):
        w = W.config4(pieces=pieces)
        dw = DeviceWorld(w)
        try:
            ctx, s = dw.ctx, torch.cuda.current_stream().cuda_stream
            st0 = w.stages[0]
            rt0, out0 = records_tensor(st0), verdicts_tensor(st0.size)
            tun = X.cg_autotune(ctx, rt0.data_ptr(), st0.size, out0.data_ptr(), X.CG_CHECK | X.CG_PROPAGATE, s,
                                TUNE_CACHE).as_dict()
            X.cg_timing(ctx, True)
            stages, ok = [], True
            for h, st in enumerate(w.stages):
                rt, out = records_tensor(st), verdicts_tensor(st.size)
                X.cg_kernel_ms(ctx)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                e0.record()
                X.check_transfers(ctx, rt.data_ptr(), st.size, out.data_ptr(), X.CG_CHECK | X.CG_PROPAGATE, s)
                e1.record()
                torch.cuda.synchronize()
                k = scan_ms(X, ctx)
                whole = e0.elapsed_time(e1)
                v = verdicts_np(out, st.size)
                ok &= int(v["undef_bytes"].sum()) == 3 * w.R + w.P
                b = algo_bytes(st, propagate=True)
                stages.append({"hop": h, "scan_ms": round(k, 3), "GBps": round(b / (k / 1e3) / 1e9, 1),
                               "whole_check_ms": round(whole, 3)})
            last = w.dev.live_idx[-1]
            dv = device_view(X.shadow_ptr(ctx, int(w.dev.base[last])), w.host.length)
            ok &= bool(torch.equal(dv, dw.hv[: w.host.length]))
            res[f"pieces_{pieces}"] = {"stages": stages, "closed_form_and_final_shadow_ok": bool(ok), "tuning": tun}
        finally:
            dw.close()
    log(f"[bench] propagation: {res}")
    return {"workload": "partial-definedness (configuration 4): 2 GiB of 16-byte records, 3 padding bytes each, "
                        "1 % single payload bits; H2D then 4 D2D hops with propagation", **res}


def serving_leg(plain_seconds):
    """Configuration 5: continuous batching vs the plain path on one event log."""
    import numpy as np
    from paper_1310_0901_amd import workloads as W, serving as S
    t0 = time.perf_counter()
    sw = W.config5()
    hv, ha = W.host_v(sw.host), W.host_a(sw.host)
    log(f"[bench] serving log: {sw.requests.size} requests, {(sw.events['type'] != 0).sum()} alloc/free events "
        f"({time.perf_counter() - t0:.1f} s)")
    out = {"workload": f"{sw.name} (configuration 5): {sw.note}; 4 GiB host region",
           "admission_cap_bytes": 16 << 30}
    # micro-batches hold 1-2 requests on average at this load: padding them to
    # 64 records rather than 512 cuts the p50 by about a third
    cfg = S.config(streams=4, max_batch=64)
    # a warm-up run of the loop on the first second of the log (a context of
    # its own): the first run in a process pays one-time costs of the runtime
    # and the device, about 20 us of p50
    warm = int(np.searchsorted(sw.events["t"], 1.0))
    wsub = W.ServeWorkload(sw.name, sw.host, sw.dev, sw.events[:warm].copy(), sw.label, sw.rate)
    dw = S.serve_world(wsub, host_arrays=(hv, ha))
    try:
        _, wsumm = S.run(dw, wsub, cfg)
    finally:
        dw.close()
    log(f"[bench] serving warm-up (first 1 s of the log): p50 {wsumm['p50_ms']} ms, p99 {wsumm['p99_ms']} ms")
    dw = S.serve_world(sw, host_arrays=(hv, ha))
    try:
        res, summ = S.run(dw, sw, cfg)
    finally:
        dw.close()
    out["warmup"] = {"seconds_of_log": 1.0, "p50_ms": wsumm["p50_ms"], "p99_ms": wsumm["p99_ms"]}
    out["batched"] = dict(summ, streams=4, max_batch=64)
    log(f"[bench] serving batched: {summ}")
    # plain path on the first `plain_seconds` of the same log (it cannot keep up
    # with the full offered load), and the batched loop on the same prefix
    cut = int(np.searchsorted(sw.events["t"], plain_seconds))
    sub = W.ServeWorkload(sw.name, sw.host, sw.dev, sw.events[:cut].copy(), sw.label, sw.rate)
    k = int((sub.events["type"] == 0).sum())
    dw = S.serve_world(sub, host_arrays=(hv, ha))
    try:
        pres, psumm = S.run(dw, sub, S.config(plain=True))
    finally:
        dw.close()
    same = all(np.array_equal(pres[f], res[f][:k]) for f in ("flags", "first_bad", "undef_bytes", "avail"))
    lat_b = (res["t_done"][:k] - res["t_arrive"][:k]) * 1e3
    out["plain_prefix"] = dict(psumm, seconds_of_log=plain_seconds, verdicts_identical_to_batched=bool(same))
    out["batched_same_prefix"] = {"p50_ms": round(float(np.percentile(lat_b, 50)), 4),
                                  "p99_ms": round(float(np.percentile(lat_b, 99)), 4)}
    log(f"[bench] serving plain (first {plain_seconds} s): {psumm}, identical: {same}")
    return out


def concurrency_leg(records, reps=10):
    """Concurrent-access join: the 1,000,000 transfers of configuration 3 on
    8 streams with a synchronisation every 4,096 copies; whole-join time from
    events on the stream the join runs on."""
    import numpy as np
    import torch
    from paper_1310_0901_amd import workloads as W, xfercheck as X
    b = W.race_from_records(records)
    T = b.records.size
    dev = torch.device("cuda", 0)
    up = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.uint8).copy()).to(dev)
    rt, st, et = up(b.records), up(b.streams), up(b.epochs)
    out = torch.empty(T * 16, dtype=torch.uint8, device=dev)
    ctx = X.cg_create(0, 1 << 16, 16)
    try:
        s = torch.cuda.current_stream(dev)
        run = lambda: X.check_concurrent(ctx, rt.data_ptr(), st.data_ptr(), et.data_ptr(), T, out.data_ptr(),
                                         s.cuda_stream)
        for _ in range(3):
            run()
        torch.cuda.synchronize(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            run()
        e1.record(s)
        torch.cuda.synchronize(dev)
        ms = e0.elapsed_time(e1) / reps
        res = out.cpu().numpy().view(W.RACE_DTYPE)
    finally:
        X.cg_destroy(ctx)
    f = res["flags"]
    o = {"workload": "race-1M: configuration 3's transfers on 8 streams, a synchronisation every 4096 copies",
         "records": int(T), "ms_per_join": round(ms, 3), "records_per_s": round(T / (ms / 1e3), 1),
         "flagged_src": int(((f & X.CG_RACE_SRC) != 0).sum()), "flagged_dst": int(((f & X.CG_RACE_DST) != 0).sum()),
         "unchecked": int(((f & X.CG_RACE_UNCHECKED) != 0).sum())}
    log(f"[bench] concurrency: {o}")
    return o


def kernel_args_leg(reps=20):
    """Kernel-argument pointer lookups: 1,000,000 pointers against a table of
    965,250 live allocations (configuration 5's size, 1 % freed), whole-call
    time from events on the stream the lookup runs on."""
    import numpy as np
    import torch
    from paper_1310_0901_amd import workloads as W, xfercheck as X
    b = W.pointer_batch()
    dev = torch.device("cuda", 0)
    pool = int(((b.sizes.astype(np.int64) + 255) // 256 * 256).sum()) + (1 << 20)
    ctx = X.cg_create(0, pool, b.bases.size + 64)
    try:
        X.shadow_alloc_batch(ctx, b.bases, b.sizes)
        X.shadow_free_batch(ctx, b.bases[b.freed])
        p = torch.from_numpy(b.ptrs.view(np.uint8).copy()).to(dev)
        out = torch.empty(b.ptrs.size * 24, dtype=torch.uint8, device=dev)
        s = torch.cuda.current_stream(dev)
        run = lambda: X.check_pointers(ctx, p.data_ptr(), b.ptrs.size, out.data_ptr(), s.cuda_stream)
        for _ in range(3):
            run()
        torch.cuda.synchronize(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            run()
        e1.record(s)
        torch.cuda.synchronize(dev)
        ms = e0.elapsed_time(e1) / reps
        res = out.cpu().numpy().view(W.PTR_DTYPE)
    finally:
        X.cg_destroy(ctx)
    o = {"workload": b.desc, "ms_per_call": round(ms, 4), "lookups_per_s": round(b.ptrs.size / (ms / 1e3), 1),
         "unallocated": int((res["flags"] != 0).sum())}
    log(f"[bench] kernel args: {o}")
    return o


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-probe", action="store_true")
    ap.add_argument("--no-given-order", dest="given_order", action="store_false",
                    help="skip the given-order (CG_KEEP_ORDER) run of the same batch")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="skip the launch-shape autotuner (by default its cached choice is used, or it tunes)")
    ap.add_argument("--cpu-bytes", type=float, default=12e9, help="sample of the all-core oracle leg")
    ap.add_argument("--cpu-bytes-one", type=float, default=2e9, help="sample of the one-thread oracle leg")
    ap.add_argument("--no-serve", dest="serve", action="store_false", help="skip the serving leg (configuration 5)")
    ap.add_argument("--plain-serve-seconds", type=float, default=2.0)
    ap.add_argument("--no-legs", dest="legs", action="store_false",
                    help="skip the plain-at-scale and propagation legs (configurations 2 and 4)")
    ap.add_argument("--leg", choices=["plain_tiny", "plain_at_scale", "propagation", "concurrency", "kernel_args",
                                      "serving"],
                    help="run only this extra leg and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.leg:
        from paper_1310_0901_amd import workloads as W
        legs = {"plain_tiny": plain_tiny_leg, "plain_at_scale": plain_at_scale_leg, "propagation": propagation_leg,
                "concurrency": lambda: concurrency_leg(W.config3().records), "kernel_args": kernel_args_leg,
                "serving": lambda: serving_leg(args.plain_serve_seconds)}
        print(json.dumps({args.leg: legs[args.leg]()}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the multi-GPU sharding is a design "
                                   "(see the design notes), --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1310_0901_amd import workloads as W, xfercheck as X
    from paper_1310_0901_amd.harness import DeviceWorld, records_tensor, verdicts_tensor, verdicts_np

    if args.config not in (1, 2, 3):
        raise SystemExit("--config takes 1, 2 or 3 (one batch per step); configuration 4 (a propagation chain) and "
                         "configuration 5 (serving) run as legs of the default benchmark (--leg propagation, "
                         "--leg serving)")
    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t_setup = time.perf_counter()
    w = W.full_config(args.config)
    log(f"[bench] workload {w.name}: {w.count} records, {w.dev.live_idx.size} live allocations")
    hv, ha = W.host_v(w.host), W.host_a(w.host)
    dw = DeviceWorld(w, host_arrays=(hv, ha))
    ctx = dw.ctx
    T = w.count
    recs_t = records_tensor(w.records, dev)
    out_t = verdicts_tensor(T, dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    bytes_step = algo_bytes(w.records)
    log(f"[bench] set-up {time.perf_counter() - t_setup:.1f} s; {bytes_step / 1e9:.1f} GB algorithmic per step")

    tuned = None
    if args.autotune:
        t0 = time.perf_counter()
        tuned = X.cg_autotune(ctx, recs_t.data_ptr(), T, out_t.data_ptr(), X.CG_CHECK, stream, TUNE_CACHE).as_dict()
        log(f"[bench] autotune {time.perf_counter() - t0:.1f} s -> {tuned}")
    tun = X.cg_get_tuning(ctx).as_dict()

    X.cg_timing(ctx, True)
    for _ in range(args.warmup):
        X.check_transfers(ctx, recs_t.data_ptr(), T, out_t.data_ptr(), X.CG_CHECK, stream)
    torch.cuda.synchronize(dev)
    X.cg_kernel_ms(ctx)   # forget warm-up pairs
    X.cg_index_ms(ctx)
    log(f"[bench] warm-up done ({args.warmup} steps)")

    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        X.check_transfers(ctx, recs_t.data_ptr(), T, out_t.data_ptr(), X.CG_CHECK, stream)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    kms, nk = X.cg_kernel_ms(ctx)
    ims, ni, (host_read, pool_read) = X.cg_index_ms(ctx)
    got = verdicts_np(out_t, T)
    ms_step = wall * 1e3 / args.steps
    value = bytes_step * args.steps / wall / 1e9
    k_avg_ms = kms / max(nk, 1)
    i_avg_ms = ims / ni if ni else None
    pool_bytes = X.cg_stats(ctx)[1]   # allocated once, in one go: the pool's used bytes are its length
    pass_bytes = (host_read + pool_read) // ni if ni else 0   # what each counting pass read (both spaces)
    log(f"[bench] batched: {ms_step:.2f} ms/step, {value:.0f} GB/s; scan kernel {k_avg_ms:.2f} ms; index counting "
        f"pass {i_avg_ms if i_avg_ms is None else round(i_avg_ms, 2)} ms over {pass_bytes / 1e9:.1f} GB (pool: "
        f"{pool_read // max(ni, 1) / 1e9:.1f} of {pool_bytes / 1e9:.1f} GB)")

    result = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": f"{w.name} (configuration {args.config}): {w.note}",
                   "records": T, "live_allocations": int(w.dev.live_idx.size),
                   "host_region_bytes": int(w.host.length), "transfer_bytes": int(w.records["n"].sum()),
                   "mode": "check", "path": "batched: classify (marking the 64 KiB shadow steps the records read); "
                           "indexes of the faulty chunks of those steps of the host region and of the shadow pool, "
                           "read once each, answering the check-only records; source-block segments and the "
                           "persistent scan kernel for any record left; hipGraph replay",
                   "tuning": tun},
        "transfers_per_s": round(T / (wall / args.steps), 1),
        "algorithmic_bytes_per_step": int(bytes_step),
        "scan_kernel_ms": round(k_avg_ms, 3),
        "index_pass_ms": None if i_avg_ms is None else round(i_avg_ms, 3),
        "pool_bytes": int(pool_bytes),
    }
    if i_avg_ms is not None:
        # what the step reads of the shadow when the indexes answer the batch:
        # the V bytes of the pool steps its records read, and the host
        # region's V and A bytes of the steps they read, once each
        sb = int((host_read + pool_read) // args.steps)
        result["index_pass_bytes"] = int(pass_bytes)
        result["pool_bytes_read_per_pass"] = int(pool_read // max(ni, 1))
        result["shadow_bytes_read_per_step"] = sb
        result["shadow_read_GBps"] = round(sb / (wall / args.steps) / 1e9, 1)

    if not args.no_plain:
        torch.cuda.synchronize(dev)
        out_p = verdicts_tensor(T, dev)
        t0 = time.perf_counter()
        X.check_transfers(ctx, recs_t.data_ptr(), T, out_p.data_ptr(), X.CG_CHECK | X.CG_PLAIN, stream)
        torch.cuda.synchronize(dev)
        pwall = time.perf_counter() - t0
        pms, _ = X.cg_kernel_ms(ctx)
        gp = verdicts_np(out_p, T)
        same = all(np.array_equal(gp[f], got[f]) for f in ("flags", "first_bad", "undef_bytes", "avail"))
        result["plain"] = {"value": round(bytes_step / pwall / 1e9, 2), "unit": "GB/s", "ms": round(pwall * 1e3, 1),
                           "launch_loop_ms": round(pms, 1), "launches": int((w.records["n"] > 0).sum()),
                           "transfers_per_s": round(T / pwall, 1), "verdicts_identical_to_batched": bool(same)}
        result["speedup_batched_over_plain"] = round(pwall / (wall / args.steps), 2)
        log(f"[bench] plain: {pwall * 1e3:.0f} ms, identical verdicts: {same}")

    if args.given_order:
        result["given_order"] = given_order_leg(X, ctx, w, recs_t, got, T, stream, dev, bytes_step)

    if not args.no_probe:
        sink = torch.zeros(1, dtype=torch.int64, device=dev)
        nb = (dw.hv.numel() // 16) * 16
        for _ in range(2):
            X.cg_probe_read(dw.hv.data_ptr(), nb, sink.data_ptr(), stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            X.cg_probe_read(dw.hv.data_ptr(), nb, sink.data_ptr(), stream)
        e1.record()
        torch.cuda.synchronize(dev)
        rd = nb * 5 / (e0.elapsed_time(e1) / 1e3) / 1e9
        cp_bytes = 1 << 30
        src = dw.hv[:cp_bytes]
        dst = torch.empty(cp_bytes, dtype=torch.uint8, device=dev)
        X.cg_probe_copy(dst.data_ptr(), src.data_ptr(), cp_bytes, stream)
        e0.record()
        for _ in range(5):
            X.cg_probe_copy(dst.data_ptr(), src.data_ptr(), cp_bytes, stream)
        e1.record()
        torch.cuda.synchronize(dev)
        # read + write bytes: the practical ceiling of the propagating variant
        cp = 2 * cp_bytes * 5 / (e0.elapsed_time(e1) / 1e3) / 1e9
        del dst
        l2 = probe_l2(X, dev, stream)
        result["probe_read_GBps"] = round(rd, 1)
        result["probe_copy_GBps"] = round(cp, 1)
        result["probe_l2_read"] = l2
        log(f"[bench] probe read {rd:.0f} GB/s, copy {cp:.0f} GB/s (read + write), L2-resident read {l2}")

    result["roofline"] = roofline(tun, args.config, k_avg_ms, i_avg_ms, pass_bytes, bytes_step,
                                  result.get("probe_l2_read", {}).get("GBps"))
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline_legs(w, hv, ha, got, args.cpu_bytes, args.cpu_bytes_one)
    dw.close()
    if args.legs:
        result["concurrency"] = concurrency_leg(w.records)
        result["kernel_args"] = kernel_args_leg()
        result["plain_tiny"] = plain_tiny_leg()
        result["plain_at_scale"] = plain_at_scale_leg()
        result["propagation"] = propagation_leg()
    if args.serve:
        result["serving"] = serving_leg(args.plain_serve_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
