"""Serving driver: runs an event log through the library's continuous-batching
loop (cg_serve_run) and summarises latency and throughput.

The loop itself is native (runtime.cpp): requests are admitted as they
arrive while the shadow bytes in flight stay under the admission cap and a
slot (stream) is free; each micro-batch is one graph replay of the batched
check on its slot's stream, so micro-batches overlap on the device;
allocation and free events are applied in arrival order, each request being
checked against the table as of its arrival.  This module only prepares the
context and reads the results.
"""
from __future__ import annotations

import numpy as np

from . import workloads as W
from . import xfercheck as X
from .harness import DeviceWorld


def serve_world(sw: W.ServeWorkload, device: int = 0, host_arrays=None) -> DeviceWorld:
    """Checker context holding the initial state of a serving workload, with
    room for the allocations the log makes."""
    ev = sw.events
    grow = ev["type"] == W.EV_ALLOC
    extra = int(((ev["n"][grow].astype(np.int64) + 255) // 256 * 256).sum())
    max_allocs = int(sw.dev.live_idx.size + grow.sum() + 64)
    return DeviceWorld(sw, device=device, pool_slack=extra + (64 << 20), max_allocs=max_allocs,
                       host_arrays=host_arrays)


def config(streams=4, max_batch=512, mem_cap=16 << 30, plain=False, open_loop=True, blocks_per_cu=1):
    c = X.cg_serve_config()
    c.streams, c.max_batch, c.mem_cap = streams, max_batch, mem_cap
    c.plain, c.open_loop, c.blocks_per_cu = int(plain), int(open_loop), blocks_per_cu
    return c


def run(dw: DeviceWorld, sw: W.ServeWorkload, cfg) -> tuple[np.ndarray, dict]:
    import torch
    torch.cuda.synchronize()
    res, st = X.cg_serve_run(dw.ctx, sw.events, cfg)
    return res, summarise(sw, res, st)


def algo_bytes(recs) -> float:
    n = recs["n"].astype(np.float64)
    return float((n * np.where(recs["kind"] == W.KIND_D2D, 1.0, 1.125)).sum())


def summarise(sw: W.ServeWorkload, res: np.ndarray, st) -> dict:
    lat = (res["t_done"] - res["t_arrive"]) * 1e3
    q = sw.requests
    wall = st.wall_s
    return {
        "requests": int(res.size), "wall_s": round(wall, 4),
        "req_per_s": round(res.size / wall, 1),
        "GBps": round(algo_bytes(q) / wall / 1e9, 3),
        "p50_ms": round(float(np.percentile(lat, 50)), 4),
        "p99_ms": round(float(np.percentile(lat, 99)), 4),
        "mean_ms": round(float(lat.mean()), 4),
        "max_ms": round(float(lat.max()), 4),
        # where the latency goes: arrival to issue (the host loop, waiting
        # for a free slot), issue to completion on the GPU
        "p50_wait_ms": round(float(np.percentile((res["t_admit"] - res["t_arrive"]) * 1e3, 50)), 4),
        "p50_gpu_ms": round(float(np.percentile((res["t_done"] - res["t_admit"]) * 1e3, 50)), 4),
        "batches": int(st.batches), "mean_batch": round(st.mean_batch, 2),
        "events_applied": int(st.events), "table_versions": int(st.table_versions),
        "max_inflight_GB": round(st.max_inflight_bytes / 1e9, 3),
        "offered_req_per_s": sw.rate,
    }
