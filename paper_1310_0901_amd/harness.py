"""Device-side set-up of a workload for the transfer checker, through the C ABI.

Builds, for a workloads.Workload, the checker context on the GPU: uploads the
host region's V bytes and A bitmap (caller-owned device mirrors, held here as
torch tensors), registers the live allocations (shadow_alloc_batch), writes
their initial shadow (shadow_set_batch) and stages the records in device
memory.  torch provides device memory and streams only; every check runs in
the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import workloads as W
from . import xfercheck as X

_hip = None


def _hiprt():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.restype = ctypes.c_int
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return _hip


def copy_raw(dst: int, src: int, nbytes: int, kind: int) -> None:
    """hipMemcpy between raw addresses (kind 1 H2D, 2 D2H, 3 D2D)."""
    if nbytes:
        rc = _hiprt().hipMemcpy(dst, src, nbytes, kind)
        if rc != 0:
            raise RuntimeError(f"hipMemcpy failed ({rc})")


def read_device(ptr: int, nbytes: int) -> np.ndarray:
    out = np.empty(nbytes, np.uint8)
    copy_raw(out.ctypes.data, ptr, nbytes, 2)
    return out


def device_view(ptr: int, nbytes: int, device="cuda") -> torch.Tensor:
    """A device copy of [ptr, ptr + nbytes)."""
    t = torch.empty(nbytes, dtype=torch.uint8, device=device)
    torch.cuda.synchronize()
    copy_raw(t.data_ptr(), ptr, nbytes, 3)
    return t


def records_tensor(recs: np.ndarray, device="cuda") -> torch.Tensor:
    r = np.ascontiguousarray(recs, W.RECORD_DTYPE)
    return torch.from_numpy(r.view(np.uint8).copy()).to(device)


def verdicts_tensor(count: int, device="cuda") -> torch.Tensor:
    return torch.empty(max(count, 1) * 32, dtype=torch.uint8, device=device)


def verdicts_np(t: torch.Tensor, count: int) -> np.ndarray:
    return t[: count * 32].cpu().numpy().view(W.VERDICT_DTYPE).copy()


class DeviceWorld:
    """Checker context holding a workload's host region and allocations."""

    def __init__(self, w: W.Workload, device: int = 0, pool_slack: int = 1 << 24, max_allocs=None,
                 host_arrays=None):
        self.w = w
        self.dev = torch.device("cuda", device)
        live = w.dev.live_idx
        sizes = w.dev.size[live].astype(np.int64)
        pool = int(((sizes + 255) // 256 * 256).sum()) + pool_slack
        self.max_allocs = max_allocs or max(16, int(live.size) + 16)
        self.ctx = X.cg_create(device, pool, self.max_allocs)
        hv, ha = host_arrays if host_arrays is not None else (W.host_v(w.host), W.host_a(w.host))
        hl = w.host.length
        self.hv = torch.zeros(((hl + 15) // 16) * 16 + 16, dtype=torch.uint8, device=self.dev)
        self.hv[:hl].copy_(torch.from_numpy(hv))
        self.ha = torch.from_numpy(np.ascontiguousarray(ha, np.uint64).view(np.int64)).to(self.dev)
        X.cg_host_register(self.ctx, w.host.base, hl, self.hv.data_ptr(), self.ha.data_ptr())
        X.shadow_alloc_batch(self.ctx, w.dev.base[live], w.dev.size[live])
        z = live[w.dev.init[live] != 0xFF]
        if z.size:
            X.shadow_set_batch(self.ctx, w.dev.base[z], w.dev.size[z], w.dev.init[z])
        r = np.asarray(w.dev.runs, np.int64).reshape(-1, 4)
        r = r[w.dev.live[r[:, 0]]] if r.shape[0] else r
        if r.shape[0]:
            X.shadow_set_batch(self.ctx, w.dev.base[r[:, 0]].astype(np.uint64) + r[:, 1].astype(np.uint64),
                               r[:, 2], r[:, 3])
        X.cg_sync(self.ctx)

    def close(self):
        if self.ctx:
            torch.cuda.synchronize()
            X.cg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, recs: np.ndarray, mode=X.CG_CHECK, stream=None) -> np.ndarray:
        rt = records_tensor(recs, self.dev)
        out = verdicts_tensor(len(recs), self.dev)
        s = stream if stream is not None else torch.cuda.current_stream(self.dev).cuda_stream
        X.check_transfers(self.ctx, rt.data_ptr(), len(recs), out.data_ptr(), mode, s)
        torch.cuda.synchronize(self.dev)
        return verdicts_np(out, len(recs))

    def alloc_shadow(self, base: int, size: int) -> np.ndarray:
        torch.cuda.synchronize(self.dev)
        X.cg_sync(self.ctx)
        return read_device(X.shadow_ptr(self.ctx, int(base)), int(size))

    def host_shadow(self) -> np.ndarray:
        torch.cuda.synchronize(self.dev)
        return self.hv[: self.w.host.length].cpu().numpy()
