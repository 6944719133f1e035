"""Python binding of libxfercheck.so: the C ABI of include/xfercheck.h with
the same names, argument marshalling only.  Pointers are plain integers
(device addresses, e.g. torch's tensor.data_ptr()); streams are hipStream_t
handles as integers (torch.cuda.current_stream().cuda_stream) or 0.

Every check runs in the HIP kernels of the library.  If the library is not
built, loading fails with an error: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxfercheck.so")

# status codes
CG_OK, CG_EINVAL, CG_ENOMEM, CG_EOVERLAP, CG_ENOTFOUND = 0, -1, -2, -3, -4
CG_ECONFLICT, CG_ECAPACITY, CG_EHIP, CG_ESTATE = -5, -6, -7, -8
# kinds
CG_H2D, CG_D2H, CG_D2D = 0, 1, 2
# flags
CG_SRC_UNADDR, CG_SRC_UNDEF, CG_SRC_UNALLOC, CG_SRC_OVERRUN = 0x1, 0x2, 0x4, 0x8
CG_DST_UNADDR, CG_DST_UNALLOC, CG_DST_OVERRUN = 0x10, 0x20, 0x40
CG_OVERLAP, CG_BAD_KIND, CG_ROWS_LIMIT = 0x80, 0x100, 0x200
CG_NONE = 0xFFFF_FFFF_FFFF_FFFF
CG_RACE_SRC, CG_RACE_DST, CG_RACE_UNCHECKED = 0x1, 0x2, 0x4
CG_PTR_UNALLOC = 0x1
# modes
CG_CHECK, CG_PROPAGATE, CG_PLAIN, CG_DEBUG_CONFLICTS, CG_EAGER, CG_KEEP_ORDER = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20
CG_NOALLOC_MAX = 4096


class CgError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        self.status = status
        super().__init__(f"{what}: {cg_strerror(status)} ({status})" + (f": {detail}" if detail else ""))


class cg_transfer(ctypes.Structure):
    _fields_ = [("src", ctypes.c_uint64), ("dst", ctypes.c_uint64), ("n", ctypes.c_uint64),
                ("kind", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class cg_verdict(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("first_bad", ctypes.c_uint64),
                ("undef_bytes", ctypes.c_uint64), ("avail", ctypes.c_uint64)]


class cg_tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_uint32), ("unroll", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32),
                ("tile_units", ctypes.c_uint32), ("nontemporal", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 3)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k in ("block", "unroll", "blocks_per_cu", "tile_units", "nontemporal")}


class cg_serve_config(ctypes.Structure):
    _fields_ = [("streams", ctypes.c_uint32), ("max_batch", ctypes.c_uint32), ("mem_cap", ctypes.c_uint64),
                ("plain", ctypes.c_uint32), ("open_loop", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class cg_serve_stats(ctypes.Structure):
    _fields_ = [("wall_s", ctypes.c_double), ("requests", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("events", ctypes.c_uint64), ("max_inflight_bytes", ctypes.c_uint64),
                ("table_versions", ctypes.c_uint64), ("mean_batch", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


CG_EV_CHECK, CG_EV_ALLOC, CG_EV_FREE = 0, 1, 2

_lib = None
P, U64, U32, I32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
PU64 = ctypes.POINTER(ctypes.c_uint64)
PU8 = ctypes.POINTER(ctypes.c_uint8)

_PROTOS = {
    "cg_create": (I32, [ctypes.POINTER(P), I32, U64, U64]),
    "cg_destroy": (I32, [P]),
    "cg_host_register": (I32, [P, U64, U64, P, P]),
    "shadow_alloc": (I32, [P, U64, U64]),
    "shadow_free": (I32, [P, U64]),
    "shadow_alloc_batch": (I32, [P, P, P, U64]),
    "shadow_free_batch": (I32, [P, P, U64]),
    "shadow_set": (I32, [P, U64, U64, ctypes.c_uint8]),
    "shadow_set_batch": (I32, [P, P, P, P, U64]),
    "shadow_ptr": (I32, [P, U64, ctypes.POINTER(P)]),
    "check_transfers": (I32, [P, P, U64, P, U32, P]),
    "check_transfers_noalloc": (I32, [P, P, U64, P, U32, P]),
    "propagate_shadow": (I32, [P, P, U64, P]),
    "check_concurrent": (I32, [P, P, P, P, U64, P, P]),
    "check_pointers": (I32, [P, P, U64, P, P]),
    "check_transfers_2d": (I32, [P, P, U64, P, U32, P]),
    "cg_format_verdict": (I32, [ctypes.POINTER(cg_transfer), ctypes.POINTER(cg_verdict), ctypes.c_char_p, U64]),
    "cg_strerror": (ctypes.c_char_p, [I32]),
    "cg_last_error": (ctypes.c_char_p, [P]),
    "cg_sync": (I32, [P]),
    "cg_stats": (I32, [P, PU64, PU64]),
    "cg_table_read": (I32, [P, P, P, P, U64, PU64, P, U32, ctypes.POINTER(U32), ctypes.POINTER(U32), PU64, PU64,
                            PU64]),
    "cg_get_tuning": (I32, [P, ctypes.POINTER(cg_tuning)]),
    "cg_set_tuning": (I32, [P, ctypes.POINTER(cg_tuning)]),
    "cg_autotune": (I32, [P, P, U64, P, U32, P, ctypes.c_char_p, ctypes.POINTER(cg_tuning)]),
    "cg_timing": (I32, [P, I32]),
    "cg_kernel_ms": (I32, [P, ctypes.POINTER(ctypes.c_double), PU64]),
    "cg_index_ms": (I32, [P, ctypes.POINTER(ctypes.c_double), PU64, P]),
    "cg_probe_read": (I32, [P, U64, P, P]),
    "cg_probe_copy": (I32, [P, P, U64, P]),
    "cg_probe_l2": (I32, [P, U64, U32, U32, P, P]),
    "cg_serve_run": (I32, [P, P, U64, ctypes.POINTER(cg_serve_config), P, ctypes.POINTER(cg_serve_stats)]),
}

EXPORTS = tuple(_PROTOS)


def lib():
    """Load the HIP library (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1310_0901_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def cg_strerror(status: int) -> str:
    return lib().cg_strerror(status).decode()


def _chk(ctx, status, what):
    if status != CG_OK:
        detail = lib().cg_last_error(ctx).decode() if ctx else ""
        raise CgError(status, what, detail)


# ---- the C ABI, same names ---------------------------------------------------

def cg_create(hip_device: int, shadow_pool_bytes: int, max_allocs: int) -> int:
    h = P()
    _chk(None, lib().cg_create(ctypes.byref(h), hip_device, shadow_pool_bytes, max_allocs), "cg_create")
    return h.value


def cg_destroy(ctx: int) -> None:
    _chk(None, lib().cg_destroy(ctx), "cg_destroy")


def cg_host_register(ctx, host_base, length, v_dev, a_bits_dev) -> None:
    _chk(ctx, lib().cg_host_register(ctx, host_base, length, v_dev, a_bits_dev), "cg_host_register")


def shadow_alloc(ctx, dev_addr, size) -> None:
    _chk(ctx, lib().shadow_alloc(ctx, dev_addr, size), "shadow_alloc")


def shadow_free(ctx, dev_addr) -> None:
    _chk(ctx, lib().shadow_free(ctx, dev_addr), "shadow_free")


def shadow_alloc_batch(ctx, addrs, sizes) -> None:
    import numpy as np
    a = np.ascontiguousarray(addrs, np.uint64)
    s = np.ascontiguousarray(sizes, np.uint64)
    assert a.size == s.size
    _chk(ctx, lib().shadow_alloc_batch(ctx, a.ctypes.data, s.ctypes.data, a.size), "shadow_alloc_batch")


def shadow_free_batch(ctx, addrs) -> None:
    import numpy as np
    a = np.ascontiguousarray(addrs, np.uint64)
    _chk(ctx, lib().shadow_free_batch(ctx, a.ctypes.data, a.size), "shadow_free_batch")


def shadow_set(ctx, dev_addr, n, v) -> None:
    _chk(ctx, lib().shadow_set(ctx, dev_addr, n, v), "shadow_set")


def shadow_set_batch(ctx, addrs, ns, vs) -> None:
    import numpy as np
    a = np.ascontiguousarray(addrs, np.uint64)
    n = np.ascontiguousarray(ns, np.uint64)
    v = np.ascontiguousarray(vs, np.uint8)
    assert a.size == n.size == v.size
    _chk(ctx, lib().shadow_set_batch(ctx, a.ctypes.data, n.ctypes.data, v.ctypes.data, a.size), "shadow_set_batch")


def shadow_ptr(ctx, dev_addr) -> int:
    p = P()
    _chk(ctx, lib().shadow_ptr(ctx, dev_addr, ctypes.byref(p)), "shadow_ptr")
    return p.value


def check_transfers(ctx, recs_dev, count, out_dev, mode, stream=0) -> None:
    _chk(ctx, lib().check_transfers(ctx, recs_dev, count, out_dev, mode, stream), "check_transfers")


def check_transfers_noalloc(ctx, recs_dev, count, out_dev, mode, stream=0) -> None:
    _chk(ctx, lib().check_transfers_noalloc(ctx, recs_dev, count, out_dev, mode, stream), "check_transfers_noalloc")


def propagate_shadow(ctx, recs_dev, count, stream=0) -> None:
    _chk(ctx, lib().propagate_shadow(ctx, recs_dev, count, stream), "propagate_shadow")


def check_concurrent(ctx, recs_dev, streams_dev, epochs_dev, count, out_dev, stream=0) -> None:
    """epochs_dev may be 0/None (all records in epoch 0)."""
    _chk(ctx, lib().check_concurrent(ctx, recs_dev, streams_dev, epochs_dev or None, count, out_dev, stream),
         "check_concurrent")


def check_transfers_2d(ctx, recs_dev, count, out_dev, mode, stream=0) -> None:
    _chk(ctx, lib().check_transfers_2d(ctx, recs_dev, count, out_dev, mode, stream), "check_transfers_2d")


def check_pointers(ctx, ptrs_dev, count, out_dev, stream=0) -> None:
    _chk(ctx, lib().check_pointers(ctx, ptrs_dev, count, out_dev, stream), "check_pointers")


def cg_format_verdict(rec, verdict) -> str:
    """rec / verdict: (src, dst, n, kind) and (flags, first_bad, undef_bytes, avail) tuples."""
    r = cg_transfer(int(rec[0]), int(rec[1]), int(rec[2]), int(rec[3]), 0)
    v = cg_verdict(int(verdict[0]), 0, int(verdict[1]), int(verdict[2]), int(verdict[3]))
    n = lib().cg_format_verdict(ctypes.byref(r), ctypes.byref(v), None, 0)
    if n < 0:
        raise CgError(n, "cg_format_verdict")
    buf = ctypes.create_string_buffer(n + 1)
    lib().cg_format_verdict(ctypes.byref(r), ctypes.byref(v), buf, n + 1)
    return buf.value.decode()


def cg_last_error(ctx) -> str:
    return lib().cg_last_error(ctx).decode()


def cg_sync(ctx) -> None:
    _chk(ctx, lib().cg_sync(ctx), "cg_sync")


def cg_table_read(ctx, cap, top_cap=1024) -> dict:
    """Host copy of the device table (test hook): base, end, off, top arrays,
    shift, pool address, merges and full uploads so far."""
    import numpy as np
    b, e, o = (np.zeros(cap, np.uint64) for _ in range(3))
    t = np.zeros(top_cap, np.uint64)
    n, pool, merges, full = (ctypes.c_uint64() for _ in range(4))
    ntop, shift = ctypes.c_uint32(), ctypes.c_uint32()
    _chk(ctx, lib().cg_table_read(ctx, b.ctypes.data, e.ctypes.data, o.ctypes.data, cap, ctypes.byref(n),
                                  t.ctypes.data, top_cap, ctypes.byref(ntop), ctypes.byref(shift), ctypes.byref(pool),
                                  ctypes.byref(merges), ctypes.byref(full)), "cg_table_read")
    k = n.value
    return {"base": b[:k], "end": e[:k], "off": o[:k], "top": t[:ntop.value], "shift": shift.value,
            "pool": pool.value, "merges": merges.value, "full_uploads": full.value}


def cg_stats(ctx):
    a, b = ctypes.c_uint64(), ctypes.c_uint64()
    _chk(ctx, lib().cg_stats(ctx, ctypes.byref(a), ctypes.byref(b)), "cg_stats")
    return a.value, b.value


def cg_get_tuning(ctx) -> cg_tuning:
    t = cg_tuning()
    _chk(ctx, lib().cg_get_tuning(ctx, ctypes.byref(t)), "cg_get_tuning")
    return t


def cg_set_tuning(ctx, t: cg_tuning) -> None:
    _chk(ctx, lib().cg_set_tuning(ctx, ctypes.byref(t)), "cg_set_tuning")


def cg_autotune(ctx, recs_dev, count, out_dev, mode, stream=0, cache_path=None) -> cg_tuning:
    t = cg_tuning()
    cp = cache_path.encode() if cache_path else None
    _chk(ctx, lib().cg_autotune(ctx, recs_dev, count, out_dev, mode, stream, cp, ctypes.byref(t)), "cg_autotune")
    return t


def cg_timing(ctx, enable: bool) -> None:
    _chk(ctx, lib().cg_timing(ctx, 1 if enable else 0), "cg_timing")


def cg_kernel_ms(ctx):
    ms, n = ctypes.c_double(), ctypes.c_uint64()
    _chk(ctx, lib().cg_kernel_ms(ctx, ctypes.byref(ms), ctypes.byref(n)), "cg_kernel_ms")
    return ms.value, n.value


def cg_index_ms(ctx):
    """(summed ms, timed passes, (host region bytes, pool bytes) read by the
    counting passes) since the last call."""
    ms, n = ctypes.c_double(), ctypes.c_uint64()
    b = (ctypes.c_uint64 * 2)()
    _chk(ctx, lib().cg_index_ms(ctx, ctypes.byref(ms), ctypes.byref(n), ctypes.cast(b, ctypes.c_void_p)),
         "cg_index_ms")
    return ms.value, n.value, (b[0], b[1])


def cg_probe_read(dev, nbytes, sink_dev, stream=0) -> None:
    _chk(None, lib().cg_probe_read(dev, nbytes, sink_dev, stream), "cg_probe_read")


def cg_probe_copy(dst, src, nbytes, stream=0) -> None:
    _chk(None, lib().cg_probe_copy(dst, src, nbytes, stream), "cg_probe_copy")


def cg_probe_l2(dev, slice_bytes, passes, blocks, sink_dev, stream=0) -> None:
    _chk(None, lib().cg_probe_l2(dev, slice_bytes, passes, blocks, sink_dev, stream), "cg_probe_l2")


def cg_serve_run(ctx, events, cfg: cg_serve_config):
    """events: numpy array of workloads.SERVE_EVENT_DTYPE (host).  Returns
    (results as workloads.SERVE_RESULT_DTYPE, stats)."""
    import numpy as np
    from .workloads import SERVE_EVENT_DTYPE, SERVE_RESULT_DTYPE
    ev = np.ascontiguousarray(events, SERVE_EVENT_DTYPE)
    nreq = int((ev["type"] == CG_EV_CHECK).sum())
    res = np.zeros(max(nreq, 1), SERVE_RESULT_DTYPE)
    st = cg_serve_stats()
    _chk(ctx, lib().cg_serve_run(ctx, ev.ctypes.data, ev.size, ctypes.byref(cfg), res.ctypes.data, ctypes.byref(st)),
         "cg_serve_run")
    return res[:nreq], st
