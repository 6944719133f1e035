// HIP API interposer: the wrapper deployment of the method, for HIP programs.
//
// The paper places its wrappers around the driver API's allocation, free and
// copy functions (Sec. 1.2, Sec. 2, Fig. 1) and loads them before the driver
// library (Sec. 3), so that every copy is checked against the context's list
// of allocations before it runs and a report names the bytes the copy needs
// and the bytes the allocation holds (Sec. 4.5, Listing 6).  Here the same
// wrappers sit around hipMalloc / hipFree / hipMemset / hipMemcpy*, loaded
// with LD_PRELOAD, and feed the transfer checker (xfercheck.h):
//   hipMalloc  -> shadow_alloc (new memory is not defined yet)
//   hipFree    -> shadow_free
//   hipMemset  -> shadow_set(0) (the bytes become defined)
//   hipMemcpy  -> check_transfers on one record, report, then the real copy;
//                 host->device and device->device copies also carry the V
//                 bits into the destination shadow.
// The host program itself is not instrumented, so host bytes of a copy count
// as addressable and defined.  Kernels are not instrumented either (the
// paper's outlook, Sec. 5.1), so undefined-source notes for device sources
// are off unless XC_REPORT_DEVICE_UNDEF=1.
//
// A copy whose device side is unallocated or too small is not performed (the
// call returns hipErrorInvalidValue, as the driver in the paper's example
// fails the call with an invalid-argument error), unless XC_ALLOW_BAD=1.
//
// hipMemcpyAsync is checked when it is issued; hipMemcpy2D is checked as one
// batch of its rows (strided copies, the case of the paper's footnote to
// the error list of Sec. 2) and reported once, with its first faulty row.
//
// Concurrent accesses (the error class of Sec. 2 for programs with several
// threads): every asynchronous copy that was performed joins a window, with
// the stream it was issued on.  The next synchronising call (device, stream
// or event synchronisation, a stream waiting for an event, a synchronous copy
// or hipFree) closes the window: check_concurrent joins its copies, and every
// pair on different streams where one writes bytes the other reads or writes
// is reported.  Copies of one window are taken as unordered unless they share
// a stream; copies in different windows as ordered, so a race across a
// synchronising call is not reported (no false reports, possibly missed ones).
// Work on the null stream (stream 0) waits for all earlier work on blocking
// streams and all later work on them waits for it, so an asynchronous copy,
// fill or kernel launch on stream 0 also closes the window, before and after
// its own copy; copies on non-blocking streams (hipStreamNonBlocking) are not
// ordered by it and stay in the window, and a pair is reported once.
//
// Kernel arguments (the outlook of Sec. 5.1): hipLaunchKernel is wrapped, the
// kernel's parameter list is recovered by demangling its name, and every
// raw-pointer argument that is neither null nor pinned host memory is looked
// up among the live allocations with check_pointers.  A pointer that is
// neither inside nor one past the end of a live allocation (freed or never
// allocated) is reported and the launch is refused.  Pointers inside structs
// passed by value, and kernels declared extern "C" (no parameter types in
// their names), are not checked.  XC_NO_KERNEL_ARGS=1 turns this off.
//
// Environment: XC_POOL_BYTES (shadow pool, default 1 GiB), XC_MAX_ALLOCS
// (default 1,048,576), XC_REPORT_DEVICE_UNDEF, XC_ALLOW_BAD, XC_QUIET=1 (no
// summary line), XC_NO_KERNEL_ARGS.
#include <cxxabi.h>
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/xfercheck.h"

namespace {

thread_local int inside = 0;   // > 0 while the checker itself calls HIP
// the error of the last call this thread refused, reported by hipGetLastError /
// hipPeekAtLastError like the runtime's own errors
thread_local hipError_t refused = hipSuccess;

hipError_t refuse()
{
    refused = hipErrorInvalidValue;
    return hipErrorInvalidValue;
}

struct Guard {
    Guard() { ++inside; }
    ~Guard() { --inside; }
};

template <typename F>
F real(const char *name)
{
    return reinterpret_cast<F>(dlsym(RTLD_NEXT, name));
}

using malloc_t = hipError_t (*)(void **, size_t);
using free_t = hipError_t (*)(void *);
using memset_t = hipError_t (*)(void *, int, size_t);
using memcpy_t = hipError_t (*)(void *, const void *, size_t, hipMemcpyKind);
using htod_t = hipError_t (*)(hipDeviceptr_t, const void *, size_t);
using dtoh_t = hipError_t (*)(void *, hipDeviceptr_t, size_t);
using dtod_t = hipError_t (*)(hipDeviceptr_t, hipDeviceptr_t, size_t);
using memcpy_async_t = hipError_t (*)(void *, const void *, size_t, hipMemcpyKind, hipStream_t);
using memcpy2d_t = hipError_t (*)(void *, size_t, const void *, size_t, size_t, size_t, hipMemcpyKind);
using devsync_t = hipError_t (*)();
using streamsync_t = hipError_t (*)(hipStream_t);
using eventsync_t = hipError_t (*)(hipEvent_t);
using waitevent_t = hipError_t (*)(hipStream_t, hipEvent_t, unsigned int);
using launch_t = hipError_t (*)(const void *, dim3, dim3, void **, size_t, hipStream_t);
using malloc_flags_t = hipError_t (*)(void **, size_t, unsigned int);
using malloc_async_t = hipError_t (*)(void **, size_t, hipStream_t);
using free_async_t = hipError_t (*)(void *, hipStream_t);
using lasterr_t = hipError_t (*)();
using memcpy2d_async_t = hipError_t (*)(void *, size_t, const void *, size_t, size_t, size_t, hipMemcpyKind,
                                        hipStream_t);
using memcpy3d_t = hipError_t (*)(const hipMemcpy3DParms *);
using memcpy3d_async_t = hipError_t (*)(const hipMemcpy3DParms *, hipStream_t);
using malloc_pitch_t = hipError_t (*)(void **, size_t *, size_t, size_t);
using malloc3d_t = hipError_t (*)(hipPitchedPtr *, hipExtent);
using memset_async_t = hipError_t (*)(void *, int, size_t, hipStream_t);
using memset_d8_t = hipError_t (*)(hipDeviceptr_t, unsigned char, size_t);
using memset_d8_async_t = hipError_t (*)(hipDeviceptr_t, unsigned char, size_t, hipStream_t);
using memset_d16_t = hipError_t (*)(hipDeviceptr_t, unsigned short, size_t);
using memset_d16_async_t = hipError_t (*)(hipDeviceptr_t, unsigned short, size_t, hipStream_t);
using memset_d32_t = hipError_t (*)(hipDeviceptr_t, int, size_t);
using memset_d32_async_t = hipError_t (*)(hipDeviceptr_t, int, size_t, hipStream_t);
using htod_async_t = hipError_t (*)(hipDeviceptr_t, const void *, size_t, hipStream_t);
using dtoh_async_t = hipError_t (*)(void *, hipDeviceptr_t, size_t, hipStream_t);
using dtod_async_t = hipError_t (*)(hipDeviceptr_t, hipDeviceptr_t, size_t, hipStream_t);

// a kernel's parameter list as far as its name tells it
struct KernelSig {
    std::string name;              // demangled signature (or the name as given)
    std::vector<std::string> params;
    std::vector<bool> is_ptr;
    bool known = false;            // parameter types recovered
};

// an asynchronous copy waiting in the window
// An asynchronous copy (or fill) in the concurrent-access window.  A fill
// writes [dst, dst + n); it joins as a D2D record with src = dst, so every
// pair it takes part in involves its write.
struct WinCopy {
    cg_transfer r;
    hipStream_t stream;
    const char *api = "hipMemcpyAsync";
    bool fill = false;
    uint64_t seq = 0;   // issue order, names the copy in reported pairs
};

// A window this long is joined at once, as if a synchronising call had come:
// a race between copies on both sides of that point is not reported.
constexpr size_t kWindowMax = size_t(1) << 20;

struct State {
    std::mutex mu;
    cg_ctx *ctx = nullptr;
    bool failed = false;
    hipStream_t s = nullptr;
    cg_transfer *d_rec = nullptr;
    cg_verdict *d_ver = nullptr;
    uint64_t rec_cap = 1;         // records d_rec / d_ver hold
    cg_transfer2d *d_rec2d = nullptr;
    cg_verdict *d_ver2d = nullptr;
    uint64_t slice_cap = 0;       // pitched records d_rec2d / d_ver2d hold
    uint8_t *zeros = nullptr;     // V of "defined" host bytes
    uint64_t *ones = nullptr;     // A of "addressable" host bytes
    uint64_t cap = 0;             // bytes covered by zeros / ones
    bool device_undef = false;
    bool allow_bad = false;
    bool quiet = false;
    uint64_t copies = 0, errors = 0;
    // the window of asynchronous copies since the last synchronising call
    std::vector<WinCopy> win;
    uint64_t win_seq = 0;
    std::set<std::pair<uint64_t, uint64_t>> reported;   // pairs (by seq) reported while their copies stay in the window
    cg_transfer *d_wrec = nullptr;
    uint32_t *d_wsid = nullptr;
    cg_race *d_wres = nullptr;
    uint64_t win_cap = 0;
    uint64_t races = 0;
    // kernel arguments
    bool kernel_args = true;
    std::unordered_map<const void *, KernelSig> sigs;
    uint64_t *d_ptrs = nullptr;
    cg_ptr_check *d_pres = nullptr;
    uint64_t ptr_cap = 0;
    uint64_t launches = 0;
} G;

uint64_t env_u64(const char *k, uint64_t d)
{
    const char *v = getenv(k);
    return v ? strtoull(v, nullptr, 0) : d;
}

void summary()
{
    if (G.ctx && !G.quiet) {
        fprintf(stderr, "==xfercheck== %" PRIu64 " copies checked, %" PRIu64 " with errors", G.copies, G.errors);
        if (G.launches) fprintf(stderr, ", %" PRIu64 " kernel launches checked", G.launches);
        if (G.races) fprintf(stderr, ", %" PRIu64 " concurrent-access pairs", G.races);
        fprintf(stderr, "\n");
    }
}

bool ensure_ctx()
{
    if (G.ctx) return true;
    if (G.failed) return false;
    Guard g;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const uint64_t pool = env_u64("XC_POOL_BYTES", 1ull << 30);
    const uint64_t maxa = env_u64("XC_MAX_ALLOCS", 1ull << 20);
    int rc = cg_create(&G.ctx, dev, pool, maxa);
    if (rc == CG_OK && hipStreamCreateWithFlags(&G.s, hipStreamNonBlocking) != hipSuccess) rc = CG_EHIP;
    if (rc == CG_OK && hipMalloc(reinterpret_cast<void **>(&G.d_rec), sizeof(cg_transfer)) != hipSuccess) rc = CG_ENOMEM;
    if (rc == CG_OK && hipMalloc(reinterpret_cast<void **>(&G.d_ver), sizeof(cg_verdict)) != hipSuccess) rc = CG_ENOMEM;
    if (rc != CG_OK) {
        fprintf(stderr, "==xfercheck== cannot start the checker: %s\n", cg_strerror(rc));
        G.failed = true;
        G.ctx = nullptr;
        return false;
    }
    G.device_undef = env_u64("XC_REPORT_DEVICE_UNDEF", 0) != 0;
    G.allow_bad = env_u64("XC_ALLOW_BAD", 0) != 0;
    G.quiet = env_u64("XC_QUIET", 0) != 0;
    G.kernel_args = env_u64("XC_NO_KERNEL_ARGS", 0) == 0;
    atexit(summary);
    return true;
}

// zeros / ones buffers covering at least n host bytes
bool ensure_host_cover(uint64_t n)
{
    if (n <= G.cap) return true;
    Guard g;
    uint64_t cap = G.cap ? G.cap : (1ull << 20);
    while (cap < n) cap <<= 1;
    (void)hipStreamSynchronize(G.s);
    (void)hipFree(G.zeros);
    (void)hipFree(G.ones);
    G.zeros = nullptr;
    G.ones = nullptr;
    if (hipMalloc(reinterpret_cast<void **>(&G.zeros), cap + 16) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&G.ones), cap / 8 + 8) != hipSuccess ||
        hipMemsetAsync(G.zeros, 0, cap + 16, G.s) != hipSuccess ||
        hipMemsetAsync(G.ones, 0xFF, cap / 8 + 8, G.s) != hipSuccess ||
        hipStreamSynchronize(G.s) != hipSuccess) {
        G.cap = 0;
        return false;
    }
    G.cap = cap;
    return true;
}

const char *kind_name(uint32_t k)
{
    return k == CG_H2D ? "hipMemcpyHostToDevice" : k == CG_D2H ? "hipMemcpyDeviceToHost" : "hipMemcpyDeviceToDevice";
}

constexpr uint32_t kRangeFaults = CG_SRC_UNALLOC | CG_SRC_OVERRUN | CG_DST_UNALLOC | CG_DST_OVERRUN;

// records / verdicts buffers for at least k rows
bool ensure_rows(uint64_t k)
{
    if (k <= G.rec_cap) return true;
    Guard g;
    (void)hipStreamSynchronize(G.s);
    (void)hipFree(G.d_rec);
    (void)hipFree(G.d_ver);
    G.d_rec = nullptr;
    G.d_ver = nullptr;
    G.rec_cap = 0;
    if (hipMalloc(reinterpret_cast<void **>(&G.d_rec), k * sizeof(cg_transfer)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&G.d_ver), k * sizeof(cg_verdict)) != hipSuccess)
        return false;
    G.rec_cap = k;
    return true;
}

// A copy of depth slices of height rows of width bytes: row y of slice z
// reads src + z*sslice + y*spitch and writes dst + z*dslice + y*dpitch.  A
// plain copy is one row, a 2D copy one slice.
struct Pitched {
    uint8_t *dst;
    const uint8_t *src;
    size_t width, height, depth, dpitch, spitch, dslice, sslice;
};

// device buffers for k pitched records and their verdicts
bool ensure_slices(uint64_t k)
{
    if (k <= G.slice_cap) return true;
    Guard g;
    (void)hipStreamSynchronize(G.s);
    (void)hipFree(G.d_rec2d);
    (void)hipFree(G.d_ver2d);
    G.d_rec2d = nullptr;
    G.d_ver2d = nullptr;
    G.slice_cap = 0;
    if (hipMalloc(reinterpret_cast<void **>(&G.d_rec2d), k * sizeof(cg_transfer2d)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&G.d_ver2d), k * sizeof(cg_verdict)) != hipSuccess)
        return false;
    G.slice_cap = k;
    return true;
}

// Check a copy before it runs and print the report; false if the copy must
// not be performed (a device side is unallocated or too small).  The whole
// copy is one check (one 2D record per slice); only when it has findings are
// its rows checked one by one, to name the first faulty row.
bool check_pitched(const char *api, const Pitched &p, uint32_t kind)
{
    std::lock_guard<std::mutex> lk(G.mu);
    if (!ensure_ctx()) return true;
    Guard g;
    const uint64_t nrows = (uint64_t)p.height * p.depth;
    if (kind != CG_D2D) {
        // the host side as one region: first row start to last row end
        const bool hsrc = kind == CG_H2D;
        const uint64_t hp = hsrc ? (uint64_t)p.src : (uint64_t)p.dst;
        const uint64_t pitch = hsrc ? p.spitch : p.dpitch, slice = hsrc ? p.sslice : p.dslice;
        const uint64_t span = (p.depth - 1) * slice + (p.height - 1) * pitch + p.width;
        if (!ensure_host_cover(span) || cg_host_register(G.ctx, hp, span ? span : 1, G.zeros, G.ones) != CG_OK)
            return true;
    }
    // no propagation into host shadow (the zeros buffer must stay zero), nor
    // when destination rows overlap (their order would be unspecified)
    const bool rows_apart = (p.height == 1 || p.dpitch >= p.width) &&
                            (p.depth == 1 || p.dslice >= (p.height - 1) * p.dpitch + p.width);
    const uint32_t mode = CG_CHECK | (kind != CG_D2H && rows_apart ? CG_PROPAGATE : 0u);
    auto masked = [&](uint32_t f) { return (!G.device_undef && kind != CG_H2D) ? f & ~CG_SRC_UNDEF : f; };
    bool bad = false;
    if (nrows == 1) {
        if (!ensure_rows(1)) return true;
        cg_transfer r{(uint64_t)p.src, (uint64_t)p.dst, (uint64_t)p.width, kind, 0};
        cg_verdict v;
        if (hipMemcpyAsync(G.d_rec, &r, sizeof r, hipMemcpyHostToDevice, G.s) != hipSuccess ||
            check_transfers(G.ctx, G.d_rec, 1, G.d_ver, mode, G.s) != CG_OK ||
            hipMemcpyAsync(&v, G.d_ver, sizeof v, hipMemcpyDeviceToHost, G.s) != hipSuccess ||
            hipStreamSynchronize(G.s) != hipSuccess) {
            fprintf(stderr, "==xfercheck== check failed: %s\n", cg_last_error(G.ctx));
            return true;
        }
        ++G.copies;
        if (!masked(v.flags)) return true;
        char buf[1024];
        v.flags = masked(v.flags);
        cg_format_verdict(&r, &v, buf, sizeof buf);
        ++G.errors;
        fprintf(stderr, "%s\n at %s(dst=%p, src=%p, %zu bytes, %s)\n", buf, api, (void *)p.dst, (const void *)p.src,
                p.width, kind_name(kind));
        return G.allow_bad || !(v.flags & kRangeFaults);
    }
    if (!ensure_slices(p.depth)) return true;
    std::vector<cg_transfer2d> r2(p.depth);
    for (size_t z = 0; z < p.depth; ++z)
        r2[z] = cg_transfer2d{(uint64_t)(p.src + z * p.sslice), (uint64_t)(p.dst + z * p.dslice), (uint64_t)p.width,
                              (uint64_t)p.height, (uint64_t)p.spitch, (uint64_t)p.dpitch, kind, {0, 0, 0}};
    std::vector<cg_verdict> v2(p.depth);
    if (hipMemcpyAsync(G.d_rec2d, r2.data(), p.depth * sizeof(cg_transfer2d), hipMemcpyHostToDevice, G.s) != hipSuccess ||
        check_transfers_2d(G.ctx, G.d_rec2d, p.depth, G.d_ver2d, mode, G.s) != CG_OK ||
        hipMemcpyAsync(v2.data(), G.d_ver2d, p.depth * sizeof(cg_verdict), hipMemcpyDeviceToHost, G.s) != hipSuccess ||
        hipStreamSynchronize(G.s) != hipSuccess) {
        fprintf(stderr, "==xfercheck== check failed: %s\n", cg_last_error(G.ctx));
        return true;
    }
    ++G.copies;
    for (const cg_verdict &v : v2) bad = bad || masked(v.flags) != 0;
    if (!bad) return true;
    // locate: every row, checked without propagation
    if (!ensure_rows(nrows)) return true;
    std::vector<cg_transfer> r(nrows);
    for (size_t z = 0, k = 0; z < p.depth; ++z)
        for (size_t y = 0; y < p.height; ++y, ++k)
            r[k] = cg_transfer{(uint64_t)(p.src + z * p.sslice + y * p.spitch),
                               (uint64_t)(p.dst + z * p.dslice + y * p.dpitch), (uint64_t)p.width, kind, 0};
    std::vector<cg_verdict> v(nrows);
    if (hipMemcpyAsync(G.d_rec, r.data(), nrows * sizeof(cg_transfer), hipMemcpyHostToDevice, G.s) != hipSuccess ||
        check_transfers(G.ctx, G.d_rec, nrows, G.d_ver, CG_CHECK, G.s) != CG_OK ||
        hipMemcpyAsync(v.data(), G.d_ver, nrows * sizeof(cg_verdict), hipMemcpyDeviceToHost, G.s) != hipSuccess ||
        hipStreamSynchronize(G.s) != hipSuccess) {
        fprintf(stderr, "==xfercheck== check failed: %s\n", cg_last_error(G.ctx));
        return true;
    }
    size_t bad_rows = 0, first = nrows;
    uint32_t all = 0;
    for (size_t k = 0; k < nrows; ++k) {
        v[k].flags = masked(v[k].flags);
        if (v[k].flags) {
            ++bad_rows;
            if (first == nrows) first = k;
            all |= v[k].flags;
        }
    }
    if (!bad_rows) return true;
    char buf[1024];
    cg_format_verdict(&r[first], &v[first], buf, sizeof buf);
    ++G.errors;
    if (p.depth == 1)
        fprintf(stderr, "%s\n in row %zu of %zu (%zu rows with errors) at %s(dst=%p, dpitch=%zu, src=%p, spitch=%zu, "
                        "width=%zu, %s)\n",
                buf, first, nrows, bad_rows, api, (void *)p.dst, p.dpitch, (const void *)p.src, p.spitch, p.width,
                kind_name(kind));
    else
        fprintf(stderr, "%s\n in row %zu of slice %zu (%zu x %zu rows, %zu with errors) at %s(dst=%p, src=%p, "
                        "width=%zu, height=%zu, depth=%zu, %s)\n",
                buf, first % p.height, first / p.height, p.height, p.depth, bad_rows, api, (void *)p.dst,
                (const void *)p.src, p.width, p.height, p.depth, kind_name(kind));
    return G.allow_bad || !(all & kRangeFaults);
}

bool check_copy(const char *api, void *dst, const void *src, size_t n, uint32_t kind)
{
    return check_pitched(api, Pitched{(uint8_t *)dst, (const uint8_t *)src, n, 1, 1, 0, 0, 0, 0}, kind);
}

// the rows of a pitched asynchronous copy join the concurrent-access window
void close_window(bool keep_non_blocking = false);
void window_push(WinCopy c);
void null_stream_point(hipStream_t stream);

void window_rows(const Pitched &p, uint32_t kind, hipStream_t stream)
{
    std::lock_guard<std::mutex> lk(G.mu);
    null_stream_point(stream);
    for (size_t z = 0; z < p.depth; ++z)
        for (size_t y = 0; y < p.height; ++y)
            window_push(WinCopy{cg_transfer{(uint64_t)(p.src + z * p.sslice + y * p.spitch),
                                            (uint64_t)(p.dst + z * p.dslice + y * p.dpitch), (uint64_t)p.width, kind,
                                            0},
                                stream, "hipMemcpy2DAsync/3DAsync row"});
    null_stream_point(stream);
}

// a 3D copy of linear memory as a Pitched copy
Pitched pitched_3d(const hipMemcpy3DParms *q)
{
    const hipPitchedPtr &s = q->srcPtr, &d = q->dstPtr;
    Pitched p;
    p.src = (const uint8_t *)s.ptr + q->srcPos.z * s.pitch * s.ysize + q->srcPos.y * s.pitch + q->srcPos.x;
    p.dst = (uint8_t *)d.ptr + q->dstPos.z * d.pitch * d.ysize + q->dstPos.y * d.pitch + q->dstPos.x;
    p.width = q->extent.width;
    p.height = q->extent.height;
    p.depth = q->extent.depth;
    p.spitch = s.pitch;
    p.dpitch = d.pitch;
    p.sslice = s.pitch * s.ysize;
    p.dslice = d.pitch * d.ysize;
    return p;
}

bool meets(uint64_t a, uint64_t na, uint64_t b, uint64_t nb) { return na && nb && a < b + nb && b < a + na; }

void describe(char *buf, size_t len, const WinCopy &c)
{
    const cg_transfer &r = c.r;
    if (c.fill)
        snprintf(buf, len, "%s(dst=%p, %" PRIu64 " bytes) on stream %p", c.api, (void *)r.dst, r.n, (void *)c.stream);
    else
        snprintf(buf, len, "%s(dst=%p, src=%p, %" PRIu64 " bytes, %s) on stream %p", c.api, (void *)r.dst,
                 (void *)r.src, r.n, kind_name(r.kind), (void *)c.stream);
}

bool non_blocking(hipStream_t s)
{
    unsigned int f = 0;
    return s != nullptr && hipStreamGetFlags(s, &f) == hipSuccess && (f & hipStreamNonBlocking);
}

void join_window(const std::vector<WinCopy> &w);

// Join the window's copies and report each conflicting pair once; the caller
// holds G.mu.  The window is emptied, or, at work on the null stream
// (keep_non_blocking), keeps the copies of non-blocking streams, which that
// work does not order.
void close_window(bool keep_non_blocking)
{
    std::vector<WinCopy> w;
    w.swap(G.win);
    join_window(w);
    if (keep_non_blocking)
        for (const WinCopy &c : w)
            if (non_blocking(c.stream)) G.win.push_back(c);
    if (G.win.empty()) G.reported.clear();
}

// a copy joins the window
void window_push(WinCopy c)
{
    c.seq = G.win_seq++;
    G.win.push_back(c);
    if (G.win.size() >= kWindowMax) close_window();
}

// asynchronous work on `stream`: on the null stream it is ordered after the
// window's copies on blocking streams, and later work on them after it
void null_stream_point(hipStream_t stream)
{
    if (stream == nullptr && !G.win.empty()) close_window(true);
}

void join_window(const std::vector<WinCopy> &w)
{
    if (w.size() < 2 || !G.ctx) return;
    std::map<hipStream_t, uint32_t> ids;
    std::vector<uint32_t> sid(w.size());
    std::vector<cg_transfer> r(w.size());
    for (size_t i = 0; i < w.size(); ++i) {
        sid[i] = ids.emplace(w[i].stream, (uint32_t)ids.size()).first->second;
        r[i] = w[i].r;
    }
    if (ids.size() < 2) return;   // one stream: all ordered
    Guard g;
    const uint64_t n = w.size();
    if (n > G.win_cap) {
        (void)hipStreamSynchronize(G.s);
        (void)hipFree(G.d_wrec);
        (void)hipFree(G.d_wsid);
        (void)hipFree(G.d_wres);
        G.d_wrec = nullptr;
        G.d_wsid = nullptr;
        G.d_wres = nullptr;
        G.win_cap = 0;
        uint64_t cap = 64;
        while (cap < n) cap <<= 1;
        if (hipMalloc(reinterpret_cast<void **>(&G.d_wrec), cap * sizeof(cg_transfer)) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&G.d_wsid), cap * sizeof(uint32_t)) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&G.d_wres), cap * sizeof(cg_race)) != hipSuccess) {
            fprintf(stderr, "==xfercheck== concurrent-access check skipped: out of device memory\n");
            return;
        }
        G.win_cap = cap;
    }
    std::vector<cg_race> res(n);
    if (hipMemcpyAsync(G.d_wrec, r.data(), n * sizeof(cg_transfer), hipMemcpyHostToDevice, G.s) != hipSuccess ||
        hipMemcpyAsync(G.d_wsid, sid.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, G.s) != hipSuccess ||
        check_concurrent(G.ctx, G.d_wrec, G.d_wsid, nullptr, n, G.d_wres, G.s) != CG_OK ||
        hipMemcpyAsync(res.data(), G.d_wres, n * sizeof(cg_race), hipMemcpyDeviceToHost, G.s) != hipSuccess ||
        hipStreamSynchronize(G.s) != hipSuccess) {
        fprintf(stderr, "==xfercheck== concurrent-access check failed: %s\n", cg_last_error(G.ctx));
        return;
    }
    for (uint64_t a = 0; a < n; ++a) {
        if (!(res[a].flags & (CG_RACE_SRC | CG_RACE_DST)) || res[a].partner >= n) continue;
        const uint64_t b = res[a].partner;
        const uint64_t qa = w[a].seq, qb = w[b].seq;
        if (!G.reported.insert({std::min(qa, qb), std::max(qa, qb)}).second) continue;
        const cg_transfer &x = r[a], &y = r[b];
        // what the first copy does to the shared bytes, and what the second does
        const bool ww = meets(x.dst, x.n, y.dst, y.n), wr = meets(x.dst, x.n, y.src, y.n);
        const char *va = (ww || wr) ? "writes" : "reads", *vb = (ww || !wr) ? "writes" : "reads";
        char da[256], db[256];
        describe(da, sizeof da, w[a]);
        describe(db, sizeof db, w[b]);
        fprintf(stderr,
                "Error: Concurrent copies access the same bytes without synchronisation.\n %s\n %s bytes that\n %s\n "
                "%s.\n",
                da, va, db, vb);
        ++G.races;
        ++G.errors;
    }
}

// a synchronising call: the copies issued so far are ordered before what follows
void sync_point()
{
    std::lock_guard<std::mutex> lk(G.mu);
    if (!G.win.empty()) close_window();
}

std::string trim(const std::string &x)
{
    const size_t a = x.find_first_not_of(' '), b = x.find_last_not_of(' ');
    return a == std::string::npos ? std::string() : x.substr(a, b - a + 1);
}

// Parameter list of a kernel from its mangled name: demangle, take the
// parenthesised list that ends the name, split it at top-level commas.  A
// parameter is a raw pointer when its type ends in '*' once qualifiers of the
// pointer itself are dropped.
KernelSig parse_signature(const char *mangled)
{
    KernelSig k;
    k.name = mangled ? mangled : "?";
    if (!mangled) return k;
    int st = 0;
    char *d = abi::__cxa_demangle(mangled, nullptr, nullptr, &st);
    if (st != 0 || !d) {
        free(d);
        return k;   // not a C++ name: no parameter types
    }
    const std::string s(d);
    free(d);
    k.name = s;
    if (s.empty() || s.back() != ')') return k;
    int depth = 0;
    size_t open = std::string::npos;
    for (size_t i = s.size(); i-- > 0;) {
        if (s[i] == ')') ++depth;
        else if (s[i] == '(' && --depth == 0) {
            open = i;
            break;
        }
    }
    if (open == std::string::npos) return k;
    const std::string list = s.substr(open + 1, s.size() - open - 2);
    std::string cur;
    int dp = 0;
    for (char ch : list) {
        if (ch == '(' || ch == '<' || ch == '[') ++dp;
        if (ch == ')' || ch == '>' || ch == ']') --dp;
        if (ch == ',' && dp == 0) {
            k.params.push_back(trim(cur));
            cur.clear();
        } else {
            cur += ch;
        }
    }
    if (!trim(cur).empty()) k.params.push_back(trim(cur));
    if (k.params.size() == 1 && k.params[0] == "void") k.params.clear();
    for (const std::string &p : k.params) {
        std::string t = p;
        for (const char *q : {" const", " volatile", " restrict", " __restrict"}) {
            const size_t n = strlen(q);
            while (t.size() > n && t.compare(t.size() - n, n, q) == 0) t = trim(t.substr(0, t.size() - n));
        }
        k.is_ptr.push_back(!t.empty() && t.back() == '*');
    }
    k.known = true;
    return k;
}

bool pinned_host(uint64_t p)
{
    hipPointerAttribute_t a;
    const bool host = hipPointerGetAttributes(&a, (const void *)p) == hipSuccess && a.type == hipMemoryTypeHost;
    (void)hipGetLastError();
    return host;
}

// Check the pointer arguments of a launch; false if it must not run.
bool check_launch(const char *api, const void *fn, void **args, hipStream_t stream)
{
    std::lock_guard<std::mutex> lk(G.mu);
    if (!ensure_ctx()) return true;
    Guard g;
    auto it = G.sigs.find(fn);
    if (it == G.sigs.end()) it = G.sigs.emplace(fn, parse_signature(hipKernelNameRefByPtr(fn, stream))).first;
    const KernelSig &k = it->second;
    if (!k.known) return true;
    std::vector<uint64_t> ptrs;
    std::vector<size_t> which;
    for (size_t i = 0; i < k.is_ptr.size(); ++i) {
        if (!k.is_ptr[i]) continue;
        uint64_t p = 0;
        memcpy(&p, args[i], sizeof p);
        if (p == 0 || pinned_host(p)) continue;
        ptrs.push_back(p);
        which.push_back(i);
    }
    ++G.launches;
    if (ptrs.empty()) return true;
    const uint64_t n = ptrs.size();
    if (n > G.ptr_cap) {
        (void)hipStreamSynchronize(G.s);
        (void)hipFree(G.d_ptrs);
        (void)hipFree(G.d_pres);
        G.d_ptrs = nullptr;
        G.d_pres = nullptr;
        G.ptr_cap = 0;
        const uint64_t cap = n < 64 ? 64 : n;
        if (hipMalloc(reinterpret_cast<void **>(&G.d_ptrs), cap * sizeof(uint64_t)) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&G.d_pres), cap * sizeof(cg_ptr_check)) != hipSuccess)
            return true;
        G.ptr_cap = cap;
    }
    std::vector<cg_ptr_check> res(n);
    if (hipMemcpyAsync(G.d_ptrs, ptrs.data(), n * sizeof(uint64_t), hipMemcpyHostToDevice, G.s) != hipSuccess ||
        check_pointers(G.ctx, G.d_ptrs, n, G.d_pres, G.s) != CG_OK ||
        hipMemcpyAsync(res.data(), G.d_pres, n * sizeof(cg_ptr_check), hipMemcpyDeviceToHost, G.s) != hipSuccess ||
        hipStreamSynchronize(G.s) != hipSuccess) {
        fprintf(stderr, "==xfercheck== kernel argument check failed: %s\n", cg_last_error(G.ctx));
        return true;
    }
    bool ok = true;
    for (uint64_t j = 0; j < n; ++j) {
        if (!(res[j].flags & CG_PTR_UNALLOC)) continue;
        ok = false;
        ++G.errors;
        fprintf(stderr,
                "Error: Kernel argument %zu (%s) points into no allocated device region.\n"
                " %p is neither inside nor one past the end of a live allocation (freed or never allocated).\n"
                " at %s(%s)\n",
                which[j], k.params[which[j]].c_str(), (void *)ptrs[j], api, k.name.c_str());
    }
    return ok || G.allow_bad;
}

uint32_t direction(void *dst, const void *src, hipMemcpyKind k)
{
    switch (k) {
    case hipMemcpyHostToDevice: return CG_H2D;
    case hipMemcpyDeviceToHost: return CG_D2H;
    case hipMemcpyDeviceToDevice: return CG_D2D;
    case hipMemcpyDefault: {
        Guard g;
        hipPointerAttribute_t a, b;
        const bool dd = hipPointerGetAttributes(&a, dst) == hipSuccess && a.type == hipMemoryTypeDevice;
        const bool sd = hipPointerGetAttributes(&b, src) == hipSuccess && b.type == hipMemoryTypeDevice;
        (void)hipGetLastError();
        if (sd && dd) return CG_D2D;
        if (dd) return CG_H2D;
        if (sd) return CG_D2H;
        return 99;
    }
    default: return 99;   // host->host: not a device transfer
    }
}

void track_alloc(const char *api, void *p, size_t size)
{
    std::lock_guard<std::mutex> lk(G.mu);
    if (!ensure_ctx()) return;
    Guard g;
    const int rc = shadow_alloc(G.ctx, (uint64_t)p, size);
    if (rc != CG_OK) fprintf(stderr, "==xfercheck== %s(%zu) at %p not tracked: %s\n", api, size, p, cg_strerror(rc));
}

void track_free(const char *api, void *p)
{
    std::lock_guard<std::mutex> lk(G.mu);
    if (!ensure_ctx()) return;
    Guard g;
    if (shadow_free(G.ctx, (uint64_t)p) != CG_OK) {
        ++G.errors;
        fprintf(stderr, "Error: %s of %p, which is not the start of an allocated device region.\n", api, p);
    }
}

// A fill of n bytes at dst: its bytes become defined (shadow_set); a fill
// outside the allocations is reported and refused.  An asynchronous fill
// also joins the concurrent-access window as a write on its stream.
bool track_fill(const char *api, void *dst, size_t n, bool async, hipStream_t stream)
{
    if (inside || !n) return true;
    std::lock_guard<std::mutex> lk(G.mu);
    if (!ensure_ctx()) return true;
    Guard g;
    if (shadow_set(G.ctx, (uint64_t)dst, n, 0) != CG_OK) {
        ++G.errors;
        fprintf(stderr, "Error: %s of %zu bytes at %p leaves allocated device memory.\n", api, n, dst);
        if (!G.allow_bad) return false;
    }
    if (async) {
        null_stream_point(stream);
        window_push(WinCopy{cg_transfer{(uint64_t)dst, (uint64_t)dst, (uint64_t)n, CG_D2D, 0}, stream, api, true});
        null_stream_point(stream);
    }
    return true;
}

// an asynchronous copy: checked when issued, then part of the window
bool async_copy(const char *api, void *dst, const void *src, size_t n, uint32_t d, hipStream_t stream)
{
    if (inside || !n || d > CG_D2D) return true;
    if (!check_copy(api, dst, src, n, d)) return false;
    std::lock_guard<std::mutex> lk(G.mu);
    null_stream_point(stream);
    window_push(WinCopy{cg_transfer{(uint64_t)src, (uint64_t)dst, (uint64_t)n, d, 0}, stream, api});
    null_stream_point(stream);
    return true;
}

}  // namespace

extern "C" {

hipError_t hipMalloc(void **ptr, size_t size)
{
    static malloc_t f = real<malloc_t>("hipMalloc");
    const hipError_t e = f(ptr, size);
    if (!inside && e == hipSuccess && ptr && *ptr && size) track_alloc("hipMalloc", *ptr, size);
    return e;
}

hipError_t hipFree(void *ptr)
{
    static free_t f = real<free_t>("hipFree");
    if (!inside) sync_point();
    if (!inside && ptr) track_free("hipFree", ptr);
    return f(ptr);
}

hipError_t hipMemset(void *dst, int value, size_t n)
{
    static memset_t f = real<memset_t>("hipMemset");
    if (!inside) sync_point();
    if (!track_fill("hipMemset", dst, n, false, nullptr)) return refuse();
    return f(dst, value, n);
}

hipError_t hipMemsetAsync(void *dst, int value, size_t n, hipStream_t stream)
{
    static memset_async_t f = real<memset_async_t>("hipMemsetAsync");
    if (!track_fill("hipMemsetAsync", dst, n, true, stream)) return refuse();
    return f(dst, value, n, stream);
}

hipError_t hipMemsetD8(hipDeviceptr_t dst, unsigned char value, size_t count)
{
    static memset_d8_t f = real<memset_d8_t>("hipMemsetD8");
    if (!inside) sync_point();
    if (!track_fill("hipMemsetD8", dst, count, false, nullptr)) return refuse();
    return f(dst, value, count);
}

hipError_t hipMemsetD8Async(hipDeviceptr_t dst, unsigned char value, size_t count, hipStream_t stream)
{
    static memset_d8_async_t f = real<memset_d8_async_t>("hipMemsetD8Async");
    if (!track_fill("hipMemsetD8Async", dst, count, true, stream)) return refuse();
    return f(dst, value, count, stream);
}

hipError_t hipMemsetD16(hipDeviceptr_t dst, unsigned short value, size_t count)
{
    static memset_d16_t f = real<memset_d16_t>("hipMemsetD16");
    if (!inside) sync_point();
    if (!track_fill("hipMemsetD16", dst, 2 * count, false, nullptr)) return refuse();
    return f(dst, value, count);
}

hipError_t hipMemsetD16Async(hipDeviceptr_t dst, unsigned short value, size_t count, hipStream_t stream)
{
    static memset_d16_async_t f = real<memset_d16_async_t>("hipMemsetD16Async");
    if (!track_fill("hipMemsetD16Async", dst, 2 * count, true, stream)) return refuse();
    return f(dst, value, count, stream);
}

hipError_t hipMemsetD32(hipDeviceptr_t dst, int value, size_t count)
{
    static memset_d32_t f = real<memset_d32_t>("hipMemsetD32");
    if (!inside) sync_point();
    if (!track_fill("hipMemsetD32", dst, 4 * count, false, nullptr)) return refuse();
    return f(dst, value, count);
}

hipError_t hipMemsetD32Async(hipDeviceptr_t dst, int value, size_t count, hipStream_t stream)
{
    static memset_d32_async_t f = real<memset_d32_async_t>("hipMemsetD32Async");
    if (!track_fill("hipMemsetD32Async", dst, 4 * count, true, stream)) return refuse();
    return f(dst, value, count, stream);
}

hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind kind)
{
    static memcpy_t f = real<memcpy_t>("hipMemcpy");
    if (!inside) sync_point();
    if (!inside && n) {
        const uint32_t d = direction(dst, src, kind);
        if (d <= CG_D2D && !check_copy("hipMemcpy", dst, src, n, d)) return refuse();
    }
    return f(dst, src, n, kind);
}

hipError_t hipMemcpyHtoD(hipDeviceptr_t dst, const void *src, size_t n)
{
    static htod_t f = real<htod_t>("hipMemcpyHtoD");
    if (!inside) sync_point();
    if (!inside && n && !check_copy("hipMemcpyHtoD", dst, src, n, CG_H2D)) return refuse();
    return f(dst, src, n);
}

hipError_t hipMemcpyDtoH(void *dst, hipDeviceptr_t src, size_t n)
{
    static dtoh_t f = real<dtoh_t>("hipMemcpyDtoH");
    if (!inside) sync_point();
    if (!inside && n && !check_copy("hipMemcpyDtoH", dst, src, n, CG_D2H)) return refuse();
    return f(dst, src, n);
}

hipError_t hipMemcpyDtoD(hipDeviceptr_t dst, hipDeviceptr_t src, size_t n)
{
    static dtod_t f = real<dtod_t>("hipMemcpyDtoD");
    if (!inside) sync_point();
    if (!inside && n && !check_copy("hipMemcpyDtoD", dst, src, n, CG_D2D)) return refuse();
    return f(dst, src, n);
}

hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind kind, hipStream_t stream)
{
    static memcpy_async_t f = real<memcpy_async_t>("hipMemcpyAsync");
    if (!inside && n && !async_copy("hipMemcpyAsync", dst, src, n, direction(dst, src, kind), stream))
        return refuse();
    return f(dst, src, n, kind, stream);
}

hipError_t hipMemcpyHtoDAsync(hipDeviceptr_t dst, const void *src, size_t n, hipStream_t stream)
{
    static htod_async_t f = real<htod_async_t>("hipMemcpyHtoDAsync");
    if (!async_copy("hipMemcpyHtoDAsync", dst, src, n, CG_H2D, stream)) return refuse();
    return f(dst, src, n, stream);
}

hipError_t hipMemcpyDtoHAsync(void *dst, hipDeviceptr_t src, size_t n, hipStream_t stream)
{
    static dtoh_async_t f = real<dtoh_async_t>("hipMemcpyDtoHAsync");
    if (!async_copy("hipMemcpyDtoHAsync", dst, src, n, CG_D2H, stream)) return refuse();
    return f(dst, src, n, stream);
}

hipError_t hipMemcpyDtoDAsync(hipDeviceptr_t dst, hipDeviceptr_t src, size_t n, hipStream_t stream)
{
    static dtod_async_t f = real<dtod_async_t>("hipMemcpyDtoDAsync");
    if (!async_copy("hipMemcpyDtoDAsync", dst, src, n, CG_D2D, stream)) return refuse();
    return f(dst, src, n, stream);
}

// a copy the host waits for: ordered after what came before, as hipMemcpy
hipError_t hipMemcpyWithStream(void *dst, const void *src, size_t n, hipMemcpyKind kind, hipStream_t stream)
{
    static memcpy_async_t f = real<memcpy_async_t>("hipMemcpyWithStream");
    if (!inside) sync_point();
    if (!inside && n) {
        const uint32_t d = direction(dst, src, kind);
        if (d <= CG_D2D && !check_copy("hipMemcpyWithStream", dst, src, n, d)) return refuse();
    }
    return f(dst, src, n, kind, stream);
}

hipError_t hipLaunchKernel(const void *fn, dim3 grid, dim3 block, void **args, size_t shmem, hipStream_t stream)
{
    static launch_t f = real<launch_t>("hipLaunchKernel");
    if (!inside && args && G.kernel_args && !check_launch("hipLaunchKernel", fn, args, stream))
        return refuse();
    if (!inside && stream == nullptr) {
        // a kernel on the null stream orders the blocking streams' copies around it
        std::lock_guard<std::mutex> lk(G.mu);
        null_stream_point(stream);
    }
    return f(fn, grid, block, args, shmem, stream);
}

hipError_t hipMallocManaged(void **ptr, size_t size, unsigned int flags)
{
    static malloc_flags_t f = real<malloc_flags_t>("hipMallocManaged");
    const hipError_t e = f(ptr, size, flags);
    if (!inside && e == hipSuccess && ptr && *ptr && size) track_alloc("hipMallocManaged", *ptr, size);
    return e;
}

hipError_t hipExtMallocWithFlags(void **ptr, size_t size, unsigned int flags)
{
    static malloc_flags_t f = real<malloc_flags_t>("hipExtMallocWithFlags");
    const hipError_t e = f(ptr, size, flags);
    if (!inside && e == hipSuccess && ptr && *ptr && size) track_alloc("hipExtMallocWithFlags", *ptr, size);
    return e;
}

hipError_t hipMallocAsync(void **ptr, size_t size, hipStream_t stream)
{
    static malloc_async_t f = real<malloc_async_t>("hipMallocAsync");
    const hipError_t e = f(ptr, size, stream);
    if (!inside && e == hipSuccess && ptr && *ptr && size) track_alloc("hipMallocAsync", *ptr, size);
    return e;
}

hipError_t hipFreeAsync(void *ptr, hipStream_t stream)
{
    static free_async_t f = real<free_async_t>("hipFreeAsync");
    if (!inside && ptr) track_free("hipFreeAsync", ptr);
    return f(ptr, stream);
}

hipError_t hipGetLastError(void)
{
    static lasterr_t f = real<lasterr_t>("hipGetLastError");
    const hipError_t e = f();
    if (inside || refused == hipSuccess) return e;
    const hipError_t r = refused;
    refused = hipSuccess;
    return r;
}

hipError_t hipPeekAtLastError(void)
{
    static lasterr_t f = real<lasterr_t>("hipPeekAtLastError");
    const hipError_t e = f();
    return (inside || refused == hipSuccess) ? e : refused;
}

hipError_t hipDeviceSynchronize(void)
{
    static devsync_t f = real<devsync_t>("hipDeviceSynchronize");
    if (!inside) sync_point();
    return f();
}

hipError_t hipStreamSynchronize(hipStream_t stream)
{
    static streamsync_t f = real<streamsync_t>("hipStreamSynchronize");
    if (!inside) sync_point();
    return f(stream);
}

hipError_t hipEventSynchronize(hipEvent_t event)
{
    static eventsync_t f = real<eventsync_t>("hipEventSynchronize");
    if (!inside) sync_point();
    return f(event);
}

hipError_t hipStreamWaitEvent(hipStream_t stream, hipEvent_t event, unsigned int flags)
{
    static waitevent_t f = real<waitevent_t>("hipStreamWaitEvent");
    if (!inside) sync_point();
    return f(stream, event, flags);
}

hipError_t hipMemcpy2D(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width, size_t height,
                       hipMemcpyKind kind)
{
    static memcpy2d_t f = real<memcpy2d_t>("hipMemcpy2D");
    if (!inside) sync_point();
    if (!inside && width && height) {
        const uint32_t d = direction(dst, src, kind);
        if (d <= CG_D2D &&
            !check_pitched("hipMemcpy2D", Pitched{(uint8_t *)dst, (const uint8_t *)src, width, height, 1, dpitch, spitch,
                                                  0, 0},
                           d))
            return refuse();
    }
    return f(dst, dpitch, src, spitch, width, height, kind);
}

hipError_t hipMemcpy2DAsync(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width, size_t height,
                            hipMemcpyKind kind, hipStream_t stream)
{
    static memcpy2d_async_t f = real<memcpy2d_async_t>("hipMemcpy2DAsync");
    if (!inside && width && height) {
        const uint32_t d = direction(dst, src, kind);
        const Pitched p{(uint8_t *)dst, (const uint8_t *)src, width, height, 1, dpitch, spitch, 0, 0};
        if (d <= CG_D2D) {
            if (!check_pitched("hipMemcpy2DAsync", p, d)) return refuse();
            window_rows(p, d, stream);
        }
    }
    return f(dst, dpitch, src, spitch, width, height, kind, stream);
}

hipError_t hipMemcpy3D(const hipMemcpy3DParms *q)
{
    static memcpy3d_t f = real<memcpy3d_t>("hipMemcpy3D");
    if (!inside) sync_point();
    if (!inside && q && !q->srcArray && !q->dstArray && q->extent.width && q->extent.height && q->extent.depth) {
        const Pitched p = pitched_3d(q);
        const uint32_t d = direction(p.dst, p.src, q->kind);
        if (d <= CG_D2D && !check_pitched("hipMemcpy3D", p, d)) return refuse();
    }
    return f(q);
}

hipError_t hipMemcpy3DAsync(const hipMemcpy3DParms *q, hipStream_t stream)
{
    static memcpy3d_async_t f = real<memcpy3d_async_t>("hipMemcpy3DAsync");
    if (!inside && q && !q->srcArray && !q->dstArray && q->extent.width && q->extent.height && q->extent.depth) {
        const Pitched p = pitched_3d(q);
        const uint32_t d = direction(p.dst, p.src, q->kind);
        if (d <= CG_D2D) {
            if (!check_pitched("hipMemcpy3DAsync", p, d)) return refuse();
            window_rows(p, d, stream);
        }
    }
    return f(q, stream);
}

hipError_t hipMallocPitch(void **ptr, size_t *pitch, size_t width, size_t height)
{
    static malloc_pitch_t f = real<malloc_pitch_t>("hipMallocPitch");
    hipError_t e;
    {
        Guard g;   // an allocation made inside is tracked here, once
        e = f(ptr, pitch, width, height);
    }
    if (!inside && e == hipSuccess && ptr && *ptr && pitch && *pitch && height)
        track_alloc("hipMallocPitch", *ptr, *pitch * height);
    return e;
}

hipError_t hipMalloc3D(hipPitchedPtr *pp, hipExtent extent)
{
    static malloc3d_t f = real<malloc3d_t>("hipMalloc3D");
    const bool outer = !inside;
    hipError_t e;
    {
        Guard g;
        e = f(pp, extent);
    }
    if (outer && e == hipSuccess && pp && pp->ptr && pp->pitch && extent.height && extent.depth)
        track_alloc("hipMalloc3D", pp->ptr, pp->pitch * extent.height * extent.depth);
    return e;
}

}  // extern "C"
