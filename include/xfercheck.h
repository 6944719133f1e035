/*
 * xfercheck.h -- C ABI of the MI355X (gfx950) transfer checker.
 *
 * Memcheck-style validation of host->device, device->host and device->device
 * copies, after Baumann & Gracia, "Cudagrind: A Valgrind Extension for CUDA"
 * (arXiv 1310.0901):
 *   - every copy is cross-checked against the context's list of live device
 *     allocations {pointer, size} (Sec. 2 and the Fig. 2 caption);
 *   - host source data must be addressable and defined, with bitwise shadow
 *     precision (Sec. 1.1, Sec. 1.2, the error list of Sec. 2);
 *   - the report names the bytes the copy needs and the bytes the allocation
 *     actually offers (Sec. 4.5, Listing 6);
 *   - definedness follows the data through all three copy directions (Sec. 5).
 *
 * Shadow conventions.  One V byte per data byte: 0 = defined, any set bit =
 * undefined (a byte counts as undefined when its V byte is non-zero; the bits
 * themselves are carried unchanged by propagation).  Host addressability is
 * one A bit per byte, 1 = addressable; the byte at region offset x is bit
 * (x & 63) of the little-endian 64-bit word x >> 6.  Bits of the last word
 * beyond the region are ignored.
 *
 * Threading and ordering.  A context is not thread-safe: call it from one
 * host thread.  Device work is stream ordered: check_transfers and
 * propagate_shadow run on the caller's stream; shadow_* calls run on the
 * context's own stream.  The library orders the two: a check sees every
 * shadow_* call made before it, and a shadow_* call waits for every check
 * issued before it.  Results in device memory are valid once the caller's
 * stream has been synchronised.
 *
 * Errors.  Every function returns an int status: CG_OK (0) or a negative
 * CG_E* code; cg_last_error() gives the detailed text of the last failure on
 * a context.  Faults found in the transfers themselves are never call
 * errors: they are reported in the verdicts.
 */
#ifndef XFERCHECK_H
#define XFERCHECK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define CG_OK          0
#define CG_EINVAL     -1   /* bad argument (null pointer, bad mode, misaligned buffer, size 0) */
#define CG_ENOMEM     -2   /* shadow pool or device memory exhausted */
#define CG_EOVERLAP   -3   /* shadow_alloc range intersects a live allocation */
#define CG_ENOTFOUND  -4   /* shadow_free / shadow_set / shadow_ptr: not a live allocation */
#define CG_ECONFLICT  -5   /* CG_DEBUG_CONFLICTS: a destination overlaps another record's shadow */
#define CG_ECAPACITY  -6   /* more live allocations than max_allocs */
#define CG_EHIP       -7   /* a HIP runtime call failed (text in cg_last_error) */
#define CG_ESTATE     -8   /* call not valid in the current state (e.g. no host region) */

/* ---- record kinds (the three copy directions of Sec. 5) ----------------- */
#define CG_H2D 0u
#define CG_D2H 1u
#define CG_D2D 2u

/* ---- verdict flags ------------------------------------------------------ */
#define CG_SRC_UNADDR   0x001u  /* a host source byte is outside the region or has A = 0 */
#define CG_SRC_UNDEF    0x002u  /* at least one valid source byte has V != 0 */
#define CG_SRC_UNALLOC  0x004u  /* device source pointer is in no live allocation */
#define CG_SRC_OVERRUN  0x008u  /* n exceeds the bytes left in the source allocation */
#define CG_DST_UNADDR   0x010u  /* a host destination byte is outside the region or has A = 0 */
#define CG_DST_UNALLOC  0x020u  /* device destination pointer is in no live allocation */
#define CG_DST_OVERRUN  0x040u  /* n exceeds the bytes left in the destination allocation */
#define CG_OVERLAP      0x080u  /* device->device copy whose ranges intersect (not propagated) */
#define CG_BAD_KIND     0x100u  /* kind is not 0, 1 or 2 */
#define CG_ROWS_LIMIT   0x200u  /* pitched 2D copy: not every row was checked (see check_transfers_2d) */
#define CG_NONE 0xFFFFFFFFFFFFFFFFull /* first_bad when the transfer is clean */

/* ---- modes of check_transfers ------------------------------------------ */
#define CG_CHECK           0x01u  /* write verdicts */
#define CG_PROPAGATE       0x02u  /* copy V bytes into the destination shadow */
#define CG_PLAIN           0x04u  /* one kernel launch per transfer (baseline path) */
#define CG_DEBUG_CONFLICTS 0x08u  /* host-side verification of the no-conflict rule (synchronous) */
#define CG_EAGER           0x10u  /* batched path without graph capture */
#define CG_KEEP_ORDER      0x20u  /* work a large batch in the given order (no source-block segments) */

/*
 * One transfer record, 32 bytes, in device memory (the parameters of a
 * copy call: destination, source, byte count and direction; Sec. 2, Listing 2).
 * src / dst are the application's addresses: host addresses for the host
 * side, device addresses for the device side.  `reserved` is ignored.
 */
typedef struct cg_transfer {
    uint64_t src, dst, n;
    uint32_t kind, reserved;
} cg_transfer;

/*
 * One verdict, 32 bytes, in device memory.
 *   flags       OR of CG_* flags above.
 *   first_bad   smallest byte index i in [0, n) that is bad: a source byte
 *               that is not valid (host: outside the region or A = 0;
 *               device: beyond the allocation), a destination byte that is
 *               not valid, or a valid source byte with V != 0; CG_NONE if
 *               none.  An unallocated device side makes it 0; an overrun
 *               makes it at most `avail`.
 *   undef_bytes number of valid source bytes with V != 0.
 *   avail       bytes from the device pointer to the end of its allocation
 *               (0 if unallocated), minimum over the device sides; this is
 *               the "found" count of the report in Sec. 4.5.
 * BAD_KIND gives {CG_BAD_KIND, CG_NONE, 0, 0}; n == 0 gives {0, CG_NONE, 0, 0}.
 */
typedef struct cg_verdict {
    uint32_t flags, reserved;
    uint64_t first_bad, undef_bytes, avail;
} cg_verdict;

typedef struct cg_ctx cg_ctx;   /* one per device context (Fig. 2 caption) */

/*
 * Create a context on HIP device `hip_device`.  The library allocates a
 * device shadow pool of `shadow_pool_bytes` (V bytes of all live device
 * allocations are sub-allocated from it, 256-byte aligned) and a table for
 * up to `max_allocs` live allocations.  *out receives the context.
 * Errors: CG_EINVAL (null out, zero sizes), CG_EHIP / CG_ENOMEM.
 */
int cg_create(cg_ctx **out, int hip_device, uint64_t shadow_pool_bytes, uint64_t max_allocs);

/* Destroy a context after synchronising its work; frees pool and tables. */
int cg_destroy(cg_ctx *ctx);

/*
 * Register the host region [host_base, host_base + len) whose shadow lives
 * in caller-owned device memory (Sec. 1.1: the host side's A and V shadow):
 *   v_dev       V bytes, 16-byte aligned, at least round_up(len, 16) bytes
 *               (bytes past len are never used but may be read);
 *   a_bits_dev  A bitmap, 8-byte aligned, ceil(len / 64) words.
 * The caller keeps both alive and unchanged while checks that use them are
 * in flight.  Host bytes outside the region are unaddressable.  Replaces any
 * earlier registration.  Errors: CG_EINVAL (null/misaligned pointer, len 0).
 */
int cg_host_register(cg_ctx *ctx, uint64_t host_base, uint64_t len, uint8_t *v_dev,
                     uint64_t *a_bits_dev);

/*
 * Record a device allocation [dev_addr, dev_addr + size), as the wrapper of
 * an allocation call does (Sec. 1.2, Sec. 2).  Its shadow is set to 0xFF:
 * nothing is defined yet.  Errors: CG_EINVAL (size 0 or address wrap),
 * CG_EOVERLAP (intersects a live allocation), CG_ECAPACITY, CG_ENOMEM
 * (shadow pool full).
 */
int shadow_alloc(cg_ctx *ctx, uint64_t dev_addr, uint64_t size);

/*
 * Forget the live allocation whose base is dev_addr (the free wrapper).
 * Later copies that touch it report UNALLOC.  Errors: CG_ENOTFOUND when
 * dev_addr is not the base of a live allocation (double or wild free).
 */
int shadow_free(cg_ctx *ctx, uint64_t dev_addr);

/* k allocations / frees at once; host arrays.  Stops at the first error and
 * returns it; the calls before it have taken effect. */
int shadow_alloc_batch(cg_ctx *ctx, const uint64_t *addr, const uint64_t *size, uint64_t k);
int shadow_free_batch(cg_ctx *ctx, const uint64_t *addr, uint64_t k);

/*
 * Set the V bytes of [dev_addr, dev_addr + n) to v: a memset, or a kernel
 * having written the bytes (kernels themselves are not instrumented; Sec. 5.1).
 * The range must lie inside one live allocation.  Errors: CG_ENOTFOUND,
 * CG_EINVAL (range leaves the allocation).
 */
int shadow_set(cg_ctx *ctx, uint64_t dev_addr, uint64_t n, uint8_t v);

/* k shadow_set calls at once (host arrays), issued as one kernel launch. */
int shadow_set_batch(cg_ctx *ctx, const uint64_t *addr, const uint64_t *n, const uint8_t *v,
                     uint64_t k);

/*
 * Device pointer of the V byte that shadows dev_addr (any address inside a
 * live allocation).  The pointer stays valid until the allocation is freed.
 * Errors: CG_ENOTFOUND.
 */
int shadow_ptr(cg_ctx *ctx, uint64_t dev_addr, uint8_t **v_dev);

/*
 * Check `count` records at recs_dev (device memory) and write one verdict
 * per record to out_dev (device memory, 32 bytes each), on `hip_stream`
 * (a hipStream_t; NULL = the null stream).
 *   mode: CG_CHECK and/or CG_PROPAGATE, optionally with CG_PLAIN (one launch
 *   per record), CG_EAGER (no graph capture), CG_DEBUG_CONFLICTS or
 *   CG_KEEP_ORDER.  A batched check of 16,384 to 2^27 records is worked as
 *   source-block segments: each record's bytes are cut at blocks of source
 *   memory (a power of two of at least 1 MiB) and the pieces are worked in
 *   block order, so that copies reading the same bytes run close together.
 *   Verdicts are the same and are written at the records' own positions
 *   either way; CG_KEEP_ORDER works the batch in the given order.
 *   A check without propagation of more than 256 records (not CG_PLAIN or
 *   CG_KEEP_ORDER) that reads its shadow spaces heavily (at least 4 bytes of
 *   the host region, or of the shadow pool, per byte of it) reads the 64 KiB
 *   steps of each such space that its records read, once, into an index of
 *   their faulty 16-byte chunks and answers its records from it, with the
 *   same verdicts (the first such call on a stream allocates the index
 *   space: about 180 MB plus 9 bytes per 64 KiB of the pool).  A host region
 *   above 64 GiB is not indexed.
 * With CG_PROPAGATE every valid destination byte receives the source's V
 * byte, or 0xFF where the source byte is not valid; overlapping D2D records
 * are not propagated.  All records read the shadow as it was before the
 * call.  Precondition for CG_PROPAGATE: no record's destination shadow
 * intersects another record's source or destination shadow (checked, with
 * CG_ECONFLICT, under CG_DEBUG_CONFLICTS).
 * The caller keeps recs_dev and out_dev alive until the stream has synced.
 * out_dev may be NULL when CG_CHECK is not set.
 * Errors: CG_EINVAL (null pointers, mode without CHECK/PROPAGATE, more than
 * 2^32 - 1024 records),
 * CG_ESTATE (a host-side record but no host region registered), CG_EHIP.
 */
int check_transfers(cg_ctx *ctx, const cg_transfer *recs_dev, uint64_t count,
                    cg_verdict *out_dev, uint32_t mode, void *hip_stream);

/*
 * A pitched 2D copy, 64 bytes, in device memory: `rows` rows of `width`
 * bytes; row r reads [src + r*spitch, + width) and writes
 * [dst + r*dpitch, + width) (the strided copies of the footnote to Sec. 2's
 * error list).  `reserved` is ignored.
 */
typedef struct cg_transfer2d {
    uint64_t src, dst, width, rows, spitch, dpitch;
    uint32_t kind, reserved[3];
} cg_transfer2d;

/*
 * check_transfers for pitched 2D copies: every row of every record is one
 * transfer of the same batch (snapshot semantics, and the no-conflict
 * precondition of CG_PROPAGATE covers the rows), and one verdict per record
 * is written to out_dev.  The bytes of a 2D copy are numbered row by row
 * (byte c of row r is r*width + c): flags = OR over its rows, first_bad =
 * smallest r*width + first_bad_r, undef_bytes = sum, avail = the first row's
 * (bytes from src / dst to the end of its allocation).  A record with no
 * rows or width 0 gives {0, CG_NONE, 0, 0}.
 * Every record is one work item whose rows are stepped through on the device,
 * so the call does not wait for the stream and can be captured in a graph:
 * under capture it needs an earlier call on the same stream, of at least this
 * count, made after the last change of allocations or host region
 * (CG_ESTATE otherwise), and a replay reads the allocations as they were at
 * capture, so the caller replays it only while they are unchanged.
 * The rows of a record checked are those below index 2^32 that start below
 * byte 2^62 of the copy; a record with more rows gets CG_ROWS_LIMIT in its
 * flags (its other fields cover the rows checked).
 * In a check without propagation, a record whose rows all lie inside the
 * first row's allocation (or the host region) is answered from the shadow
 * indexes when check_transfers would build them for the rows' bytes: its rows
 * are not read, and its verdict is the same.
 * With CG_PLAIN or CG_DEBUG_CONFLICTS the rows are instead expanded into
 * transfer records (a launch per row, or the host-side conflict check on the
 * rows): that call waits for the stream once, to learn the number of rows, and
 * fails with CG_EINVAL above 2^32 - 1024 rows in total.
 * Modes as check_transfers otherwise; the context's tuning applies.
 * Errors: as check_transfers, and CG_EINVAL for 2^31 records or more.
 */
int check_transfers_2d(cg_ctx *ctx, const cg_transfer2d *recs_dev, uint64_t count, cg_verdict *out_dev,
                       uint32_t mode, void *hip_stream);

/* Propagation only: check_transfers(ctx, recs, count, NULL, CG_PROPAGATE, stream). */
int propagate_shadow(cg_ctx *ctx, const cg_transfer *recs_dev, uint64_t count, void *hip_stream);

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.
 * check_transfers for a batch of at most CG_NOALLOC_MAX records, with the same
 * arguments, results (verdicts, and destination shadows with CG_PROPAGATE)
 * and stream order.  The batch is worked in one launch; its per-record
 * accumulators live in a fixed device array of the library, one per GPU
 * (CG_NOALLOC_MAX * 24 bytes, set up by cg_create for its device and held
 * until the process ends), which every call leaves in its starting state.
 * The call makes no device allocation or free and no graph; its completion
 * events were made by cg_create.  Every call on one GPU shares that GPU's
 * array, so calls that overlap in time on one GPU (other streams, threads or
 * contexts) race and give wrong verdicts: the caller orders them.
 * mode: CG_CHECK and/or CG_PROPAGATE (CG_EAGER and CG_KEEP_ORDER are
 * accepted and change nothing).  Errors: CG_EINVAL (count above
 * CG_NOALLOC_MAX, CG_PLAIN or CG_DEBUG_CONFLICTS or unknown mode bits, null
 * pointers), CG_ESTATE (no array on this device), CG_EHIP.
 */
#define CG_NOALLOC_MAX 4096u
int check_transfers_noalloc(cg_ctx *ctx, const cg_transfer *recs_dev, uint64_t count, cg_verdict *out_dev,
                            uint32_t mode, void *hip_stream);

/*
 * Paper-style text for one verdict (the report of Sec. 4.5, Listing 6), for
 * host copies of a record and its verdict.  Writes at most len bytes,
 * NUL-terminated; returns the length of the full text (like snprintf), or a
 * negative status.  A clean verdict gives an empty string.
 */
int cg_format_verdict(const cg_transfer *rec, const cg_verdict *v, char *buf, uint64_t len);

/* Static text of a status code. */
const char *cg_strerror(int status);

/* Detailed text of the last failing call on ctx ("" if none). */
const char *cg_last_error(cg_ctx *ctx);

/* Block until all of the context's own stream work is done. */
int cg_sync(cg_ctx *ctx);

/* Number of live allocations and bytes of shadow pool in use. */
int cg_stats(cg_ctx *ctx, uint64_t *live_allocs, uint64_t *pool_used);

/*
 * Test hook: the device copy of the allocation list (Sec. 2, Fig. 2 caption)
 * as the next check will read it, copied to host memory.  A new table version
 * is made first if allocations or frees are pending (by device merge of the
 * previous version with the changes, or by full upload when the changes are
 * many).  base/end/off get the n live allocations sorted by base: their
 * [base, end) and the byte offset of their V bytes in the shadow pool (cap
 * entries at most); top gets every 2^shift-th base (ntop entries, top_cap at
 * most).  pool, merges and full_uploads (each may be NULL) get the pool's
 * device address and how many versions were made by device merge and by full
 * upload so far.  Synchronous; host buffers are the caller's.
 * Errors: CG_EINVAL (null arguments, buffers too small), CG_EHIP.
 */
int cg_table_read(cg_ctx *ctx, uint64_t *base, uint64_t *end, uint64_t *off, uint64_t cap, uint64_t *n,
                  uint64_t *top, uint32_t top_cap, uint32_t *ntop, uint32_t *shift, uint64_t *pool,
                  uint64_t *merges, uint64_t *full_uploads);

/* ---- concurrent accesses ------------------------------------------------- */
/*
 * Sec. 2 counts some concurrent accesses, when a program uses several
 * threads, among the errors the checker reports; the paper describes no
 * mechanism.  Reading used here: a record reads [src, src + n) and writes
 * [dst, dst + n) of the process's one address space (host and device
 * pointers never coincide); streams[i] is the stream (or thread) record i
 * was issued on, epochs[i] the number of synchronising calls made before it.
 * Records on one stream, or in different epochs, are ordered.  Two distinct
 * unordered records conflict when a written range of one meets a read or
 * written range of the other; two reads never conflict.  Every address,
 * length and epoch is decided: [src, src + n) is a range of integers that
 * does not wrap past 2^64, and only equality of epochs matters.
 */
#define CG_RACE_SRC       0x1u  /* the source bytes are written by a conflicting record */
#define CG_RACE_DST       0x2u  /* the destination bytes are read or written by a conflicting record */
#define CG_RACE_UNCHECKED 0x4u  /* kind not 0/1/2: the record names no ranges and meets nothing */

/* One result, 16 bytes, in device memory: the flags above, and the index of
 * one record this one conflicts with (CG_NONE when there is none).  When
 * several records conflict with it, which one is named is unspecified. */
typedef struct cg_race {
    uint32_t flags, reserved;
    uint64_t partner;
} cg_race;

/*
 * Join `count` records (count <= 2^30) at recs_dev against each other and
 * write one cg_race per record to out_dev, on `hip_stream`.  streams_dev
 * holds count uint32 stream ids; epochs_dev holds count uint32 epochs, or is
 * NULL for all epochs 0.  All arrays are device memory that the caller keeps
 * alive until the stream has synced.  Records with n == 0 touch nothing.
 * The shadow state and the allocation table are not used: this is a pure
 * function of the records.  Device work space is kept per stream and grows
 * to the largest batch seen.
 * Errors: CG_EINVAL (null pointers, count too large), CG_EHIP / CG_ENOMEM.
 */
int check_concurrent(cg_ctx *ctx, const cg_transfer *recs_dev, const uint32_t *streams_dev,
                     const uint32_t *epochs_dev, uint64_t count, cg_race *out_dev, void *hip_stream);

/* ---- kernel-argument pointers ---------------------------------------------- */
/*
 * The outlook (Sec. 5.1) proposes checking the pointer arguments of kernel
 * launches against the same list of allocations.  A pointer p is valid when a
 * live allocation [base, base + size) holds it, or when it is one past the end
 * of one (p == base + size, as C allows for array ends); an allocation that
 * holds p wins over one that p is one past.
 */
#define CG_PTR_UNALLOC 0x1u   /* no live allocation holds p or ends at p */

/* One result, 24 bytes, in device memory: the flag above, the allocation's
 * base, and avail = base + size - p (0 one past the end); base = avail = 0
 * with CG_PTR_UNALLOC. */
typedef struct cg_ptr_check {
    uint32_t flags, reserved;
    uint64_t base, avail;
} cg_ptr_check;

/*
 * Look up `count` pointers at ptrs_dev (device memory, u64 each) among the
 * live allocations and write one cg_ptr_check per pointer to out_dev (device
 * memory), on `hip_stream`.  Like check_transfers it sees every shadow_alloc /
 * shadow_free made before it; the caller keeps both arrays alive until the
 * stream has synced.  Errors: CG_EINVAL (null pointers, count of 2^31 or
 * more), CG_EHIP.
 */
int check_pointers(cg_ctx *ctx, const uint64_t *ptrs_dev, uint64_t count, cg_ptr_check *out_dev, void *hip_stream);

/* ---- tuning (the batched kernel's launch shape) -------------------------- */
typedef struct cg_tuning {
    uint32_t block;          /* threads per block: 256 or 512 */
    uint32_t unroll;         /* 16-byte chunks in flight per lane: 1, 2, 4 or 8 */
    uint32_t blocks_per_cu;  /* persistent blocks per compute unit */
    uint32_t tile_units;     /* 16-byte units per work tile (power of two, >= 4096) */
    uint32_t nontemporal;    /* 1: stream V with non-temporal loads */
    uint32_t reserved[3];
} cg_tuning;

int cg_get_tuning(cg_ctx *ctx, cg_tuning *t);
int cg_set_tuning(cg_ctx *ctx, const cg_tuning *t);

/*
 * Time candidate launch shapes of the batched check on these records (each
 * run is a full check; out_dev is overwritten) and keep the fastest; *best
 * (may be NULL) receives it.  If cache_path is non-NULL the choice is read
 * from / appended to that JSON-lines file, keyed by device, CU count and a
 * workload signature.  Synchronous.
 */
int cg_autotune(cg_ctx *ctx, const cg_transfer *recs_dev, uint64_t count, cg_verdict *out_dev,
                uint32_t mode, void *hip_stream, const char *cache_path, cg_tuning *best);

/*
 * Kernel timing: when enabled, each check records a pair of HIP events on the
 * caller's stream around its scan work: around the persistent scan kernel
 * (batched path; in graph mode the scan kernel then runs as a graph of its
 * own after the graph of the preparation kernels), or around the whole
 * per-record launch loop (plain path).  cg_kernel_ms waits for the pending
 * pairs, returns their summed milliseconds and their number, and forgets them.
 */
int cg_timing(cg_ctx *ctx, int enable);
int cg_kernel_ms(cg_ctx *ctx, double *ms, uint64_t *launches);

/*
 * As cg_kernel_ms, for the counting pass of the shadow indexes (one launch
 * over the host region's and the pool's listed steps per large check-only
 * batch that uses the indexes, bracketed by events while timing is on): its
 * summed time in ms since the last call, and the number of timed passes.
 * When bytes is not NULL (2 entries), it
 * receives the shadow bytes the counting passes of the indexes read since the
 * last such call, timed or not: [0] of the host region (V and A bits), [1] of
 * the shadow pool (V); that count then restarts.  A pass reads the 64 KiB
 * steps of V that the batch's records read, not the whole space.  With bytes,
 * the call waits for the device.  Errors: CG_EINVAL, CG_EHIP.
 */
int cg_index_ms(cg_ctx *ctx, double *ms, uint64_t *launches, uint64_t *bytes);

/* ---- bandwidth probes (roofline reference) -------------------------------- */
/* Read `bytes` (multiple of 16) at dev and fold them into *sink_dev (u64). */
int cg_probe_read(const void *dev, uint64_t bytes, uint64_t *sink_dev, void *hip_stream);
/* Copy `bytes` (multiple of 16) from src to dst. */
int cg_probe_copy(void *dst, const void *src, uint64_t bytes, void *hip_stream);
/* L2-resident read ceiling: dev holds 8 slices of slice_bytes (a multiple of
 * 16 KiB, at least 16 KiB); `blocks` blocks of 256 threads each read slice
 * (block mod 8), the XCD the block runs on, `passes` times with cached
 * 16-byte loads, each block from its own offset.  Bytes read =
 * blocks * slice_bytes * passes.  Errors: CG_EINVAL, CG_EHIP. */
int cg_probe_l2(const void *dev, uint64_t slice_bytes, uint32_t passes, uint32_t blocks, uint64_t *sink_dev,
                void *hip_stream);


/* ---- serving: continuous batching of check requests ----------------------- */
#define CG_EV_CHECK 0u   /* a check request */
#define CG_EV_ALLOC 1u   /* an allocation: rec.dst = address, rec.n = size */
#define CG_EV_FREE  2u   /* a free: rec.dst = address */

/* One entry of an event log, 48 bytes, host memory, ordered by t. */
typedef struct cg_serve_event {
    double t;          /* arrival time in seconds after the start of the run */
    uint32_t type;     /* CG_EV_* */
    uint32_t reserved;
    cg_transfer rec;
} cg_serve_event;

typedef struct cg_serve_config {
    uint32_t streams;        /* micro-batch slots, one HIP stream each (1..16) */
    uint32_t max_batch;      /* records per micro-batch (1..65536) */
    uint64_t mem_cap;        /* admission cap: algorithmic shadow bytes in flight */
    uint32_t plain;          /* 1: baseline, one request per check, one launch per record */
    uint32_t open_loop;      /* 1: requests arrive at their times t; 0: all at once */
    uint32_t blocks_per_cu;  /* persistent blocks per CU for a micro-batch (0: 1) */
    uint32_t reserved;
} cg_serve_config;

/* Per check request, in event-log order; host memory, 72 bytes. */
typedef struct cg_serve_result {
    cg_verdict v;
    double t_arrive;   /* scheduled arrival (open loop) or 0 */
    double t_admit;    /* when its micro-batch was issued */
    double t_done;     /* when its micro-batch finished on the GPU */
    uint64_t epoch;    /* allocation events applied before the request */
    uint32_t batch, slot;
} cg_serve_result;

typedef struct cg_serve_stats {
    double wall_s;
    uint64_t requests, batches, events;
    uint64_t max_inflight_bytes;
    uint64_t table_versions;   /* device table versions made (merges + full uploads) */
    double mean_batch;
} cg_serve_stats;

/*
 * Serve an event log: a request loop that admits check requests as they
 * arrive, keeps the shadow and the allocation table resident on the device,
 * and applies the interleaved allocation / free events in arrival order
 * (the wrappers of Sec. 2 update the context's list on every allocation and
 * free and check every copy against it).  Continuous batching: whenever a
 * slot is free, the requests that have arrived (up to max_batch, and while
 * the shadow bytes in flight stay within mem_cap) form a micro-batch that is
 * checked on that slot's stream (a graph replay); micro-batches on different
 * slots overlap on the device.  Each request is checked against the table as
 * of its arrival (every event before it in the log is applied, none after).
 * results (one per CG_EV_CHECK, in log order) and stats are host memory.
 * Synchronous: returns when every request has finished.  Errors: CG_EINVAL,
 * status codes of shadow_alloc / shadow_free for a bad event, CG_EHIP.
 */
int cg_serve_run(cg_ctx *ctx, const cg_serve_event *events, uint64_t n, const cg_serve_config *cfg,
                 cg_serve_result *results, cg_serve_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* XFERCHECK_H */
