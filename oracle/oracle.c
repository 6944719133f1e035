/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, byte-by-byte CPU evaluation of the transfer check.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load this library; the product path never calls it.  It shares no code,
 * header, table or helper with the GPU library: every struct below is
 * declared here on its own.
 *
 * What it evaluates (Baumann & Gracia, "Cudagrind", arXiv 1310.0901):
 *   - Sec. 1.1: memory has a shadow copy with bitwise precision; reading
 *     memory that was allocated but never defined, or touching memory that
 *     is not addressable, is an error.  Here: one V byte per data byte
 *     (non-zero = undefined) and one A bit per host byte (1 = addressable).
 *   - Sec. 2 and the Fig. 2 caption: the device allocations of a context are
 *     kept in a list of {device pointer, size}; every copy is cross-checked
 *     against that list.  The error classes listed in Sec. 2: copies into or
 *     from unallocated device memory; undefined host data copied to the
 *     device; more bytes copied than were allocated.
 *   - Sec. 4.5 (the worked example's report): the verdict carries the
 *     expected byte count and the bytes actually found in the allocation.
 *   - Sec. 5: definedness is tracked through host->device, device->host and
 *     device->device copies, i.e. the destination shadow receives the
 *     source's V bytes.
 *
 * For each record (src, dst, n, kind) and each byte index i in [0, n):
 *   ok_src(i), ok_dst(i)  -- a host side is valid where the byte lies inside
 *                            the registered host region and its A bit is 1;
 *                            a device side is valid for i < avail, where
 *                            avail = base + size - p of the live allocation
 *                            holding p (0 if none);
 *   undef(i)  = ok_src(i) and V_src(i) != 0;
 *   bad(i)    = !ok_src(i) or !ok_dst(i) or undef(i);
 *   first_bad = min bad index (all ones if none), undef_bytes = count of undef,
 *   avail     = min over the device sides.
 * Propagation writes V_dst(i) = ok_src(i) ? V_src(i) : 0xFF wherever
 * ok_dst(i), except for overlapping device->device copies.  All records of
 * one call read the state as it was before the call (a snapshot) and their
 * writes land afterwards.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 wide;

enum {
    OR_SRC_UNADDR = 1u, OR_SRC_UNDEF = 2u, OR_SRC_UNALLOC = 4u, OR_SRC_OVERRUN = 8u,
    OR_DST_UNADDR = 16u, OR_DST_UNALLOC = 32u, OR_DST_OVERRUN = 64u,
    OR_OVERLAP = 128u, OR_BAD_KIND = 256u
};
enum { OR_H2D = 0, OR_D2H = 1, OR_D2D = 2 };
enum { OR_MODE_CHECK = 1u, OR_MODE_PROPAGATE = 2u };
#define OR_NONE 0xFFFFFFFFFFFFFFFFull

typedef struct { uint64_t src, dst, n; uint32_t kind, reserved; } or_record;
typedef struct { uint32_t flags, reserved; uint64_t first_bad, undef_bytes, avail; } or_verdict;

typedef struct {
    uint64_t hb, hl;          /* host region [hb, hb + hl) */
    uint8_t *hv;              /* its V bytes */
    const uint64_t *ha;       /* its A bitmap, bit (x & 63) of word x >> 6 */
    uint64_t nalloc;          /* live device allocations (any order) */
    const uint64_t *abase, *asize;
    uint8_t **av;             /* V bytes of each allocation */
} or_state;

/* Is the host byte at absolute address x addressable? (Sec. 1.1) */
static int host_ok(const or_state *s, wide x)
{
    if (x < (wide)s->hb || x >= (wide)s->hb + s->hl) return 0;
    uint64_t off = (uint64_t)(x - s->hb);
    return (int)((s->ha[off >> 6] >> (off & 63)) & 1u);
}

/* The live allocation that holds address p, or -1 (Fig. 2 caption). */
static int64_t find_alloc(const or_state *s, uint64_t p)
{
    for (uint64_t j = 0; j < s->nalloc; j++)
        if ((wide)s->abase[j] <= p && (wide)p < (wide)s->abase[j] + s->asize[j])
            return (int64_t)j;
    return -1;
}

static void check_one(const or_state *rd, or_state *wr, const or_record *r,
                      or_verdict *out, int propagate)
{
    uint32_t flags = 0;
    uint64_t first = OR_NONE, undef = 0, avail = 0;
    uint64_t n = r->n;

    if (r->kind > OR_D2D) {
        out->flags = OR_BAD_KIND; out->reserved = 0;
        out->first_bad = OR_NONE; out->undef_bytes = 0; out->avail = 0;
        return;
    }
    if (n == 0) {
        out->flags = 0; out->reserved = 0;
        out->first_bad = OR_NONE; out->undef_bytes = 0; out->avail = 0;
        return;
    }
    int src_host = (r->kind == OR_H2D);
    int dst_host = (r->kind == OR_D2H);

    int64_t as = -1, ad = -1;
    uint64_t avail_s = 0, avail_d = 0;
    if (!src_host) {
        as = find_alloc(rd, r->src);
        if (as < 0) flags |= OR_SRC_UNALLOC;
        else {
            avail_s = rd->abase[as] + rd->asize[as] - r->src;
            if (n > avail_s) flags |= OR_SRC_OVERRUN;
        }
    }
    if (!dst_host) {
        ad = find_alloc(rd, r->dst);
        if (ad < 0) flags |= OR_DST_UNALLOC;
        else {
            avail_d = rd->abase[ad] + rd->asize[ad] - r->dst;
            if (n > avail_d) flags |= OR_DST_OVERRUN;
        }
    }
    int overlap = 0;
    if (r->kind == OR_D2D) {
        wide s0 = r->src, s1 = (wide)r->src + n, d0 = r->dst, d1 = (wide)r->dst + n;
        if (s0 < d1 && d0 < s1) { overlap = 1; flags |= OR_OVERLAP; }
    }

    for (uint64_t i = 0; i < n; i++) {
        int ok_s = src_host ? host_ok(rd, (wide)r->src + i) : (as >= 0 && i < avail_s);
        int ok_d = dst_host ? host_ok(rd, (wide)r->dst + i) : (ad >= 0 && i < avail_d);
        uint8_t vs = 0xFF;
        int und = 0;
        if (ok_s) {
            vs = src_host ? rd->hv[r->src + i - rd->hb]
                          : rd->av[as][r->src - rd->abase[as] + i];
            und = (vs != 0);
        }
        if (src_host && !ok_s) flags |= OR_SRC_UNADDR;
        if (dst_host && !ok_d) flags |= OR_DST_UNADDR;
        if (und) undef++;
        if (first == OR_NONE && (!ok_s || !ok_d || und)) first = i;
        if (propagate && !overlap && ok_d) {
            uint8_t w = ok_s ? vs : 0xFF;
            if (dst_host) wr->hv[r->dst + i - wr->hb] = w;
            else wr->av[ad][r->dst - wr->abase[ad] + i] = w;
        }
    }
    if (undef) flags |= OR_SRC_UNDEF;

    if (src_host) avail = avail_d;
    else if (dst_host) avail = avail_s;
    else avail = avail_s < avail_d ? avail_s : avail_d;

    out->flags = flags; out->reserved = 0;
    out->first_bad = first; out->undef_bytes = undef; out->avail = avail;
}

/*
 * Evaluate `count` records.  mode bit 0: write verdicts to `out` (may be NULL
 * otherwise); bit 1: propagate V bytes into hv / av.  Returns 0, or -1 if
 * memory for the snapshot could not be obtained.
 */
int oracle_run(uint64_t hb, uint64_t hl, uint8_t *hv, const uint64_t *ha,
               uint64_t nalloc, const uint64_t *abase, const uint64_t *asize,
               uint8_t **av, uint64_t count, const or_record *recs,
               or_verdict *out, uint32_t mode)
{
    or_state live = { hb, hl, hv, ha, nalloc, abase, asize, av };
    or_state snap = live;
    int propagate = (mode & OR_MODE_PROPAGATE) != 0;
    uint8_t *hv_copy = NULL;
    uint8_t **av_copy = NULL;

    if (propagate) {
        /* reads see the state before the call: take a full copy to read from */
        hv_copy = (uint8_t *)malloc(hl ? hl : 1);
        av_copy = (uint8_t **)calloc(nalloc ? nalloc : 1, sizeof(uint8_t *));
        if (!hv_copy || !av_copy) { free(hv_copy); free(av_copy); return -1; }
        memcpy(hv_copy, hv, hl);
        for (uint64_t j = 0; j < nalloc; j++) {
            av_copy[j] = (uint8_t *)malloc(asize[j] ? asize[j] : 1);
            if (!av_copy[j]) {
                for (uint64_t k = 0; k < j; k++) free(av_copy[k]);
                free(av_copy); free(hv_copy);
                return -1;
            }
            memcpy(av_copy[j], av[j], asize[j]);
        }
        snap.hv = hv_copy;
        snap.av = av_copy;
    }

    or_verdict scratch;
    for (uint64_t t = 0; t < count; t++) {
        or_verdict *o = (out && (mode & OR_MODE_CHECK)) ? &out[t] : &scratch;
        check_one(&snap, &live, &recs[t], o, propagate);
    }

    if (propagate) {
        for (uint64_t j = 0; j < nalloc; j++) free(av_copy[j]);
        free(av_copy);
        free(hv_copy);
    }
    return 0;
}

/*
 * Concurrent accesses.  Next to the copy errors, Sec. 2 names the detection
 * of some concurrent accesses in programs that use several threads, without
 * describing a mechanism.  The reading evaluated here:
 *   - a record (src, dst, n, kind) reads the bytes R = [src, src + n) and
 *     writes the bytes W = [dst, dst + n), all in the process's one address
 *     space (host and device pointers never coincide);
 *   - each record also carries the stream it was issued on and an epoch,
 *     the number of synchronising calls made before it was issued; two
 *     records are ordered when they share a stream or differ in epoch;
 *   - distinct records a and b conflict when they are unordered and
 *     W_a meets W_b, W_a meets R_b, or R_a meets W_b (two reads never
 *     conflict);
 *   - flags of a: RACE_SRC when R_a meets W_b of a conflicting b, RACE_DST
 *     when W_a meets W_b or R_b of a conflicting b;
 *   - byte ranges are sets of integers: [src, src + n) never wraps, even
 *     where src + n exceeds 2^64; any 32-bit epoch and any address count;
 *   - a record whose kind is not 0, 1 or 2 names no ranges: it is not
 *     checked (RACE_UNCHECKED) and meets nothing.  n == 0 touches no byte.
 * Each requested record is compared with every other record, one pair at a
 * time.
 */
enum { OR_RACE_SRC = 1u, OR_RACE_DST = 2u, OR_RACE_UNCHECKED = 4u };

static int race_unchecked(const or_record *r) { return r->kind > OR_D2D; }

/* do [a, a + na) and [b, b + nb) share a byte? */
static int meets(uint64_t a, uint64_t na, uint64_t b, uint64_t nb)
{
    return na > 0 && nb > 0 && (wide)a < (wide)b + nb && (wide)b < (wide)a + na;
}

void oracle_race(uint64_t count, const or_record *recs, const uint32_t *streams,
                 const uint32_t *epochs, uint64_t nwhich, const uint64_t *which,
                 uint32_t *flags)
{
    for (uint64_t k = 0; k < nwhich; k++) {
        uint64_t a = which[k];
        const or_record *ra = &recs[a];
        uint32_t ea = epochs ? epochs[a] : 0;
        uint32_t f = 0;
        if (race_unchecked(ra)) {
            flags[k] = OR_RACE_UNCHECKED;
            continue;
        }
        for (uint64_t b = 0; b < count; b++) {
            if (b == a) continue;
            const or_record *rb = &recs[b];
            uint32_t eb = epochs ? epochs[b] : 0;
            if (race_unchecked(rb)) continue;
            if (eb != ea || streams[b] == streams[a]) continue;
            if (meets(ra->dst, ra->n, rb->dst, rb->n) || meets(ra->dst, ra->n, rb->src, rb->n))
                f |= OR_RACE_DST;
            if (meets(ra->src, ra->n, rb->dst, rb->n))
                f |= OR_RACE_SRC;
        }
        flags[k] = f;
    }
}

/*
 * Kernel-argument pointers.  The outlook (Sec. 5.1) proposes checking the
 * pointer arguments of kernel launches against the same list of allocations.
 * Reading evaluated here: a pointer p is valid when a live allocation
 * [base, base + size) holds it, or when it is one past the end of one
 * (p == base + size, as C allows for array ends); an allocation that holds p
 * wins over one that p is one past.  Then base is that allocation's base and
 * avail = base + size - p (0 one past the end).  Otherwise PTR_UNALLOC with
 * base = avail = 0.
 */
enum { OR_PTR_UNALLOC = 1u };
typedef struct { uint32_t flags, reserved; uint64_t base, avail; } or_ptr;

void oracle_pointers(uint64_t nalloc, const uint64_t *abase, const uint64_t *asize, uint64_t count,
                     const uint64_t *ptrs, or_ptr *out)
{
    for (uint64_t t = 0; t < count; t++) {
        uint64_t p = ptrs[t];
        int64_t hold = -1, past = -1;
        for (uint64_t j = 0; j < nalloc; j++) {
            wide end = (wide)abase[j] + asize[j];
            if ((wide)abase[j] <= p && (wide)p < end) hold = (int64_t)j;
            else if ((wide)p == end) past = (int64_t)j;
        }
        int64_t j = hold >= 0 ? hold : past;
        out[t].reserved = 0;
        if (j < 0) {
            out[t].flags = OR_PTR_UNALLOC;
            out[t].base = 0;
            out[t].avail = 0;
        } else {
            out[t].flags = 0;
            out[t].base = abase[j];
            out[t].avail = abase[j] + asize[j] - p;
        }
    }
}
