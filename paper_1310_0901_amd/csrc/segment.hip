// Work of a large check batch in order of source block (gfx950).
//
// A batch whose records read the same bytes many times keeps the re-reads in
// cache only if the work on one stretch of source memory runs at about the
// same time, on one XCD.  Ordering whole records by source address falls
// short of that: a large record covers megabytes past its start, while the
// records that start inside that range come much later.  Here every record's
// units are cut where its source chunks cross a multiple of a block size B
// in shadow memory; the pieces ("segments") are sorted by block (stable, so
// in record order inside a block) and become the positions of the batch:
// position p holds the record's descriptor with its first unit moved to the
// segment's first unit, and the record's index for the findings.  Verdicts
// do not change: a record's findings combine by OR / min / sum over any split
// of its units, as they already do over the tiles of the scan kernel.
//
// B is the smallest power of two at or above both 2^min_log2 and
// 16 * ceil(W / count), W the sum of the records' work weights (units, at
// least 1).  A record of L source bytes spans at most L / B + 2 blocks, so a
// batch has at most 3 * count segments: the positions the caller provides.
// Records with units that read no source byte stay one segment, with key 0;
// records without units (nothing to scan: their verdicts are complete, as
// for those the shadow indexes answered) have none.
//
//   k_seg_plan    one block: W, then log2 B
//   k_seg_count   one lane per record: segments, block-local prefix
//   k_seg_scan    one block: prefix of the block sums; the segment count
//   k_seg_first   one lane per record: its first segment
//   k_seg_keys    one lane per segment: its record (binary search), key =
//                 block, value = segment; per block the key bits that differ
//                 from segment 0's key, for the sort's pass mask
//   (sort.hip)    stable radix sort of the segments' keys
//   k_seg_layout  one lane per position: descriptor, record, work weight
//                 (positions past the segments: empty, weight 0), and the
//                 block-local prefix and block sums that k_classify makes
//                 for a batch in its given order
#include <hip/hip_runtime.h>

#include "xc_internal.h"
#include "sort.h"

namespace xc {
namespace {

constexpr int kT = 256;
static_assert(kT == kClassifyBlock, "position blocks match the classify blocks of the scan kernels");
static_assert(kT == kSortKeyBlock, "one part of the key mask per block of k_seg_keys");

// the record reads source bytes through its units
__device__ __forceinline__ bool seg_split(const Desc &d) { return d.units > 0 && d.v_hi > d.v_lo; }

// shadow address of the source chunk of the record's first unit
__device__ __forceinline__ uint64_t seg_a0(const Desc &d)
{
    const uint64_t delta = (d.ctl & CTL_DELTA) ? 1u : 0u;
    return d.src_sh + 16u * (d.e0 - delta);
}

__device__ __forceinline__ uint64_t seg_count(const Desc &d, uint32_t lb)
{
    if (d.units == 0) return 0;
    if (!seg_split(d)) return 1;
    const uint64_t a0 = seg_a0(d), a1 = a0 + 16u * (d.units - 1);
    return (a1 >> lb) - (a0 >> lb) + 1;
}

// a segment of a record whose source is the host region
__device__ __forceinline__ bool seg_host(const Desc &d) { return seg_split(d) && (d.ctl & CTL_SRC_HOST); }

// the block of segment j; with host_last, host-source segments after all
// others (the key's top bit: bit 31 of 4-byte keys, else bit 63)
__device__ __forceinline__ uint64_t seg_key(const SegArgs &g, const Desc &d, uint32_t lb, uint64_t j)
{
    if (!seg_split(d)) return 0ull;
    const uint64_t top = g.key_bytes == 4 ? 1ull << 31 : 1ull << 63;
    return ((seg_a0(d) >> lb) + j) | (g.host_last && (d.ctl & CTL_SRC_HOST) ? top : 0ull);
}

// units [u0, u1) of segment j
__device__ __forceinline__ void seg_range(const Desc &d, uint32_t lb, uint64_t j, uint64_t *u0, uint64_t *u1)
{
    if (!seg_split(d)) {
        *u0 = 0;
        *u1 = d.units;
        return;
    }
    const uint64_t a0 = seg_a0(d), b0 = a0 >> lb;
    *u0 = j == 0 ? 0 : (((b0 + j) << lb) - a0) >> 4;
    const uint64_t e = (((b0 + j + 1) << lb) - a0) >> 4;
    *u1 = e < d.units ? e : d.units;
}

// exclusive prefix over the block; *total receives the block's sum
__device__ uint64_t block_excl(uint64_t x, uint64_t *total)
{
    __shared__ uint64_t wsum[kT / 64];
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    uint64_t inc = x;
    for (uint32_t d = 1; d < 64u; d <<= 1) {
        const uint64_t y = __shfl_up(inc, d);
        if (lane >= d) inc += y;
    }
    if (lane == 63u) wsum[w] = inc;
    __syncthreads();
    uint64_t off = 0, tot = 0;
    for (uint32_t k = 0; k < kT / 64; ++k) {
        if (k < w) off += wsum[k];
        tot += wsum[k];
    }
    *total = tot;
    return off + inc - x;
}

__global__ void __launch_bounds__(1024) k_seg_plan(SegArgs g, uint64_t nbr)
{
    __shared__ uint64_t wsum[16];
    uint64_t s = 0;
    for (uint64_t b = threadIdx.x; b < nbr; b += 1024) s += g.wbsum[b];
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
    if ((threadIdx.x & 63u) == 0) wsum[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t tot = 0;
        for (int k = 0; k < 16; ++k) tot += wsum[k];
        const uint64_t per = (tot + g.count - 1) / g.count;   // tot >= count >= 1
        const uint64_t need = 16u * per;
        uint32_t lb = need <= 1 ? 0u : 64u - (uint32_t)__clzll(need - 1);
        if (lb < g.min_log2) lb = g.min_log2;
        g.meta[1] = lb;
    }
}

__global__ void __launch_bounds__(kT) k_seg_count(SegArgs g)
{
    const uint64_t r = (uint64_t)blockIdx.x * kT + threadIdx.x;
    const uint32_t lb = (uint32_t)g.meta[1];
    const uint64_t c = r < g.count ? seg_count(g.rdesc[r], lb) : 0;
    uint64_t tot;
    const uint64_t ex = block_excl(c, &tot);
    if (r < g.count) g.first[r] = ex;
    if (threadIdx.x == 0) g.sbsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) k_seg_scan(SegArgs g, uint64_t nbr)
{
    __shared__ uint64_t wsum[16];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
    const uint64_t per = (nbr + 1023) / 1024;
    const uint64_t b0 = tid * per < nbr ? tid * per : nbr, b1 = b0 + per < nbr ? b0 + per : nbr;
    uint64_t s = 0;
    for (uint64_t b = b0; b < b1; ++b) s += g.sbsum[b];
    uint64_t x = s;
    for (uint32_t d = 1; d < 64u; d <<= 1) {
        const uint64_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63u) wsum[w] = x;
    __syncthreads();
    uint64_t off = 0;
    for (uint32_t k = 0; k < w; ++k) off += wsum[k];
    uint64_t run = off + x - s;
    for (uint64_t b = b0; b < b1; ++b) {
        const uint64_t v = g.sbsum[b];
        g.sbsum[b] = run;
        run += v;
    }
    if (tid == 1023) {
        const uint64_t total = off + x;
        g.meta[0] = total < g.npos ? total : g.npos;   // total <= 3 * count = npos by the choice of B
        g.meta[2] = g.meta[0];                           // no host-source position yet (k_seg_layout)
    }
}

__global__ void __launch_bounds__(kT) k_seg_first(SegArgs g)
{
    const uint64_t r = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (r < g.count) g.first[r] += g.sbsum[blockIdx.x];
}

// The record holding segment q < ns: the last r with first[r] <= q (first[]
// does not decrease, and a record without segments shares its first with the
// records after it up to the next one that has some).
__device__ __forceinline__ uint64_t seg_record(const SegArgs &g, uint64_t q)
{
    uint64_t lo = 0, hi = g.count - 1;
    while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) >> 1;
        if (g.first[mid] <= q) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(kT) k_seg_keys(SegArgs g, uint64_t *keys, uint32_t *vals, uint64_t *parts)
{
    __shared__ uint64_t part[kT / 64];
    const uint64_t ns = g.meta[0];
    const uint32_t lb = (uint32_t)g.meta[1];
    const uint64_t q = (uint64_t)blockIdx.x * kT + threadIdx.x;
    uint64_t x = 0;
    if (q < ns) {
        const uint64_t r0 = seg_record(g, 0);
        const uint64_t key0 = seg_key(g, g.rdesc[r0], lb, 0);   // segment 0's
        const uint64_t lo = seg_record(g, q);
        const uint64_t key = seg_key(g, g.rdesc[lo], lb, q - g.first[lo]);
        keys[q] = key;
        vals[q] = (uint32_t)q;
        g.srec[q] = (uint32_t)lo;
        x = key ^ key0;
    }
    for (int d = 32; d >= 1; d >>= 1) x |= __shfl_xor(x, d);
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t y = 0;
        for (int k = 0; k < kT / 64; ++k) y |= part[k];
        parts[blockIdx.x] = y;
    }
}

__global__ void __launch_bounds__(kT) k_seg_layout(SegArgs g, const uint32_t *va, const uint32_t *vb,
                                                   const uint64_t *maskp, Desc *desc, uint32_t *perm,
                                                   uint64_t *weight, uint64_t *local, uint64_t *bsum)
{
    const uint64_t ns = g.meta[0];
    const uint32_t lb = (uint32_t)g.meta[1];
    const uint32_t *sorted = sort_parity(*maskp) ? vb : va;
    const uint64_t p = (uint64_t)blockIdx.x * kT + threadIdx.x;
    uint64_t w = 0;
    if (p < g.npos) {
        Desc o = {};
        uint32_t r = 0;
        bool host = false;
        if (p < ns) {
            const uint32_t q = sorted[p];
            r = g.srec[q];
            const Desc d = g.rdesc[r];
            uint64_t u0, u1;
            seg_range(d, lb, q - g.first[r], &u0, &u1);
            o = d;
            o.e0 = d.e0 + u0;
            o.units = u1 - u0;
            host = g.host_last && seg_host(d);
            // the first host-source position (they sort last)
            if (host && (p == 0 || !seg_host(g.rdesc[g.srec[sorted[p - 1]]]))) g.meta[2] = p;
            desc[p] = o;
            perm[p] = r;
        }
        // (the positions past the segments weigh 0: no unit reaches them, so
        // their descriptor and record are never read)
        weight[p] = o.units;
        // a segment weighs its units (at least 1: records without units have
        // no segment); the empty positions past the segments, and with
        // host_last the host-source ones (worked by k_host_lds), weigh 0, so
        // no unit of the scan kernel reaches them
        w = p < ns && !host ? o.units : 0;
    }
    uint64_t tot;
    const uint64_t ex = block_excl(w, &tot);
    if (p < g.npos) local[p] = ex;
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

}  // namespace

hipError_t launch_segments(const SegArgs &g, SortWs &sort, const BatchArgs &ap, uint32_t *perm, hipStream_t s)
{
    const uint64_t nbr = ceil_div(g.count, kT), nbp = ceil_div(g.npos, kT);
    hipLaunchKernelGGL(k_seg_plan, dim3(1), dim3(1024), 0, s, g, nbr);
    hipLaunchKernelGGL(k_seg_count, dim3((uint32_t)nbr), dim3(kT), 0, s, g);
    hipLaunchKernelGGL(k_seg_scan, dim3(1), dim3(1024), 0, s, g, nbr);
    hipLaunchKernelGGL(k_seg_first, dim3((uint32_t)nbr), dim3(kT), 0, s, g);
    hipLaunchKernelGGL(k_seg_keys, dim3((uint32_t)nbp), dim3(kT), 0, s, g, sort.keys[0], sort.vals[0], sort.parts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = sort_pairs(sort, g.npos, s, g.meta, (int)g.key_bytes)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_seg_layout, dim3((uint32_t)nbp), dim3(kT), 0, s, g, sort.vals[0], sort.vals[1], sort.mask,
                       ap.desc, perm, ap.weight, ap.local, ap.bsum);
    return hipGetLastError();
}

}  // namespace xc
