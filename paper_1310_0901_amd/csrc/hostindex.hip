// Index of the host region's faulty chunks for large check-only batches (gfx950).
//
// A batch worked as segments reads every host byte many times (about 160 on
// the 1M-record configuration).  A host-to-device record checked without
// propagation needs three facts about its valid source bytes [a, b) (region
// offsets): how many are undefined (V != 0 where A = 1), the first undefined
// one and the first unaddressable one (A = 0).  Its destination is device
// memory, whose range the lookup of k_classify has already judged.  Here the
// region is read once per batch into two sorted lists, the chunks holding an
// undefined byte (with its mask and the undefined bytes of all chunks before
// it) and the chunks holding an unaddressable byte (with its mask), and each
// such record's facts come from two binary searches per list and the masks of
// its edge chunks.  When faults are rare the lists are short; when either
// would exceed its capacity, or the batch reads too few host bytes to repay a
// pass over the region, the index stays invalid and the records are scanned
// as before.  The facts are exact, so verdicts do not depend on the choice.
//
//   k_hidx_reset   one lane: state = {0, 0, 0, 0}
//   (k_classify adds the batch's valid host-source bytes to state[0])
//   k_hidx_count   block b over its contiguous range of chunks: list entries
//                  and undefined bytes
//   k_hidx_scan    one block: the blocks' offsets, the totals, validity
//   k_hidx_fill    block b writes its entries in chunk order (a block with
//                  none returns at once)
//   k_hidx_query   one lane per record: answers the host-to-device records
//                  of a check without propagation into their verdicts, and
//                  takes their units out of the scan
#include <hip/hip_runtime.h>

#include "xc_internal.h"

namespace xc {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 256;
constexpr uint32_t kPer = 16;                          // chunks per thread per step
constexpr uint64_t kStep = (uint64_t)kT * kPer;        // chunks per block per step

// one bit per non-zero byte of w (SWAR: no carry crosses a byte)
__device__ __forceinline__ uint32_t nz4(uint32_t w)
{
    const uint32_t t = (((w & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | w) & 0x80808080u;
    return ((t >> 7) | (t >> 14) | (t >> 21) | (t >> 28)) & 0xFu;
}

__device__ __forceinline__ uint32_t nz16(u32x4 v)
{
    return nz4(v.x) | (nz4(v.y) << 4) | (nz4(v.z) << 8) | (nz4(v.w) << 12);
}

__device__ __forceinline__ uint64_t region_chunks(const Region &R) { return (R.hl + 15) >> 4; }

// the index is built for this batch: a region, and enough host-source bytes
__device__ __forceinline__ bool worth(const HostIndex &x, const Region &R)
{
    return R.hl > 0 && (x.ratio == 0 || x.state[0] / x.ratio >= R.hl);
}

// chunks [lo, hi) of block b
__device__ __forceinline__ void block_range(const Region &R, uint32_t grid, uint32_t b, uint64_t *lo, uint64_t *hi)
{
    const uint64_t n = region_chunks(R);
    const uint64_t steps = (n + (uint64_t)grid * kStep - 1) / ((uint64_t)grid * kStep);
    const uint64_t span = steps * kStep;
    *lo = (uint64_t)b * span < n ? (uint64_t)b * span : n;
    *hi = *lo + span < n ? *lo + span : n;
}

// undefined (V != 0, A = 1) and unaddressable (A = 0) bytes of chunk c < the
// region's chunks; bits of bytes past the region's end are clear
__device__ __forceinline__ void chunk_faults(const Region &R, uint64_t c, uint32_t *und, uint32_t *un)
{
    const u32x4 v = *reinterpret_cast<const u32x4 *>(R.v + 16 * c);
    const uint32_t a = R.a16[c];
    const uint64_t left = R.hl - 16 * c;
    const uint32_t live = left < 16 ? (1u << left) - 1u : 0xFFFFu;
    *und = nz16(v) & a & live;
    *un = ~a & live;
}

// block-wide exclusive scan of three values; tot receives the block's sums
__device__ void block_scan3(uint64_t x[3], uint64_t ex[3], uint64_t tot[3])
{
    __shared__ uint64_t ws[kT / 64][3];
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    uint64_t inc[3] = {x[0], x[1], x[2]};
    for (uint32_t d = 1; d < 64u; d <<= 1) {
        uint64_t y[3];
        for (int k = 0; k < 3; ++k) y[k] = __shfl_up(inc[k], d);
        if (lane >= d)
            for (int k = 0; k < 3; ++k) inc[k] += y[k];
    }
    if (lane == 63u)
        for (int k = 0; k < 3; ++k) ws[w][k] = inc[k];
    __syncthreads();
    for (int k = 0; k < 3; ++k) {
        uint64_t off = 0, all = 0;
        for (uint32_t q = 0; q < kT / 64; ++q) {
            if (q < w) off += ws[q][k];
            all += ws[q][k];
        }
        ex[k] = off + inc[k] - x[k];
        tot[k] = all;
    }
    __syncthreads();   // ws is reused by the next call
}

__global__ void k_hidx_reset(HostIndex x)
{
    for (int k = 0; k < 4; ++k) x.state[k] = 0;
}

__global__ void __launch_bounds__(kT) k_hidx_count(HostIndex x, const DevState *stp)
{
    const Region R = stp->region;
    if (!worth(x, R)) return;
    uint64_t lo, hi;
    block_range(R, x.grid, blockIdx.x, &lo, &hi);
    uint64_t c3[3] = {0, 0, 0};
    for (uint64_t base = lo; base < hi; base += kStep) {
#pragma unroll 4
        for (uint32_t j = 0; j < kPer; ++j) {
            const uint64_t c = base + (uint64_t)j * kT + threadIdx.x;
            if (c < hi) {
                uint32_t und, un;
                chunk_faults(R, c, &und, &un);
                c3[0] += und ? 1u : 0u;
                c3[1] += un ? 1u : 0u;
                c3[2] += (uint32_t)__builtin_popcount(und);
            }
        }
    }
    uint64_t ex[3], tot[3];
    block_scan3(c3, ex, tot);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) x.bcnt[3 * blockIdx.x + k] = tot[k];
}

// offsets of the blocks' entries in [3 grid, 6 grid) of bcnt
__global__ void __launch_bounds__(1024) k_hidx_scan(HostIndex x, const DevState *stp)
{
    __shared__ uint64_t ws[16][3];
    const Region R = stp->region;
    if (!worth(x, R)) {
        if (threadIdx.x == 0) x.state[1] = 0;
        return;
    }
    const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
    const uint32_t per = (x.grid + 1023) / 1024;
    const uint32_t b0 = tid * per < x.grid ? tid * per : x.grid, b1 = b0 + per < x.grid ? b0 + per : x.grid;
    uint64_t s[3] = {0, 0, 0};
    for (uint32_t b = b0; b < b1; ++b)
        for (int k = 0; k < 3; ++k) s[k] += x.bcnt[3 * b + k];
    uint64_t inc[3] = {s[0], s[1], s[2]};
    for (uint32_t d = 1; d < 64u; d <<= 1) {
        uint64_t y[3];
        for (int k = 0; k < 3; ++k) y[k] = __shfl_up(inc[k], d);
        if (lane >= d)
            for (int k = 0; k < 3; ++k) inc[k] += y[k];
    }
    if (lane == 63u)
        for (int k = 0; k < 3; ++k) ws[w][k] = inc[k];
    __syncthreads();
    uint64_t run[3];
    for (int k = 0; k < 3; ++k) {
        uint64_t off = 0;
        for (uint32_t q = 0; q < w; ++q) off += ws[q][k];
        run[k] = off + inc[k] - s[k];
    }
    for (uint32_t b = b0; b < b1; ++b)
        for (int k = 0; k < 3; ++k) {
            x.bcnt[3 * (x.grid + b) + k] = run[k];
            run[k] += x.bcnt[3 * b + k];
        }
    if (tid == 1023) {
        // run[] now holds the totals (thread 1023 covers the last blocks, or none)
        uint64_t tot[3];
        for (int k = 0; k < 3; ++k) {
            uint64_t all = 0;
            for (uint32_t q = 0; q < 16; ++q) all += ws[q][k];
            tot[k] = all;
        }
        const bool valid = tot[0] <= x.cap_u && tot[1] <= x.cap_n;
        x.state[1] = valid ? 1u : 0u;
        x.state[2] = tot[0];
        x.state[3] = tot[1];
        if (valid) {
            x.uchunk[tot[0]] = ~0ull;
            x.ucum[tot[0]] = tot[2];
        }
    }
}

__global__ void __launch_bounds__(kT) k_hidx_fill(HostIndex x, const DevState *stp)
{
    if (!x.state[1]) return;
    const Region R = stp->region;
    const uint32_t b = blockIdx.x;
    if (x.bcnt[3 * b] == 0 && x.bcnt[3 * b + 1] == 0) return;
    uint64_t lo, hi;
    block_range(R, x.grid, b, &lo, &hi);
    uint64_t ou = x.bcnt[3 * (x.grid + b)], on = x.bcnt[3 * (x.grid + b) + 1], op = x.bcnt[3 * (x.grid + b) + 2];
    const uint64_t end_u = ou + x.bcnt[3 * b], end_n = on + x.bcnt[3 * b + 1];
    for (uint64_t base = lo; base < hi && (ou < end_u || on < end_n); base += kStep) {
        for (uint32_t j = 0; j < kPer; ++j) {
            const uint64_t c = base + (uint64_t)j * kT + threadIdx.x;
            uint32_t und = 0, un = 0;
            if (c < hi) chunk_faults(R, c, &und, &un);
            uint64_t v[3] = {und ? 1u : 0u, un ? 1u : 0u, (uint64_t)__builtin_popcount(und)};
            uint64_t ex[3], tot[3];
            block_scan3(v, ex, tot);
            if (und) {
                x.uchunk[ou + ex[0]] = c;
                x.umask[ou + ex[0]] = und;
                x.ucum[ou + ex[0]] = op + ex[2];
            }
            if (un) {
                x.nchunk[on + ex[1]] = c;
                x.nmask[on + ex[1]] = un;
            }
            ou += tot[0];
            on += tot[1];
            op += tot[2];
        }
    }
}

// first i in [0, n) with key[i] >= k (n if none)
__device__ __forceinline__ uint64_t lower_bound(const uint64_t *key, uint64_t n, uint64_t k)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (key[mid] < k) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// bytes of chunk c inside region offsets [a, b), as a mask (ca = a / 16, cb = (b - 1) / 16)
__device__ __forceinline__ uint32_t range_mask(uint64_t c, uint64_t ca, uint64_t cb, uint32_t lo_bit, uint32_t hi_bit)
{
    uint32_t m = 0xFFFFu;
    if (c == ca) m &= (0xFFFFu << lo_bit) & 0xFFFFu;
    if (c == cb) m &= (2u << hi_bit) - 1u;
    return m;
}

// first faulty byte in [a, b) among list entries [i0, i1) (region offset, or ~0):
// only the first two entries can hold it, since every entry's mask is non-zero
// and only the edge chunks are cut
__device__ __forceinline__ uint64_t first_in(const uint64_t *chunk, const uint32_t *mask, uint64_t i0, uint64_t i1,
                                             uint64_t ca, uint64_t cb, uint32_t lo_bit, uint32_t hi_bit)
{
    for (uint64_t i = i0; i < i1 && i < i0 + 2; ++i) {
        const uint32_t bits = mask[i] & range_mask(chunk[i], ca, cb, lo_bit, hi_bit);
        if (bits) return 16 * chunk[i] + (uint64_t)__builtin_ctz(bits);
    }
    return ~0ull;
}

__global__ void __launch_bounds__(kT) k_hidx_query(BatchArgs a, HostIndex x, uint64_t *wbsum)
{
    const uint64_t t = (uint64_t)blockIdx.x * kT + threadIdx.x;
    uint64_t removed = 0;
    if (x.state[1] && a.out && t < a.count) {
        const Desc d = a.desc[t];
        // a host source and nothing to do on the destination: a host-to-device
        // record checked without propagation
        if ((d.ctl & CTL_SRC_HOST) && (d.ctl & CTL_CHECK) && !(d.ctl & (CTL_PROP | CTL_DST_A)) && d.units > 0 &&
            d.v_hi > d.v_lo) {
            const uint32_t phi = (d.ctl >> CTL_PHI_SHIFT) & 15u;
            const int64_t off0 = d.a_src + (int64_t)phi;   // region offset of the record's byte 0
            const uint64_t ra = (uint64_t)(off0 + d.v_lo), rb = (uint64_t)(off0 + d.v_hi);
            const uint64_t ca = ra >> 4, cb = (rb - 1) >> 4;
            const uint32_t lo_bit = (uint32_t)(ra & 15u), hi_bit = (uint32_t)((rb - 1) & 15u);
            const uint64_t nu = x.state[2], nn = x.state[3];
            // undefined bytes: running counts between the edge entries, minus the
            // edge chunks' bytes outside [ra, rb)
            const uint64_t i0 = lower_bound(x.uchunk, nu, ca), i1 = lower_bound(x.uchunk, nu, cb + 1);
            uint64_t undef = x.ucum[i1] - x.ucum[i0];
            if (i1 > i0) {
                if (x.uchunk[i0] == ca) undef -= (uint64_t)__builtin_popcount(x.umask[i0] & ~(0xFFFFu << lo_bit) & 0xFFFFu);
                if (x.uchunk[i1 - 1] == cb) undef -= (uint64_t)__builtin_popcount(x.umask[i1 - 1] & ~((2u << hi_bit) - 1u));
            }
            const uint64_t fu = first_in(x.uchunk, x.umask, i0, i1, ca, cb, lo_bit, hi_bit);
            const uint64_t j0 = lower_bound(x.nchunk, nn, ca), j1 = lower_bound(x.nchunk, nn, cb + 1);
            const uint64_t fn = first_in(x.nchunk, x.nmask, j0, j1, ca, cb, lo_bit, hi_bit);
            cg_verdict v = a.out[t];
            uint64_t first = v.first_bad;
            if (undef) {
                v.flags |= CG_SRC_UNDEF;
                const uint64_t i = (uint64_t)((int64_t)fu - off0);
                first = i < first ? i : first;
            }
            if (fn != ~0ull) {
                v.flags |= CG_SRC_UNADDR;
                const uint64_t i = (uint64_t)((int64_t)fn - off0);
                first = i < first ? i : first;
            }
            v.first_bad = first;
            v.undef_bytes += undef;
            a.out[t] = v;
            a.desc[t].units = 0;
            removed = d.units - 1;   // its weight max(units, 1) becomes 1
        }
    }
    // the block's weight sum as k_classify left it, for the segment plan
    uint64_t r = removed;
    for (int k = 32; k >= 1; k >>= 1) r += __shfl_xor(r, k);
    __shared__ uint64_t wr[kT / 64];
    if ((threadIdx.x & 63u) == 0) wr[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t all = 0;
        for (int k = 0; k < kT / 64; ++k) all += wr[k];
        if (all) wbsum[blockIdx.x] -= all;
    }
}

}  // namespace

hipError_t launch_hidx_reset(const HostIndex &x, hipStream_t s)
{
    hipLaunchKernelGGL(k_hidx_reset, dim3(1), dim3(1), 0, s, x);
    return hipGetLastError();
}

hipError_t launch_hidx_build(const HostIndex &x, const DevState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_hidx_count, dim3(x.grid), dim3(kT), 0, s, x, st);
    hipLaunchKernelGGL(k_hidx_scan, dim3(1), dim3(1024), 0, s, x, st);
    hipLaunchKernelGGL(k_hidx_fill, dim3(x.grid), dim3(kT), 0, s, x, st);
    return hipGetLastError();
}

hipError_t launch_hidx_query(const BatchArgs &ar, const HostIndex &x, uint64_t *wbsum, hipStream_t s)
{
    const uint64_t blocks = (ar.count + kT - 1) / kT;
    hipLaunchKernelGGL(k_hidx_query, dim3((uint32_t)blocks), dim3(kT), 0, s, ar, x, wbsum);
    return hipGetLastError();
}

}  // namespace xc
