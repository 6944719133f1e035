// Indexes of the faulty shadow chunks for large check-only batches (gfx950).
//
// A batch worked as segments reads the same shadow bytes many times (each
// host byte about 160 times, each device byte about 15 times on the
// 1M-record configuration).  A record checked without propagation needs few
// facts about the bytes it reads: for its valid source bytes, how many are
// undefined (V != 0 where A = 1), the first undefined one and the first
// unaddressable one (A = 0, host sources only); for the valid bytes of a host
// destination, the first unaddressable one.  The ranges themselves were
// judged by k_classify's lookups.  Here the parts of each shadow space the
// batch reads heavily (its steps of 4,096 chunks that some record reads) are
// read once into two sorted lists: the chunks holding an undefined byte, with
// its mask and the undefined bytes of all chunks before it, and the chunks
// holding an unaddressable byte, with its mask.  A record's facts then come
// from two binary searches per list and the masks of its edge chunks: its
// range lies inside listed steps, so the entries between its searches are
// all of its faulty chunks.  The spaces are the host region (V and A bits) and the shadow pool
// (V only; addressability there is the allocation table's).  An index is
// built when the batch's valid bytes in its space reach `ratio` times the
// space's length, and is valid when both lists fit their capacity; a record
// whose spaces all have a valid index is answered and leaves the scan, any
// other is scanned as before.  The facts are exact, so verdicts do not depend
// on the choice.
//
//   k_sidx_reset   one lane: both states = {0, ...}
//   (k_classify adds the batch's valid bytes per space to state[0], and
//   marks the steps of 4,096 chunks that its records read)
//   k_sidx_mark_count, k_sidx_mark_list
//                  the marked steps as an ascending list (marks cleared)
//   k_sidx_count   block b over its contiguous slice of the listed steps of
//                  the host region, then of the pool: list entries and
//                  undefined bytes
//   k_sidx_scan    one block: the blocks' offsets, the totals, validity
//   k_sidx_fill    block b writes its entries in chunk order (a block with
//                  none returns at once)
//   k_sidx_query   one lane per record: answers the records of a check
//                  without propagation whose spaces are indexed, and takes
//                  their units out of the scan
//   k_sidx_rows    one wave per pitched 2D record whose rows follow row 0:
//                  the same, with the list entries of its span mapped onto
//                  its rows
#include <hip/hip_runtime.h>

#include "xc_internal.h"

namespace xc {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <typename T> using gcptr = const __attribute__((address_space(1))) T *;

constexpr int kT = 256;
constexpr uint32_t kPer = 16;                          // chunks per thread per step
constexpr uint64_t kStep = (uint64_t)kT * kPer;        // chunks per block per step
static_assert(kStep * 16 == (1ull << kIdxStepShift), "a step is the marks' unit");
constexpr uint32_t kMarkT = 1024;                      // threads of the marking kernels
constexpr uint64_t kMarkBlock = 16ull * kMarkT;        // marks per block of them (16 per thread)

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

// one shadow space as the kernels read it: V bytes (16-byte aligned), A bits
// as 16-bit words (none for the pool), length in bytes
struct Space {
    const uint8_t *v;
    const uint16_t *a16;
    uint64_t len;
};

__device__ __forceinline__ Space space_of(uint32_t space, const DevState *st)
{
    if (space == 0) return Space{st->region.v, st->region.a16, st->region.hl};
    return Space{reinterpret_cast<const uint8_t *>(st->pool), nullptr, st->pool_len};
}

__device__ __forceinline__ Space space_of(const ShadowIndex &x, const DevState *st) { return space_of(x.space, st); }

__device__ __forceinline__ uint64_t space_chunks(const Space &S) { return (S.len + 15) >> 4; }

__device__ __forceinline__ uint64_t space_steps(const Space &S) { return (space_chunks(S) + kStep - 1) / kStep; }

// the index is built for this batch: a space whose steps fit the step list,
// and enough of the batch's bytes in it
__device__ __forceinline__ bool worth(const ShadowIndex &x, const Space &S)
{
    return S.len > 0 && space_steps(S) <= x.steps_cap && (x.ratio == 0 || x.state[0] / x.ratio >= S.len);
}

// positions [p0, p1) of the step list that block b works
__device__ __forceinline__ void block_slice(const ShadowIndex &x, uint32_t b, uint64_t *p0, uint64_t *p1)
{
    const uint64_t m = x.state[kIdxSteps];
    const uint64_t per = (m + x.grid - 1) / x.grid;
    *p0 = (uint64_t)b * per < m ? (uint64_t)b * per : m;
    *p1 = *p0 + per < m ? *p0 + per : m;
}

// undefined (V != 0, A = 1) and unaddressable (A = 0) bytes of chunk c < the
// space's chunks; bits of bytes past the space's end are clear
__device__ __forceinline__ void chunk_faults(const Space &S, uint64_t c, uint32_t *und, uint32_t *un)
{
    const u32x4 v = *reinterpret_cast<const u32x4 *>(S.v + 16 * c);
    const uint32_t a = S.a16 ? (uint32_t)S.a16[c] : 0xFFFFu;
    const uint64_t left = S.len - 16 * c;
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

__global__ void k_sidx_reset(ShadowIndex h, ShadowIndex p)
{
    for (int k = 0; k < 8; ++k) {
        h.state[k] = 0;
        p.state[k] = 0;
    }
}

// The marks of steps m0 .. m0 + 15 as bits, for a space of `steps` steps
// (none when the index is not built; every step of the space when the batch
// asked for all of them).
__device__ __forceinline__ uint32_t marked16(const ShadowIndex &x, uint64_t m0, uint64_t steps, bool all, u32x4 v)
{
    if (m0 >= steps) return 0;
    const uint32_t live = steps - m0 >= 16 ? 0xFFFFu : (1u << (uint32_t)(steps - m0)) - 1u;
    return (all ? 0xFFFFu : nz16(v)) & live;
}

__device__ __forceinline__ uint64_t block_sum(uint64_t v)
{
    __shared__ uint64_t ws[kMarkT / 64];
    for (int k = 32; k >= 1; k >>= 1) v += __shfl_xor(v, k);
    if ((threadIdx.x & 63u) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    uint64_t all = 0;
    for (uint32_t q = 0; q < kMarkT / 64; ++q) all += ws[q];
    __syncthreads();   // ws is reused by the next call
    return all;
}

__device__ __forceinline__ u32x4 load_marks(const ShadowIndex &x, uint64_t m0)
{
    return *reinterpret_cast<const u32x4 *>(x.smark + m0);
}

// marked steps among block b's kMarkBlock marks
__global__ void __launch_bounds__(kMarkT) k_sidx_mark_count(ShadowIndex x, const DevState *stp)
{
    const Space S = space_of(x, stp);
    const uint64_t steps = worth(x, S) ? space_steps(S) : 0;
    const uint64_t m0 = (uint64_t)blockIdx.x * kMarkBlock + 16ull * threadIdx.x;
    const bool all = x.state[kIdxAll] != 0;
    const uint32_t bits = m0 < steps ? marked16(x, m0, steps, all, all ? u32x4{0, 0, 0, 0} : load_marks(x, m0)) : 0u;
    const uint64_t n = block_sum((uint64_t)__builtin_popcount(bits));
    if (threadIdx.x == 0) x.mcnt[blockIdx.x] = n;
}

// Block b lists its marked steps after those of the blocks before it and
// clears its marks (all of them, listed or not); block 0 writes the list's
// length.  Each block adds the bytes the counting pass will read for its steps.
__global__ void __launch_bounds__(kMarkT) k_sidx_mark_list(ShadowIndex x, const DevState *stp)
{
    __shared__ uint64_t ws[kMarkT / 64];
    const Space S = space_of(x, stp);
    const uint64_t steps = worth(x, S) ? space_steps(S) : 0;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
    uint64_t before = 0, total = 0;
    for (uint32_t k = tid; k < gridDim.x; k += kMarkT) {
        const uint64_t c = x.mcnt[k];
        total += c;
        before += k < blockIdx.x ? c : 0;
    }
    before = block_sum(before);
    total = block_sum(total);
    const uint64_t m0 = (uint64_t)blockIdx.x * kMarkBlock + 16ull * tid;
    const u32x4 v = load_marks(x, m0);
    const uint32_t bits = marked16(x, m0, steps, x.state[kIdxAll] != 0, v);
    if (v.x | v.y | v.z | v.w) *reinterpret_cast<u32x4 *>(x.smark + m0) = u32x4{0, 0, 0, 0};
    // block exclusive scan of the threads' marked steps
    const uint64_t n = (uint64_t)__builtin_popcount(bits);
    uint64_t inc = n;
    for (uint32_t d = 1; d < 64u; d <<= 1) {
        const uint64_t y = __shfl_up(inc, d);
        if (lane >= d) inc += y;
    }
    if (lane == 63u) ws[w] = inc;
    __syncthreads();
    uint64_t off = before;
    for (uint32_t q = 0; q < w; ++q) off += ws[q];
    off += inc - n;
    // the chunks the counting pass reads for these steps (the space's last step may be short)
    const uint64_t nch = space_chunks(S);
    uint64_t chunks = 0;
    for (uint32_t b = bits; b; b &= b - 1u) {
        const uint64_t st = m0 + (uint64_t)__builtin_ctz(b);
        x.slist[off++] = (uint32_t)st;
        chunks += st * kStep + kStep <= nch ? kStep : nch - st * kStep;
    }
    chunks = block_sum(chunks);
    if (tid == 0) {
        if (chunks) atomicAdd((unsigned long long *)x.read, (unsigned long long)(chunks * (x.space == 0 ? 18u : 16u)));
        if (blockIdx.x == 0) x.state[kIdxSteps] = total;
    }
}

// The counting pass of one index over block b's slice of its listed steps
// (nothing when the index is not built).  A step's 16 chunks per thread are
// loaded back to back (non-temporal: each byte is read once), then examined;
// each wave flags the listed steps where it met a faulty chunk, so that the
// fill reads only those.  The steps of the slice are read from the list 64 at
// a time, one per lane.
__device__ __forceinline__ void count_slice(const ShadowIndex &x, const Space &S)
{
    if (!worth(x, S)) return;
    const bool has_a = S.a16 != nullptr;   // the host region's A bits
    uint64_t p0, p1;
    block_slice(x, blockIdx.x, &p0, &p1);
    const uint64_t nch = space_chunks(S);
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const gcptr<u32x4> vp = reinterpret_cast<gcptr<u32x4>>(reinterpret_cast<uint64_t>(S.v));
    uint64_t c3[3] = {0, 0, 0};
    for (uint64_t g = p0; g < p1; g += 64) {
        const uint32_t mine = g + lane < p1 ? x.slist[g + lane] : 0u;
        const uint32_t ng = p1 - g < 64 ? (uint32_t)(p1 - g) : 64u;
        for (uint32_t k = 0; k < ng; ++k) {
            const uint64_t base = (uint64_t)__builtin_amdgcn_readlane((int)mine, (int)k) * kStep;
            const uint64_t hi = base + kStep < nch ? base + kStep : nch;
            u32x4 v[kPer];
            uint32_t a[kPer];
            if (base + kStep <= hi) {
#pragma unroll
                for (uint32_t j = 0; j < kPer; ++j) v[j] = __builtin_nontemporal_load(vp + base + (uint64_t)j * kT + threadIdx.x);
#pragma unroll
                for (uint32_t j = 0; j < kPer; ++j) a[j] = has_a ? (uint32_t)S.a16[base + (uint64_t)j * kT + threadIdx.x] : 0xFFFFu;
            } else {
#pragma unroll
                for (uint32_t j = 0; j < kPer; ++j) {
                    const uint64_t c = base + (uint64_t)j * kT + threadIdx.x;
                    v[j] = u32x4{0u, 0u, 0u, 0u};
                    a[j] = 0xFFFFu;
                    if (c < hi) {
                        v[j] = __builtin_nontemporal_load(vp + c);
                        if (has_a) a[j] = S.a16[c];
                    }
                }
            }
            // almost every chunk is clean (V all 0, A all 1): the lane's step is
            // examined chunk by chunk only when it is not, or when it holds the
            // space's end (bytes past it must not count)
            uint32_t orv = 0, anda = 0xFFFFu;
#pragma unroll
            for (uint32_t j = 0; j < kPer; ++j) {
                orv |= v[j].x | v[j].y | v[j].z | v[j].w;
                anda &= a[j];
            }
            const bool edge = base + kStep > hi || ((S.len & 15u) && base + kStep >= nch);
            uint32_t any = 0;
            if (orv != 0u || anda != 0xFFFFu || edge) {
#pragma unroll
                for (uint32_t j = 0; j < kPer; ++j) {
                    const uint64_t c = base + (uint64_t)j * kT + threadIdx.x;
                    // bytes past the space's end (its last chunk, or none) are clear
                    const uint64_t left = c < hi ? S.len - 16 * c : 0;
                    const uint32_t live = left < 16 ? (1u << left) - 1u : 0xFFFFu;
                    const uint32_t und = nz16(v[j]) & a[j] & live, un = ~a[j] & live;
                    c3[0] += und ? 1u : 0u;
                    c3[1] += un ? 1u : 0u;
                    c3[2] += (uint32_t)__builtin_popcount(und);
                    any |= und | un;
                }
            }
            const uint64_t seen = __ballot(any != 0);
            if (lane == 0) x.sflag[4 * (g + k) + wave] = seen ? 1u : 0u;
        }
    }
    uint64_t ex[3], tot[3];
    block_scan3(c3, ex, tot);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) x.bcnt[3 * blockIdx.x + k] = tot[k];
}

// Both indexes' counting passes in one launch: each block counts its slice of
// the host region's listed steps, then its slice of the pool's, so that the
// shorter pass leaves no tail of its own (both indexes have the same grid).
__global__ void __launch_bounds__(kT) k_sidx_count(ShadowIndex h, ShadowIndex p, const DevState *stp)
{
#pragma nounroll
    for (uint32_t k = 0; k < 2; ++k) count_slice(k ? p : h, space_of(k, stp));
}

// offsets of the blocks' entries into [3 grid, 6 grid) of bcnt
__global__ void __launch_bounds__(1024) k_sidx_scan(ShadowIndex x, const DevState *stp)
{
    __shared__ uint64_t ws[16][3];
    const Space S = space_of(x, stp);
    if (!worth(x, S)) {
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
    if (tid == 0) {
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

// The entries of one step of block b's range, in chunk order, at the running
// offsets ou / on / op: here thread t takes the step's chunks 16 t .. 16 t + 15
// (consecutive, so that one block scan of the threads' counts orders them).
__device__ __forceinline__ void fill_step(const ShadowIndex &x, const Space &S, uint64_t base, uint64_t hi,
                                          uint64_t &ou, uint64_t &on, uint64_t &op)
{
    const uint64_t c0 = base + (uint64_t)threadIdx.x * kPer;
    uint32_t und[kPer], un[kPer];
    uint64_t v[3] = {0, 0, 0};
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
        und[j] = un[j] = 0;
        if (c0 + j < hi) chunk_faults(S, c0 + j, &und[j], &un[j]);
        v[0] += und[j] ? 1u : 0u;
        v[1] += un[j] ? 1u : 0u;
        v[2] += (uint64_t)__builtin_popcount(und[j]);
    }
    uint64_t ex[3], tot[3];
    block_scan3(v, ex, tot);
    uint64_t iu = ou + ex[0], in = on + ex[1], ip = op + ex[2];
#pragma unroll
    for (uint32_t j = 0; j < kPer; ++j) {
        if (und[j]) {
            x.uchunk[iu] = c0 + j;
            x.umask[iu] = und[j];
            x.ucum[iu] = ip;
            ++iu;
            ip += (uint64_t)__builtin_popcount(und[j]);
        }
        if (un[j]) {
            x.nchunk[in] = c0 + j;
            x.nmask[in] = un[j];
            ++in;
        }
    }
    ou += tot[0];
    on += tot[1];
    op += tot[2];
}

// The block reads the flags of its slice 256 steps at a time, one per
// thread, lists the flagged ones in order, and fills only those.
__global__ void __launch_bounds__(kT) k_sidx_fill(ShadowIndex x, const DevState *stp)
{
    __shared__ uint32_t list[kT];
    __shared__ uint32_t nlist;
    if (!x.state[1]) return;
    const Space S = space_of(x, stp);
    const uint32_t b = blockIdx.x;
    if (x.bcnt[3 * b] == 0 && x.bcnt[3 * b + 1] == 0) return;
    uint64_t p0, p1;
    block_slice(x, b, &p0, &p1);
    const uint64_t nch = space_chunks(S);
    uint64_t ou = x.bcnt[3 * (x.grid + b)], on = x.bcnt[3 * (x.grid + b) + 1], op = x.bcnt[3 * (x.grid + b) + 2];
    for (uint64_t g0 = p0; g0 < p1; g0 += kT) {
        const uint64_t g = g0 + threadIdx.x;
        const uint32_t f = g < p1 && *reinterpret_cast<const uint32_t *>(x.sflag + 4 * g) != 0;
        uint64_t v[3] = {f, 0, 0};
        uint64_t ex[3], tot[3];
        block_scan3(v, ex, tot);
        if (f) list[ex[0]] = (uint32_t)threadIdx.x;
        if (threadIdx.x == 0) nlist = (uint32_t)tot[0];
        __syncthreads();
        const uint32_t n = nlist;
        for (uint32_t k = 0; k < n; ++k) {
            const uint64_t base = (uint64_t)x.slist[g0 + list[k]] * kStep;
            fill_step(x, S, base, base + kStep < nch ? base + kStep : nch, ou, on, op);
        }
        __syncthreads();   // list and nlist are rewritten next
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

// Facts about space offsets [ra, rb) (ra < rb): bytes [ra, rb) of chunk c
// are the bits of range_mask(c).
struct Range {
    uint64_t ca, cb;
    uint32_t lo_bit, hi_bit;
    __device__ Range(uint64_t ra, uint64_t rb)
        : ca(ra >> 4), cb((rb - 1) >> 4), lo_bit((uint32_t)(ra & 15u)), hi_bit((uint32_t)((rb - 1) & 15u)) {}
    __device__ uint32_t mask(uint64_t c) const
    {
        uint32_t m = 0xFFFFu;
        if (c == ca) m &= (0xFFFFu << lo_bit) & 0xFFFFu;
        if (c == cb) m &= (2u << hi_bit) - 1u;
        return m;
    }
};

// first faulty byte of the range among list entries [i0, i1) (space offset,
// or ~0): only the first two entries can hold it, since every entry's mask
// is non-zero and only the edge chunks are cut
__device__ __forceinline__ uint64_t first_in(const uint64_t *chunk, const uint32_t *mask, uint64_t i0, uint64_t i1,
                                             const Range &g)
{
    for (uint64_t i = i0; i < i1 && i < i0 + 2; ++i) {
        const uint32_t bits = mask[i] & g.mask(chunk[i]);
        if (bits) return 16 * chunk[i] + (uint64_t)__builtin_ctz(bits);
    }
    return ~0ull;
}

// undefined bytes of the range and the first one (space offset, or ~0)
// A list's chunk indices with every stride-th of them (samples) in LDS, for a
// two-level search: the samples first, then at most stride - 1 entries in
// global memory.
constexpr uint32_t kSamp = 256;   // samples per list

struct Sampled {
    const uint64_t *chunk;
    uint64_t n, stride, ns;
    const uint64_t *s;   // LDS: chunk[i * stride], i < ns
};

// the block fills s (kSamp entries) for a list of n entries (none when the
// index is not valid); every thread of the block calls it
__device__ __forceinline__ Sampled sample_list(uint64_t *s, const uint64_t *chunk, uint64_t n, bool valid)
{
    if (!valid) n = 0;
    const uint64_t st = n <= kSamp ? 1 : (n + kSamp - 1) / kSamp;
    const uint64_t m = (n + st - 1) / st;
    for (uint64_t i = threadIdx.x; i < m; i += kT) s[i] = chunk[i * st];
    return Sampled{chunk, n, st, m, s};
}

// lower_bound over the sampled list
__device__ __forceinline__ uint64_t lower_bound(const Sampled &x, uint64_t k)
{
    uint64_t lo = 0, hi = x.ns;   // the first sample >= k
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (x.s[mid] < k) lo = mid + 1; else hi = mid;
    }
    // the entries after sample lo - 1 (< k) up to sample lo (>= k), or the list's end
    const uint64_t a = lo == 0 ? 0 : (lo - 1) * x.stride + 1, b = lo < x.ns ? lo * x.stride : x.n;
    return a + lower_bound(x.chunk + a, b - a, k);
}

__device__ __forceinline__ uint64_t undef_in(const ShadowIndex &x, const Sampled &su, const Range &g, uint64_t *first)
{
    const uint64_t i0 = lower_bound(su, g.ca), i1 = lower_bound(su, g.cb + 1);
    uint64_t n = x.ucum[i1] - x.ucum[i0];
    if (i1 > i0) {
        // the edge chunks' bytes outside the range
        if (x.uchunk[i0] == g.ca) n -= (uint64_t)__builtin_popcount(x.umask[i0] & ~(0xFFFFu << g.lo_bit) & 0xFFFFu);
        if (x.uchunk[i1 - 1] == g.cb) n -= (uint64_t)__builtin_popcount(x.umask[i1 - 1] & ~((2u << g.hi_bit) - 1u));
    }
    *first = first_in(x.uchunk, x.umask, i0, i1, g);
    return n;
}

// the first unaddressable byte of the range (space offset, or ~0)
__device__ __forceinline__ uint64_t unaddr_in(const ShadowIndex &x, const Sampled &sn, const Range &g)
{
    const uint64_t j0 = lower_bound(sn, g.ca), j1 = lower_bound(sn, g.cb + 1);
    return first_in(x.nchunk, x.nmask, j0, j1, g);
}

__device__ __forceinline__ void take_first(uint64_t *first, uint64_t off, int64_t off0)
{
    const uint64_t i = (uint64_t)((int64_t)off - off0);   // record byte index of space offset off
    *first = i < *first ? i : *first;
}

// With `pitch`, the positions are pitched 2D records: only those worked as
// one transfer (kRowsContig, whose descriptor is that transfer's) are
// answered, and their units per row go to 0.
__global__ void __launch_bounds__(kT) k_sidx_query(BatchArgs a, ShadowIndex h, ShadowIndex p, uint64_t *wbsum,
                                                   Pitch *pitch)
{
    __shared__ uint64_t samp[3][kSamp];
    // the lists' samples: the host region's undefined and unaddressable
    // chunks, the pool's undefined chunks
    const Sampled hu = sample_list(samp[0], h.uchunk, h.state[2], h.state[1] != 0);
    const Sampled hn = sample_list(samp[1], h.nchunk, h.state[3], h.state[1] != 0);
    const Sampled pu = sample_list(samp[2], p.uchunk, p.state[2], p.state[1] != 0);
    __syncthreads();
    const uint64_t t = (uint64_t)blockIdx.x * kT + threadIdx.x;
    uint64_t removed = 0;
    if (a.out && t < a.count && (!pitch || pitch[t].uniform == kRowsContig)) {
        const Desc d = a.desc[t];
        const bool src_host = (d.ctl & CTL_SRC_HOST) != 0;
        const bool has_src = d.v_hi > d.v_lo;
        const bool dsta = (d.ctl & CTL_DST_A) != 0 && d.d_hi > d.d_lo;
        // a check without propagation whose spaces have a valid index
        const bool ok = (d.ctl & CTL_CHECK) && !(d.ctl & CTL_PROP) && d.units > 0 &&
                        (!has_src || (src_host ? h.state[1] : p.state[1])) && (!dsta || h.state[1]);
        if (ok) {
            cg_verdict v = a.out[t];
            uint64_t first = v.first_bad;
            if (has_src) {
                const uint32_t phi = (d.ctl >> CTL_PHI_SHIFT) & 15u;
                // space offset of the record's byte 0: host region offset, or pool offset
                const int64_t off0 = src_host ? d.a_src + (int64_t)phi
                                              : (int64_t)(d.src_sh + phi - a.st->pool);
                const Range g((uint64_t)(off0 + d.v_lo), (uint64_t)(off0 + d.v_hi));
                uint64_t fu;
                const uint64_t undef = src_host ? undef_in(h, hu, g, &fu) : undef_in(p, pu, g, &fu);
                if (undef) {
                    v.flags |= CG_SRC_UNDEF;
                    take_first(&first, fu, off0);
                }
                v.undef_bytes += undef;
                if (src_host) {
                    const uint64_t fn = unaddr_in(h, hn, g);
                    if (fn != ~0ull) {
                        v.flags |= CG_SRC_UNADDR;
                        take_first(&first, fn, off0);
                    }
                }
            }
            if (dsta) {
                const uint32_t psi = (d.ctl >> CTL_PSI_SHIFT) & 15u;
                const int64_t off0 = d.a_dst + (int64_t)psi;   // host region offset of the destination's byte 0
                const Range g((uint64_t)(off0 + d.d_lo), (uint64_t)(off0 + d.d_hi));
                const uint64_t fn = unaddr_in(h, hn, g);
                if (fn != ~0ull) {
                    v.flags |= CG_DST_UNADDR;
                    take_first(&first, fn, off0);
                }
            }
            v.first_bad = first;
            a.out[t] = v;
            a.desc[t].units = 0;
            a.weight[t] = 0;
            if (pitch) pitch[t].upr = 0;
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

// One side of a pitched record in a shadow space: byte c of row r (r < R,
// c < w) is space offset S + r q + c and byte r w + c of the record (its
// bytes are numbered row by row).  Rows may overlap (q < w), even coincide
// (q = 0): a byte then belongs to several rows.
struct RowSide {
    uint64_t S, R, q, w;
};

// the rows holding the byte at offset o = space offset - S: how many, and the
// record byte index of its first one (CG_NONE if none)
__device__ __forceinline__ void byte_rows(const RowSide &x, uint64_t o, uint64_t *n, uint64_t *first)
{
    uint64_t lo, hi;
    if (x.q == 0) {
        if (o >= x.w) return;
        lo = 0;
        hi = x.R - 1;
    } else {
        hi = o / x.q;
        if (hi > x.R - 1) hi = x.R - 1;
        lo = o < x.w ? 0 : (o - x.w) / x.q + 1;   // the first row whose end passes o
    }
    if (lo > hi) return;
    *n += hi - lo + 1;
    const uint64_t i = lo * x.w + (o - lo * x.q);
    *first = i < *first ? i : *first;
}

// bits [lo, hi) of a 16-bit mask (0 <= lo, both clamped to 16)
__device__ __forceinline__ uint32_t bit_range(uint64_t lo, uint64_t hi)
{
    if (hi > 16) hi = 16;
    if (lo >= hi) return 0;
    return ((1u << (uint32_t)hi) - 1u) & ~((1u << (uint32_t)lo) - 1u);
}

// The bytes of chunk c marked in `sel` that lie in rows of side x: how many
// (a byte counted once per row holding it) and the first one's record byte
// index.  Chunks meet at most two rows, and a byte at most one, when
// q >= max(w, 16): one division per chunk; otherwise byte by byte.
__device__ __forceinline__ void chunk_rows(const RowSide &x, uint64_t c, uint32_t sel, uint64_t *n, uint64_t *first)
{
    const uint64_t b0 = 16 * c;
    const uint32_t k0 = b0 < x.S ? (uint32_t)(x.S - b0) : 0u;   // bytes below the first row are in none
    sel &= (0xFFFFu << k0) & 0xFFFFu;
    if (!sel) return;
    const uint64_t o0 = b0 + k0 - x.S;   // offset of byte k0
    if (x.q >= 16 && x.q >= x.w) {
        const uint64_t r = o0 / x.q, m = o0 - r * x.q;
        // bytes k0 + j: row r for m + j < q, row r + 1 after
        uint32_t in = 0;
        if (r < x.R && m < x.w) in |= bit_range(k0, k0 + (x.w - m));
        if (r + 1 < x.R && x.q - m < 16) in |= bit_range(k0 + (x.q - m), k0 + (x.q - m) + x.w);
        const uint32_t hit = sel & in;
        if (!hit) return;
        *n += (uint64_t)__builtin_popcount(hit);
        const uint64_t j = (uint64_t)__builtin_ctz(hit) - k0;
        const uint64_t i = m + j < x.q ? r * x.w + m + j : (r + 1) * x.w + (m + j - x.q);
        *first = i < *first ? i : *first;
        return;
    }
    for (uint32_t bits = sel; bits; bits &= bits - 1u) byte_rows(x, o0 + ((uint64_t)__builtin_ctz(bits) - k0), n, first);
}

// the list entries [i0, i1) against side x, one lane per entry
__device__ __forceinline__ void walk_rows(const uint64_t *chunk, const uint32_t *mask, uint64_t i0, uint64_t i1,
                                          const RowSide &x, uint32_t lane, uint64_t *n, uint64_t *first)
{
    for (uint64_t i = i0 + lane; i < i1; i += 64) chunk_rows(x, chunk[i], mask[i], n, first);
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v)
{
    for (int k = 32; k >= 1; k >>= 1) v += __shfl_xor(v, k);
    return v;
}

__device__ __forceinline__ uint64_t wave_min(uint64_t v)
{
    for (int k = 32; k >= 1; k >>= 1) {
        const uint64_t o = __shfl_xor(v, k);
        v = o < v ? o : v;
    }
    return v;
}

// Pitched positions whose rows follow row 0 (kRowsUniform, kRowsStep: every
// row whole inside row 0's allocation or the host region) in a check without
// propagation, one wave per position.  The list entries between the first
// row's start and the last row's end are mapped onto the rows: undefined
// bytes counted once per row holding them, the first faulty byte by the
// record's row-by-row numbering.  A position whose spaces lack a valid index,
// or whose span holds more entries than a scan of its rows would read
// chunks (and more than 4,096), is left to the scan.
__global__ void __launch_bounds__(kT) k_sidx_rows(BatchArgs a, ShadowIndex h, ShadowIndex p, Pitch *pitch)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t t = (uint64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
    if (!a.out || t >= a.count) return;
    const Pitch P = pitch[t];
    if (P.uniform != kRowsUniform && P.uniform != kRowsStep) return;
    const Desc d = a.desc[t];
    const bool src_host = (d.ctl & CTL_SRC_HOST) != 0;
    const bool dsta = (d.ctl & CTL_DST_A) != 0 && d.d_hi > d.d_lo;
    const int64_t w = (int64_t)P.width;
    // row 0 is valid whole on both sides (its verdict has no flags)
    const bool ok = (d.ctl & CTL_CHECK) && !(d.ctl & CTL_PROP) && d.units > 0 && P.rows > 0 && d.v_lo == 0 &&
                    d.v_hi == w && (!dsta || (d.d_lo == 0 && d.d_hi == w)) &&
                    (src_host ? h.state[1] : p.state[1]) && (!dsta || h.state[1]);
    if (!ok) return;
    const ShadowIndex &xs = src_host ? h : p;
    const uint32_t phi = (d.ctl >> CTL_PHI_SHIFT) & 15u, psi = (d.ctl >> CTL_PSI_SHIFT) & 15u;
    const RowSide rs{src_host ? (uint64_t)(d.a_src + (int64_t)phi) : d.src_sh + phi - a.st->pool, P.rows, P.spitch,
                     P.width};
    const RowSide rd{(uint64_t)(d.a_dst + (int64_t)psi), P.rows, P.dpitch, P.width};
    // the chunks of each side's span, first row to last
    const uint64_t sa = rs.S >> 4, sb = (rs.S + (rs.R - 1) * rs.q + rs.w - 1) >> 4;
    const uint64_t da = rd.S >> 4, db = (rd.S + (rd.R - 1) * rd.q + rd.w - 1) >> 4;
    // the six list bounds, one lane each: undefined entries of the source span,
    // unaddressable ones of the host source's and of the host destination's
    uint64_t bound = 0;
    if (lane < 2) bound = lower_bound(xs.uchunk, xs.state[2], lane == 0 ? sa : sb + 1);
    else if (lane < 4 && src_host) bound = lower_bound(h.nchunk, h.state[3], lane == 2 ? sa : sb + 1);
    else if (lane >= 4 && lane < 6 && dsta) bound = lower_bound(h.nchunk, h.state[3], lane == 4 ? da : db + 1);
    const uint64_t i0 = __shfl(bound, 0), i1 = __shfl(bound, 1), j0 = __shfl(bound, 2), j1 = __shfl(bound, 3),
                   k0 = __shfl(bound, 4), k1 = __shfl(bound, 5);
    const uint64_t entries = (i1 - i0) + (j1 - j0) + (k1 - k0);
    const uint64_t chunks = P.rows * ((P.width + 15) >> 4) * (dsta ? 2 : 1);
    if (entries > 4096 && entries > chunks) return;
    uint64_t undef = 0, fu = CG_NONE, fs = CG_NONE, fd = CG_NONE, unused = 0;
    walk_rows(xs.uchunk, xs.umask, i0, i1, rs, lane, &undef, &fu);
    walk_rows(h.nchunk, h.nmask, j0, j1, rs, lane, &unused, &fs);
    walk_rows(h.nchunk, h.nmask, k0, k1, rd, lane, &unused, &fd);
    undef = wave_sum(undef);
    fu = wave_min(fu);
    fs = wave_min(fs);
    fd = wave_min(fd);
    if (lane == 0) {
        cg_verdict v = a.out[t];
        if (undef) v.flags |= CG_SRC_UNDEF;
        if (fs != CG_NONE) v.flags |= CG_SRC_UNADDR;
        if (fd != CG_NONE) v.flags |= CG_DST_UNADDR;
        v.undef_bytes += undef;
        uint64_t first = v.first_bad;
        first = fu < first ? fu : first;
        first = fs < first ? fs : first;
        first = fd < first ? fd : first;
        v.first_bad = first;
        a.out[t] = v;
        a.desc[t].units = 0;
        a.weight[t] = 0;
        pitch[t].upr = 0;
    }
}

}  // namespace

hipError_t launch_sidx_reset(const ShadowIndex &h, const ShadowIndex &p, hipStream_t s)
{
    hipLaunchKernelGGL(k_sidx_reset, dim3(1), dim3(1), 0, s, h, p);
    return hipGetLastError();
}

hipError_t launch_sidx_count(const ShadowIndex &h, const ShadowIndex &p, const DevState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_sidx_count, dim3(h.grid), dim3(kT), 0, s, h, p, st);
    return hipGetLastError();
}

hipError_t launch_sidx_finish(const ShadowIndex &x, const DevState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_sidx_scan, dim3(1), dim3(1024), 0, s, x, st);
    hipLaunchKernelGGL(k_sidx_fill, dim3(x.grid), dim3(kT), 0, s, x, st);
    return hipGetLastError();
}

hipError_t launch_sidx_marks(const ShadowIndex &x, const DevState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_sidx_mark_count, dim3(x.mark_grid), dim3(kMarkT), 0, s, x, st);
    hipLaunchKernelGGL(k_sidx_mark_list, dim3(x.mark_grid), dim3(kMarkT), 0, s, x, st);
    return hipGetLastError();
}

hipError_t launch_sidx_build(const ShadowIndex &h, const ShadowIndex &p, const DevState *st, hipStream_t s)
{
    hipError_t e = launch_sidx_marks(h, st, s);
    if (e == hipSuccess) e = launch_sidx_marks(p, st, s);
    if (e == hipSuccess) e = launch_sidx_count(h, p, st, s);
    if (e == hipSuccess) e = launch_sidx_finish(h, st, s);
    return e != hipSuccess ? e : launch_sidx_finish(p, st, s);
}

hipError_t launch_sidx_query(const BatchArgs &ar, const ShadowIndex &h, const ShadowIndex &p, uint64_t *wbsum,
                             hipStream_t s, Pitch *pitch)
{
    const uint64_t blocks = (ar.count + kT - 1) / kT;
    hipLaunchKernelGGL(k_sidx_query, dim3((uint32_t)blocks), dim3(kT), 0, s, ar, h, p, wbsum, pitch);
    if (pitch) {
        const uint64_t wblocks = (ar.count + kT / 64 - 1) / (kT / 64);
        hipLaunchKernelGGL(k_sidx_rows, dim3((uint32_t)wblocks), dim3(kT), 0, s, ar, h, p, pitch);
    }
    return hipGetLastError();
}

}  // namespace xc
