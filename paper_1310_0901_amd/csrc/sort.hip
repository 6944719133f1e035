// Stable LSD radix sort of (u64 key, u32 value) pairs, 8-bit digits.  The
// key bits that differ between keys are gathered first (each key-building
// block ORs key ^ first key); a pass over a byte that is the same in every
// key is skipped on the device, and each kernel finds its input buffer from
// that mask.  A pass is count -> per-digit scan -> stable scatter: inside a
// 4,096-key tile each wave ranks its keys with 8 ballots per key, the tile is
// sorted locally through LDS and written out as contiguous runs per digit.
#include <hip/hip_runtime.h>

#include "sort.h"

namespace xc {
namespace {

constexpr int kT = 256;                          // threads per block
constexpr int kWaves = kT / 64;
constexpr int kSortTile = 4096;                  // keys per sort tile
constexpr int kWaveItems = kSortTile / kWaves;   // contiguous keys per wave
constexpr int kRounds = kWaveItems / 64;
static_assert(kT == kSortKeyBlock, "one part per block of the key kernels");

// the key bits that differ anywhere: OR of the per-block partials
__global__ __launch_bounds__(kT) void k_sort_mask(const uint64_t *parts, uint32_t nparts, uint64_t *mask)
{
    __shared__ uint64_t part[kWaves];
    uint64_t x = 0;
    for (uint32_t j = threadIdx.x; j < nparts; j += kT) x |= parts[j];
    for (int d = 32; d >= 1; d >>= 1) x |= __shfl_xor(x, d);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t y = 0;
        for (int w = 0; w < kWaves; ++w) y |= part[w];
        *mask = y;
    }
}

// ---- radix sort ----------------------------------------------------------


// keys to sort: mcap, or the count held in device memory when there is one
// (never above mcap)
__device__ __forceinline__ uint64_t sort_count_of(uint64_t mcap, const uint64_t *mdev)
{
    if (!mdev) return mcap;
    const uint64_t m = *mdev;
    return m < mcap ? m : mcap;
}

// exclusive sum over the block's threads; *total receives the block sum
__device__ uint32_t block_excl_sum(uint32_t x, uint32_t *total)
{
    __shared__ uint32_t wsum[kWaves];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = x;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d);
        if (l >= d) inc += y;
    }
    if (l == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
    for (int j = 0; j < kWaves; ++j) {
        if (j < w) off += wsum[j];
        tot += wsum[j];
    }
    __syncthreads();
    *total = tot;
    return off + inc - x;
}

// per-tile digit counts, digit-major: counts[d * tiles + tile]
__global__ __launch_bounds__(kT) void k_sort_count(const uint64_t *ka, const uint64_t *kb, uint64_t mcap,
                                                   const uint64_t *mdev, uint32_t tiles, const uint64_t *maskp,
                                                   int pass, uint32_t *counts)
{
    const uint64_t mask = *maskp;
    if (!sort_pass_live(mask, pass)) return;
    const uint64_t m = sort_count_of(mcap, mdev);
    const uint64_t *kin = sort_parity(mask, pass) ? kb : ka;
    const int shift = 8 * pass;
    __shared__ uint32_t h[kWaves][256];
    for (int j = threadIdx.x; j < kWaves * 256; j += kT) (&h[0][0])[j] = 0;
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile + (uint64_t)w * kWaveItems + l;
    uint32_t d[kRounds];
#pragma unroll
    for (int i = 0; i < kRounds; ++i) {
        const uint64_t idx = base + (uint64_t)i * 64;
        d[i] = idx < m ? (uint32_t)(kin[idx] >> shift) & 0xFFu : 0u;
    }
#pragma unroll
    for (int i = 0; i < kRounds; ++i) {
        const bool valid = base + (uint64_t)i * 64 < m;
        const uint64_t peers = match8(d[i], valid);
        if (valid && (peers & lanes_below()) == 0) h[w][d[i]] += (uint32_t)__popcll(peers);
    }
    __syncthreads();
    const int t = threadIdx.x;
    uint32_t c = 0;
    for (int j = 0; j < kWaves; ++j) c += h[j][t];
    counts[(uint64_t)t * tiles + blockIdx.x] = c;
}

// per digit (one block each): exclusive prefix of the tile counts in place,
// and the digit's total
__global__ __launch_bounds__(kT) void k_sort_scan_digits(uint32_t *counts, uint32_t tiles, uint32_t *dtot,
                                                         const uint64_t *maskp, int pass)
{
    if (!sort_pass_live(*maskp, pass)) return;
    uint32_t *row = counts + (uint64_t)blockIdx.x * tiles;
    const uint32_t per = (tiles + kT - 1) / kT;
    const uint32_t lo = min(tiles, threadIdx.x * per), hi = min(tiles, lo + per);
    uint32_t s = 0;
    for (uint32_t j = lo; j < hi; ++j) s += row[j];
    uint32_t tot;
    uint32_t run = block_excl_sum(s, &tot);
    for (uint32_t j = lo; j < hi; ++j) {
        const uint32_t c = row[j];
        row[j] = run;
        run += c;
    }
    if (threadIdx.x == 0) dtot[blockIdx.x] = tot;
}

// stable scatter of one tile: ranks within the tile, a local sort through
// LDS, then runs of equal digits written contiguously
__global__ __launch_bounds__(kT) void k_sort_scatter(uint64_t *ka, uint64_t *kb, uint32_t *va, uint32_t *vb,
                                                     uint64_t mcap, const uint64_t *mdev, uint32_t tiles,
                                                     const uint64_t *maskp, int pass, const uint32_t *counts,
                                                     const uint32_t *dtot)
{
    const uint64_t mask = *maskp;
    if (!sort_pass_live(mask, pass)) return;
    const uint64_t m = sort_count_of(mcap, mdev);
    if ((uint64_t)blockIdx.x * kSortTile >= m) return;   // a tile past the keys (the whole block leaves)
    const int par = sort_parity(mask, pass);
    const uint64_t *kin = par ? kb : ka;
    const uint32_t *vin = par ? vb : va;
    uint64_t *kout = par ? ka : kb;
    uint32_t *vout = par ? va : vb;
    const int shift = 8 * pass;

    __shared__ uint64_t skey[kSortTile];
    __shared__ uint32_t sval[kSortTile];
    __shared__ uint32_t wrun[kWaves][256];   // per wave: running count, then exclusive prefix across waves
    __shared__ uint32_t dstart[256];         // first tile-local position of each digit
    __shared__ uint32_t gbase[256];          // global position of this tile's first key of each digit

    for (int j = threadIdx.x; j < kWaves * 256; j += kT) (&wrun[0][0])[j] = 0;
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const uint64_t base = (uint64_t)blockIdx.x * kSortTile + (uint64_t)w * kWaveItems + l;
    uint64_t k[kRounds];
    uint32_t v[kRounds], pk[kRounds];
#pragma unroll
    for (int i = 0; i < kRounds; ++i) {
        const uint64_t idx = base + (uint64_t)i * 64;
        k[i] = idx < m ? kin[idx] : 0ull;
        v[i] = idx < m ? vin[idx] : 0u;
    }
#pragma unroll
    for (int i = 0; i < kRounds; ++i) {
        const bool valid = base + (uint64_t)i * 64 < m;
        const uint32_t d = (uint32_t)(k[i] >> shift) & 0xFFu;
        const uint64_t peers = match8(d, valid);
        const uint32_t rank = (uint32_t)__popcll(peers & lanes_below());
        uint32_t run = 0;
        if (valid) run = wrun[w][d];
        if (valid && rank == 0) wrun[w][d] = run + (uint32_t)__popcll(peers);
        pk[i] = valid ? (d << 16) | (run + rank) : 0xFFFFFFFFu;
    }
    __syncthreads();
    const int t = threadIdx.x;
    uint32_t acc = 0;
    for (int j = 0; j < kWaves; ++j) {
        const uint32_t c = wrun[j][t];
        wrun[j][t] = acc;
        acc += c;
    }
    uint32_t unused;
    dstart[t] = block_excl_sum(acc, &unused);
    gbase[t] = block_excl_sum(dtot[t], &unused) + counts[(uint64_t)t * tiles + blockIdx.x];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kRounds; ++i) {
        if (pk[i] != 0xFFFFFFFFu) {
            const uint32_t d = pk[i] >> 16;
            const uint32_t pos = dstart[d] + wrun[w][d] + (pk[i] & 0xFFFFu);
            skey[pos] = k[i];
            sval[pos] = v[i];
        }
    }
    __syncthreads();
    const uint64_t left = m - (uint64_t)blockIdx.x * kSortTile;
    const uint32_t nvalid = left < (uint64_t)kSortTile ? (uint32_t)left : (uint32_t)kSortTile;
    for (uint32_t j = t; j < nvalid; j += kT) {
        const uint64_t key = skey[j];
        const uint32_t d = (uint32_t)(key >> shift) & 0xFFu;
        const uint64_t g = (uint64_t)gbase[d] + (j - dstart[d]);
        if (g < m) {
            kout[g] = key;
            vout[g] = sval[j];
        }
    }
}


uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

}  // namespace

hipError_t sort_reserve(SortWs &w, uint64_t n)
{
    if (n <= w.cap) return hipSuccess;
    sort_release(w);
    const uint64_t tiles = ceil_div(n, kSortTile);
    hipError_t e = hipSuccess;
    auto get = [&](void **p, uint64_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, bytes ? bytes : 8);
    };
    for (int i = 0; i < 2; ++i) {
        get((void **)&w.keys[i], n * sizeof(uint64_t));
        get((void **)&w.vals[i], n * sizeof(uint32_t));
    }
    get((void **)&w.counts, 256 * tiles * sizeof(uint32_t));
    get((void **)&w.dtot, 256 * sizeof(uint32_t));
    get((void **)&w.parts, ceil_div(n, kT) * sizeof(uint64_t));
    get((void **)&w.mask, sizeof(uint64_t));
    if (e != hipSuccess) {
        sort_release(w);
        return e;
    }
    w.cap = n;
    return hipSuccess;
}

void sort_release(SortWs &w)
{
    void *ps[] = {w.keys[0], w.keys[1], w.vals[0], w.vals[1], w.counts, w.dtot, w.parts, w.mask};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    w = SortWs{};
}

hipError_t sort_mask_only(SortWs &w, uint64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sort_mask, dim3(1), dim3(kT), 0, s, w.parts, (uint32_t)ceil_div(n, kT), w.mask);
    return hipGetLastError();
}

hipError_t sort_pairs(SortWs &w, uint64_t n, hipStream_t s, const uint64_t *n_dev, int bytes)
{
    if (n == 0) return hipSuccess;
    if (bytes < 1 || bytes > 8) return hipErrorInvalidValue;
    const uint32_t tiles = (uint32_t)ceil_div(n, kSortTile);
    hipLaunchKernelGGL(k_sort_mask, dim3(1), dim3(kT), 0, s, w.parts, (uint32_t)ceil_div(n, kT), w.mask);
    for (int pass = 0; pass < bytes; ++pass) {
        hipLaunchKernelGGL(k_sort_count, dim3(tiles), dim3(kT), 0, s, w.keys[0], w.keys[1], n, n_dev, tiles, w.mask,
                           pass, w.counts);
        hipLaunchKernelGGL(k_sort_scan_digits, dim3(256), dim3(kT), 0, s, w.counts, tiles, w.dtot, w.mask, pass);
        hipLaunchKernelGGL(k_sort_scatter, dim3(tiles), dim3(kT), 0, s, w.keys[0], w.keys[1], w.vals[0], w.vals[1], n,
                           n_dev, tiles, w.mask, pass, w.counts, w.dtot);
    }
    return hipGetLastError();
}

}  // namespace xc
