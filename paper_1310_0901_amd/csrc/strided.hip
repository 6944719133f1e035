// Pitched 2D copies (the strided copies of the footnote to Sec. 2's error
// list) on the device.  Row r of a record reads [src + r*spitch, + width) and
// writes [dst + r*dpitch, + width).  The rows are expanded into transfer
// records, checked as one batch by the batched path, and folded back: the
// bytes of a 2D copy are numbered row by row, so its verdict is the OR of the
// rows' flags, the smallest r*width + first_bad_r, the sum of undefined bytes
// and the first row's avail.
//
//   k2d_count   per block: exclusive scan of the records' row counts, and the
//               rows of records with short rows (a launch-shape choice)
//   k2d_sums    one block: exclusive scan of the block sums; the totals
//   k2d_add     block offsets added: first row of every record
//   k2d_expand  one lane per row: its record (binary search in the first
//               rows), its transfer record
//   k2d_init    one lane per record: the verdict before any row is folded
//   k2d_fold    one lane per row: rows with findings fold into their record
//               with atomics (clean rows touch nothing)
#include <hip/hip_runtime.h>

#include "xc_internal.h"

namespace xc {
namespace {

constexpr int kT = 256;

constexpr uint64_t kShortRow = 16384;   // bytes: rows this wide or less are short

// a record's rows, at most 2^32 (the sum over 2^31 records cannot wrap, and a
// batch with a record this tall is refused for too many rows)
__device__ __forceinline__ uint64_t rows_of(const cg_transfer2d &r)
{
    return r.width ? (r.rows < (1ull << 32) ? r.rows : (1ull << 32)) : 0;
}

// block sum of x over the kT threads
__device__ __forceinline__ uint64_t block_sum(uint64_t x)
{
    __shared__ uint64_t part[kT / 64];
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
    __syncthreads();
    uint64_t t = 0;
    for (int k = 0; k < kT / 64; ++k) t += part[k];
    return t;
}

__global__ void __launch_bounds__(kT) k2d_count(const cg_transfer2d *recs, uint64_t count, uint64_t *first,
                                                uint64_t *bsum, uint64_t *bshort)
{
    __shared__ uint64_t wsum[kT / 64];
    const uint64_t t = (uint64_t)blockIdx.x * kT + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const cg_transfer2d r = t < count ? recs[t] : cg_transfer2d{};
    const uint64_t c = t < count ? rows_of(r) : 0;
    const uint64_t sh = block_sum(r.width <= kShortRow ? c : 0);
    if (threadIdx.x == 0) bshort[blockIdx.x] = sh;
    uint64_t x = c;
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint64_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint64_t off = 0;
    for (uint32_t k = 0; k < w; ++k) off += wsum[k];
    if (t < count) first[t] = off + x - c;
    if (threadIdx.x == kT - 1) bsum[blockIdx.x] = off + x;
}

__global__ void __launch_bounds__(1024) k2d_sums(uint64_t *bsum, const uint64_t *bshort, uint64_t nb, uint64_t *total)
{
    __shared__ uint64_t wsum[16], ssum[16];
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint64_t per = (nb + 1023) / 1024;
    const uint64_t b0 = tid * per < nb ? tid * per : nb, b1 = b0 + per < nb ? b0 + per : nb;
    uint64_t s = 0, sh = 0;
    for (uint64_t b = b0; b < b1; ++b) {
        s += bsum[b];
        sh += bshort[b];
    }
    for (int d = 32; d >= 1; d >>= 1) sh += __shfl_xor(sh, d);
    if (lane == 0) ssum[w] = sh;
    uint64_t x = s;
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const uint64_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint64_t off = 0;
    for (uint32_t k = 0; k < w; ++k) off += wsum[k];
    uint64_t run = off + x - s;
    for (uint64_t b = b0; b < b1; ++b) {
        const uint64_t v = bsum[b];
        bsum[b] = run;
        run += v;
    }
    if (tid == 1023) {
        total[0] = off + x;
        uint64_t t = 0;
        for (int k = 0; k < 16; ++k) t += ssum[k];
        total[1] = t;   // rows of records with short rows
    }
}

__global__ void __launch_bounds__(kT) k2d_add(uint64_t *first, const uint64_t *boff, uint64_t count)
{
    const uint64_t t = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (t < count) first[t] += boff[blockIdx.x];
}

// the record holding row q: the largest t with first[t] <= q (records with no
// rows before it share its first row; the ones after it start past q)
__device__ __forceinline__ uint64_t record_of(const uint64_t *first, uint64_t count, uint64_t q)
{
    uint64_t lo = 0, hi = count - 1;
    while (lo < hi) {
        const uint64_t mid = (lo + hi + 1) >> 1;
        if (first[mid] <= q) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(kT) k2d_expand(const cg_transfer2d *recs, const uint64_t *first, uint64_t count,
                                                 uint64_t nrows, cg_transfer *rows, uint32_t *rec_of)
{
    const uint64_t stride = (uint64_t)gridDim.x * kT;
    for (uint64_t q = (uint64_t)blockIdx.x * kT + threadIdx.x; q < nrows; q += stride) {
        const uint64_t t = record_of(first, count, q);
        const cg_transfer2d r = recs[t];
        const uint64_t k = q - first[t];
        cg_transfer o;
        o.src = r.src + k * r.spitch;
        o.dst = r.dst + k * r.dpitch;
        o.n = r.width;
        o.kind = r.kind;
        o.reserved = 0;
        rows[q] = o;
        rec_of[q] = (uint32_t)t;
    }
}

__global__ void __launch_bounds__(kT) k2d_init(const cg_transfer2d *recs, const uint64_t *first, uint64_t count,
                                               const cg_verdict *rowv, cg_verdict *out)
{
    const uint64_t t = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (t >= count) return;
    cg_verdict v;
    v.flags = 0;
    v.reserved = 0;
    v.first_bad = CG_NONE;
    v.undef_bytes = 0;
    v.avail = rows_of(recs[t]) ? rowv[first[t]].avail : 0;
    out[t] = v;
}

__global__ void __launch_bounds__(kT) k2d_fold(const cg_transfer2d *recs, const uint64_t *first,
                                               const uint32_t *rec_of, const cg_verdict *rowv, uint64_t nrows,
                                               cg_verdict *out)
{
    const uint64_t stride = (uint64_t)gridDim.x * kT;
    for (uint64_t q = (uint64_t)blockIdx.x * kT + threadIdx.x; q < nrows; q += stride) {
        const cg_verdict v = rowv[q];
        if (v.flags == 0 && v.undef_bytes == 0) continue;
        const uint32_t t = rec_of[q];
        const uint64_t k = q - first[t];
        if (v.flags) atomicOr(&out[t].flags, v.flags);
        if (v.first_bad != CG_NONE)
            atomicMin((unsigned long long *)&out[t].first_bad,
                      (unsigned long long)(k * recs[t].width + v.first_bad));
        if (v.undef_bytes) atomicAdd((unsigned long long *)&out[t].undef_bytes, (unsigned long long)v.undef_bytes);
    }
}

uint32_t grid_for(uint64_t n, uint64_t cap)
{
    const uint64_t b = (n + kT - 1) / kT;
    return (uint32_t)(b < cap ? (b ? b : 1) : cap);
}

}  // namespace

hipError_t launch_2d_prefix(const cg_transfer2d *recs, uint64_t count, uint64_t *first, uint64_t *bsum,
                            uint64_t *bshort, uint64_t *total, hipStream_t s)
{
    const uint64_t nb = (count + kT - 1) / kT;
    hipLaunchKernelGGL(k2d_count, dim3((uint32_t)nb), dim3(kT), 0, s, recs, count, first, bsum, bshort);
    hipLaunchKernelGGL(k2d_sums, dim3(1), dim3(1024), 0, s, bsum, bshort, nb, total);
    hipLaunchKernelGGL(k2d_add, dim3((uint32_t)nb), dim3(kT), 0, s, first, bsum, count);
    return hipGetLastError();
}

hipError_t launch_2d_expand(const cg_transfer2d *recs, const uint64_t *first, uint64_t count, uint64_t nrows,
                            cg_transfer *rows, uint32_t *rec_of, hipStream_t s)
{
    hipLaunchKernelGGL(k2d_expand, dim3(grid_for(nrows, 1u << 16)), dim3(kT), 0, s, recs, first, count, nrows, rows,
                       rec_of);
    return hipGetLastError();
}

hipError_t launch_2d_fold(const cg_transfer2d *recs, const uint64_t *first, uint64_t count, const uint32_t *rec_of,
                          const cg_verdict *rowv, uint64_t nrows, cg_verdict *out, hipStream_t s)
{
    hipLaunchKernelGGL(k2d_init, dim3(grid_for(count, 1ull << 32)), dim3(kT), 0, s, recs, first, count, rowv, out);
    if (nrows)
        hipLaunchKernelGGL(k2d_fold, dim3(grid_for(nrows, 1u << 16)), dim3(kT), 0, s, recs, first, rec_of, rowv,
                           nrows, out);
    return hipGetLastError();
}

}  // namespace xc
