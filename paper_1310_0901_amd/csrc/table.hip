// Device-side update of the sorted allocation table (the per-context list of
// Sec. 2 / Fig. 2, kept sorted by base for interval lookups).  A new table
// version is the merge of the previous version, minus the bases freed since,
// plus the allocations made since; the result goes to another buffer of the
// version ring, so checks still in flight keep reading their own version.
//
//   k_merge_keep     one lane per old entry: keep flag (not freed), block-local
//                    exclusive scan of the flags, block sums
//   k_merge_sums     one block: exclusive scan of the block sums
//   k_merge_scatter  one lane per kept old entry or inserted entry: its index
//                    in the new table = kept entries before it + inserted
//                    entries before it
//   k_merge_top      every 2^shift-th base of the new table (LDS top level)
#include <hip/hip_runtime.h>

#include "xc_internal.h"

namespace xc {
namespace {

constexpr int kB = 256;

// number of entries of a[0..n) that are < x (a sorted ascending)
__device__ __forceinline__ uint64_t lower_bound(const uint64_t *a, uint64_t n, uint64_t x)
{
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ void __launch_bounds__(kB) k_merge_keep(MergeArgs m)
{
    __shared__ uint32_t wsum[kB / 64];
    const uint32_t tid = threadIdx.x, lane = __lane_id(), wid = tid >> 6;
    const uint64_t i = (uint64_t)blockIdx.x * kB + tid;
    uint32_t keep = 0;
    if (i < m.n_old) {
        const uint64_t b = m.old_base[i];
        const uint64_t k = lower_bound(m.del, m.n_del, b);
        keep = (k < m.n_del && m.del[k] == b) ? 0u : 1u;
    }
    uint32_t x = keep;
    for (uint32_t d = 1; d < 64u; d <<= 1) {
        const uint32_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63u) wsum[wid] = x;
    __syncthreads();
    uint32_t off = 0;
    for (uint32_t k = 0; k < wid; ++k) off += wsum[k];
    if (i < m.n_old) {
        m.keep[i] = (uint8_t)keep;
        m.loc[i] = off + x - keep;
    }
    if (tid == kB - 1) m.bsum[blockIdx.x] = off + x;
}

__global__ void __launch_bounds__(1024) k_merge_sums(MergeArgs m)
{
    __shared__ uint64_t wsum[16];
    const uint32_t tid = threadIdx.x, lane = __lane_id(), wid = tid >> 6;
    const uint64_t nb = (m.n_old + kB - 1) / kB;
    const uint64_t per = (nb + 1023) / 1024;
    const uint64_t b0 = tid * per, b1 = (b0 + per < nb) ? b0 + per : nb;
    uint64_t s = 0;
    for (uint64_t b = b0; b < b1; ++b) s += m.bsum[b];
    uint64_t x = s;
    for (uint32_t d = 1; d < 64u; d <<= 1) {
        const uint64_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63u) wsum[wid] = x;
    __syncthreads();
    uint64_t off = 0;
    for (uint32_t k = 0; k < wid; ++k) off += wsum[k];
    uint64_t run = off + x - s;
    for (uint64_t b = b0; b < b1; ++b) {
        m.boff[b] = run;
        run += m.bsum[b];
    }
    if (tid == 1023) m.boff[nb] = off + x;   // number of kept entries
}

// kept entries among the first j old entries (none when the old version is
// empty: then k_merge_keep and k_merge_sums do not run and boff is not written)
__device__ __forceinline__ uint64_t kept_before(const MergeArgs &m, uint64_t j)
{
    if (m.n_old == 0) return 0;
    const uint64_t nb = (m.n_old + kB - 1) / kB;
    if (j >= m.n_old) return m.boff[nb];
    return m.boff[j / kB] + m.loc[j];
}

__global__ void __launch_bounds__(kB) k_merge_scatter(MergeArgs m)
{
    const uint64_t i = (uint64_t)blockIdx.x * kB + threadIdx.x;
    if (i < m.n_old) {
        if (!m.keep[i]) return;
        const uint64_t b = m.old_base[i];
        const uint64_t pos = kept_before(m, i) + lower_bound(m.ins_base, m.n_ins, b);
        m.new_base[pos] = b;
        m.new_end[pos] = m.old_end[i];
        m.new_off[pos] = m.old_off[i];
    } else if (i < m.n_old + m.n_ins) {
        const uint64_t j = i - m.n_old;
        const uint64_t b = m.ins_base[j];
        const uint64_t pos = j + kept_before(m, lower_bound(m.old_base, m.n_old, b));
        m.new_base[pos] = b;
        m.new_end[pos] = m.ins_end[j];
        m.new_off[pos] = m.ins_off[j];
    }
}

__global__ void __launch_bounds__(kB) k_merge_top(MergeArgs m)
{
    const uint64_t k = (uint64_t)blockIdx.x * kB + threadIdx.x;
    if (k < m.ntop) m.new_top[k] = m.new_base[k << m.top_shift];
}

}  // namespace

hipError_t launch_merge(const MergeArgs &m, hipStream_t s)
{
    const uint64_t nb = (m.n_old + kB - 1) / kB;
    if (m.n_old) {
        hipLaunchKernelGGL(k_merge_keep, dim3((uint32_t)nb), dim3(kB), 0, s, m);
        hipLaunchKernelGGL(k_merge_sums, dim3(1), dim3(1024), 0, s, m);
    }
    const uint64_t tot = m.n_old + m.n_ins;
    if (tot) hipLaunchKernelGGL(k_merge_scatter, dim3((uint32_t)((tot + kB - 1) / kB)), dim3(kB), 0, s, m);
    if (m.ntop) hipLaunchKernelGGL(k_merge_top, dim3((uint32_t)((m.ntop + kB - 1) / kB)), dim3(kB), 0, s, m);
    return hipGetLastError();
}

hipError_t launch_merge_warm(hipStream_t s)
{
    MergeArgs m{};
    hipLaunchKernelGGL(k_merge_top, dim3(1), dim3(kB), 0, s, m);   // ntop = 0: loads the code only
    return hipGetLastError();
}

}  // namespace xc
