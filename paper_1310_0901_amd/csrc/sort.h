// Stable radix sort of (u64 key, u32 value) pairs on the device (sort.hip),
// used by the concurrent-access join and to order the work of large check
// batches by source block (segment.hip).  Internal interface.
#pragma once

#include <stdint.h>
#include <hip/hip_runtime.h>

#include "../../include/xfercheck.h"

namespace xc {

// Work space of one sort of up to `cap` pairs.  keys[0] / vals[0] take the
// input; the sorted pairs end in keys[b] / vals[b] with b = sort_parity(mask)
// (known only on the device); the other pair of buffers is free afterwards.
struct SortWs {
    uint64_t cap = 0;
    uint64_t *keys[2] = {nullptr, nullptr};
    uint32_t *vals[2] = {nullptr, nullptr};
    uint32_t *counts = nullptr;   // per-digit, per-tile counts [256][tiles]
    uint32_t *dtot = nullptr;     // per-digit totals [256]
    uint64_t *parts = nullptr;    // per key-building block: OR of (key ^ first key)
    uint64_t *mask = nullptr;     // key bits that differ anywhere
};

constexpr int kSortKeyBlock = 256;   // keys per key-building block (one part each)

hipError_t sort_reserve(SortWs &w, uint64_t n);
void sort_release(SortWs &w);

// Sort the first pairs in keys[0] / vals[0]: n of them, or, when n_dev is
// given, the count in device memory at n_dev (at most n; read when the
// kernels run, so that a count computed on the device needs no copy back).
// parts[0 .. ceil(n / kSortKeyBlock)) must hold the key-building blocks'
// parts (0 for blocks past the keys).  Only `bytes` passes are launched:
// every key must be below 2^(8 * bytes), so that the higher bytes are all
// equal (the mask, and so the parity, then hold no bits above them).
hipError_t sort_pairs(SortWs &w, uint64_t n, hipStream_t s, const uint64_t *n_dev = nullptr, int bytes = 8);

// Only the key-bit mask of n keys (from the parts), for pairs already in
// order in keys[0] / vals[0] whose parts were cleared: no pass runs.
hipError_t sort_mask_only(SortWs &w, uint64_t n, hipStream_t s);

// lanes of the wave whose valid 8-bit digit equals this lane's (8 ballots)
__device__ __forceinline__ uint64_t match8(uint32_t d, bool valid)
{
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t y = __ballot(bit);
        m &= bit ? y : ~y;
    }
    return valid ? m : 0ull;
}

__device__ __forceinline__ uint64_t lanes_below() { return (1ull << __lane_id()) - 1ull; }

// a pass over key byte `pass` is skipped when that byte is the same in every key
__device__ __forceinline__ bool sort_pass_live(uint64_t mask, int pass) { return ((mask >> (8 * pass)) & 0xFFu) != 0; }

// which of the two buffers holds the keys before `pass` (pass 8: after the sort)
__device__ __forceinline__ int sort_parity(uint64_t mask, int pass = 8)
{
    int p = 0;
    for (int q = 0; q < pass; ++q) p ^= sort_pass_live(mask, q) ? 1 : 0;
    return p;
}

}  // namespace xc
