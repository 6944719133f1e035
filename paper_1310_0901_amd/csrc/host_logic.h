// Host-side bookkeeping of the transfer checker: the per-context list of live
// device allocations (Sec. 2, Fig. 2 caption: each allocation adds an entry
// {device pointer, size}; a free removes it) and the sub-allocator of the
// device shadow pool.  Plain C++, no HIP: the CPU tests build it with the
// host compiler and sanitizers.
#pragma once

#include <stdint.h>

#include <cstddef>
#include <map>

namespace xc {

// Best-fit sub-allocator over [0, bytes) with `align`-byte granularity.
class PoolAllocator {
public:
    explicit PoolAllocator(uint64_t bytes, uint64_t align = 256);
    // true and *off on success; false when no free block is large enough
    bool alloc(uint64_t size, uint64_t *off);
    // returns a block obtained from alloc(size) (merged with its free neighbours)
    void release(uint64_t off, uint64_t size);
    uint64_t used() const { return used_; }
    uint64_t capacity() const { return bytes_; }
    // end of the highest block ever handed out (no byte past it was ever used)
    uint64_t high() const { return high_; }
    uint64_t rounded(uint64_t size) const { return (size + align_ - 1) / align_ * align_; }
    size_t free_blocks() const { return by_off_.size(); }

private:
    void insert_free(uint64_t off, uint64_t len);
    void erase_free(std::map<uint64_t, uint64_t>::iterator it);
    uint64_t bytes_, align_, used_ = 0, high_ = 0;
    std::map<uint64_t, uint64_t> by_off_;            // free: offset -> length
    std::multimap<uint64_t, uint64_t> by_len_;       // free: length -> offset
};

struct AllocEntry {
    uint64_t size;
    uint64_t off;   // offset of the allocation's V bytes in the shadow pool
};

// Live allocations, disjoint, ordered by base address.
class AllocTable {
public:
    // CG_OK, CG_EINVAL (size 0 or end beyond 2^64 - 1) or CG_EOVERLAP
    int check_insert(uint64_t base, uint64_t size) const;
    void insert(uint64_t base, uint64_t size, uint64_t off)
    {
        m_[base] = AllocEntry{size, off};
        ++by_bits_[bits(size)];
    }
    // CG_OK or CG_ENOTFOUND (not the base of a live allocation)
    int erase(uint64_t base, AllocEntry *out);
    // live allocation containing p, or nullptr
    const AllocEntry *find(uint64_t p, uint64_t *base) const;
    size_t size() const { return m_.size(); }
    // sorted arrays of bases, ends and pool offsets (each size() long)
    void export_sorted(uint64_t *base, uint64_t *end, uint64_t *off) const;
    // a bound of every live allocation's size, within a factor of two:
    // 2^k - 1 for the smallest k that covers them all (0 when there is none)
    uint64_t size_bound() const;

private:
    static int bits(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }
    std::map<uint64_t, AllocEntry> m_;
    uint64_t by_bits_[65] = {};   // live allocations by the bit length of their size
};

}  // namespace xc
