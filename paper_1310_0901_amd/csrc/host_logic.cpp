#include "host_logic.h"

#include "../../include/xfercheck.h"

namespace xc {

PoolAllocator::PoolAllocator(uint64_t bytes, uint64_t align) : bytes_(bytes / align * align), align_(align)
{
    if (bytes_) insert_free(0, bytes_);
}

void PoolAllocator::insert_free(uint64_t off, uint64_t len)
{
    by_off_[off] = len;
    by_len_.emplace(len, off);
}

void PoolAllocator::erase_free(std::map<uint64_t, uint64_t>::iterator it)
{
    auto range = by_len_.equal_range(it->second);
    for (auto j = range.first; j != range.second; ++j) {
        if (j->second == it->first) {
            by_len_.erase(j);
            break;
        }
    }
    by_off_.erase(it);
}

bool PoolAllocator::alloc(uint64_t size, uint64_t *off)
{
    if (size == 0) return false;
    const uint64_t need = rounded(size);
    if (need < size) return false;
    auto it = by_len_.lower_bound(need);   // smallest block that fits
    if (it == by_len_.end()) return false;
    const uint64_t boff = it->second, blen = it->first;
    by_len_.erase(it);
    by_off_.erase(boff);
    if (blen > need) insert_free(boff + need, blen - need);
    used_ += need;
    high_ = boff + need > high_ ? boff + need : high_;
    *off = boff;
    return true;
}

void PoolAllocator::release(uint64_t off, uint64_t size)
{
    uint64_t len = rounded(size);
    used_ -= len;
    auto next = by_off_.lower_bound(off);
    if (next != by_off_.end() && off + len == next->first) {
        len += next->second;
        erase_free(next);
    }
    auto prev = by_off_.lower_bound(off);
    if (prev != by_off_.begin()) {
        --prev;
        if (prev->first + prev->second == off) {
            off = prev->first;
            len += prev->second;
            erase_free(prev);
        }
    }
    insert_free(off, len);
}

int AllocTable::check_insert(uint64_t base, uint64_t size) const
{
    if (size == 0) return CG_EINVAL;
    if (base + size < base || base + size == 0) return CG_EINVAL;   // no wrap past 2^64 - 1
    auto it = m_.lower_bound(base);
    if (it != m_.end() && it->first < base + size) return CG_EOVERLAP;
    if (it != m_.begin()) {
        --it;
        if (it->first + it->second.size > base) return CG_EOVERLAP;
    }
    return CG_OK;
}

int AllocTable::erase(uint64_t base, AllocEntry *out)
{
    auto it = m_.find(base);
    if (it == m_.end()) return CG_ENOTFOUND;
    if (out) *out = it->second;
    --by_bits_[bits(it->second.size)];
    m_.erase(it);
    return CG_OK;
}

uint64_t AllocTable::size_bound() const
{
    for (int k = 64; k > 0; --k)
        if (by_bits_[k]) return k == 64 ? ~0ull : (1ull << k) - 1;
    return 0;
}

const AllocEntry *AllocTable::find(uint64_t p, uint64_t *base) const
{
    auto it = m_.upper_bound(p);
    if (it == m_.begin()) return nullptr;
    --it;
    if (p - it->first >= it->second.size) return nullptr;
    if (base) *base = it->first;
    return &it->second;
}

void AllocTable::export_sorted(uint64_t *base, uint64_t *end, uint64_t *off) const
{
    size_t i = 0;
    for (const auto &kv : m_) {
        base[i] = kv.first;
        end[i] = kv.first + kv.second.size;
        off[i] = kv.second.off;
        ++i;
    }
}

}  // namespace xc
