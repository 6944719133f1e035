// Concurrent-access join (race.hip): internal interface used by the runtime.
#pragma once

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#include "../../include/xfercheck.h"
#include "sort.h"

namespace xc {

// Device buffers of one join, sized for `cap` intervals (two per record).
// After the sorts, keys/vals hold each sorted interval's epoch and id, the
// sort's spare pair of buffers its last byte and stream, `first` its first
// byte.
struct RaceWs {
    uint64_t cap = 0;
    SortWs sort;
    uint32_t *res = nullptr;                  // per-interval partner (or none)
    uint64_t *first = nullptr;                // per sorted interval: first byte
    void *agg = nullptr;                      // per sweep tile: 4 monoid aggregates
    void *pre = nullptr;                      // per sweep tile: prefix / suffix of those
    uint32_t *flag = nullptr;                 // 0 when every epoch is sorted in LDS (per-epoch path)
};

// Grow `w` to hold `intervals` intervals (frees and reallocates; the caller
// makes sure no join using `w` is still running).
hipError_t race_reserve(RaceWs &w, uint64_t intervals);
void race_release(RaceWs &w);

// Enqueue one join of `count` records (count < 2^31) on stream `s`.
hipError_t race_launch(RaceWs &w, const cg_transfer *recs, const uint32_t *streams, const uint32_t *epochs,
                       uint64_t count, cg_race *out, hipStream_t s);

}  // namespace xc
