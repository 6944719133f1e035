// Concurrent-access join (race.hip): internal interface used by the runtime.
#pragma once

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#include "../../include/xfercheck.h"

namespace xc {

// Device buffers of one join, sized for `cap` intervals (two per record).
struct RaceWs {
    uint64_t cap = 0;
    uint64_t *keys[2] = {nullptr, nullptr};   // sort keys, ping-pong
    uint32_t *vals[2] = {nullptr, nullptr};   // interval ids, ping-pong
    uint32_t *counts = nullptr;               // per-digit, per-tile counts [256][tiles]
    uint32_t *dtot = nullptr;                 // per-digit totals [256]
    uint64_t *mask = nullptr;                 // key bits that differ between intervals
    uint64_t *parts = nullptr;                // per key-building block: its part of mask
    uint32_t *res = nullptr;                  // per-interval partner (or none)
    void *agg = nullptr;                      // per sweep tile: 4 monoid aggregates
    void *pre = nullptr;                      // per sweep tile: prefix / suffix of those
};

// Grow `w` to hold `intervals` intervals (frees and reallocates; the caller
// makes sure no join using `w` is still running).
hipError_t race_reserve(RaceWs &w, uint64_t intervals);
void race_release(RaceWs &w);

// Enqueue one join of `count` records (count < 2^31) on stream `s`.
hipError_t race_launch(RaceWs &w, const cg_transfer *recs, const uint32_t *streams, const uint32_t *epochs,
                       uint64_t count, cg_race *out, hipStream_t s);

}  // namespace xc
