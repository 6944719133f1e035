// Internal types shared by the HIP kernels (kernels.hip) and the host runtime
// (runtime.cpp).  Not part of the public C ABI.
#pragma once

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#include "../../include/xfercheck.h"

namespace xc {

// Per-record scan descriptor written by the classify kernel.
//
// A record's byte index i runs over [0, n).  The source side is read in
// 16-byte "chunks" aligned in shadow memory: source chunk c covers byte
// indices [16c - phi, 16c - phi + 16), destination chunk e covers
// [16e - psi, 16e - psi + 16).  One unit of work handles destination chunk
// e = e0 + k together with source chunk c = e - delta; delta is 1 when the
// source phase is behind the destination phase, so that destination chunk e
// is byte window [s, s + 16) of source chunks c and c + 1, s = (phi - psi) mod 16.
struct alignas(16) Desc {
    uint64_t src_sh;   // device address of source chunk 0 (16-byte aligned)
    uint64_t dst_sh;   // device address of destination chunk 0 (16-byte aligned)
    int64_t v_lo, v_hi;  // source bytes that are valid to read: [v_lo, v_hi)
    int64_t d_lo, d_hi;  // destination bytes inside the region / allocation
    int64_t a_src;     // A-bit index of source chunk 0 (host source only)
    int64_t a_dst;     // A-bit index of destination chunk 0 (host destination only)
    uint64_t e0;       // first unit's destination-chunk index
    uint64_t units;    // number of units
    uint32_t ctl;      // CTL_* bits, phase fields
    uint32_t pad[3];
};
static_assert(sizeof(Desc) == 96, "descriptor layout");

enum : uint32_t {
    CTL_SRC_HOST = 1u << 0,
    CTL_DST_HOST = 1u << 1,
    CTL_CHECK = 1u << 2,      // accumulate findings
    CTL_PROP = 1u << 3,       // write destination shadow
    CTL_DST_A = 1u << 4,      // scan destination A bits (host destination, checking)
    CTL_PHI_SHIFT = 8,        // 4 bits
    CTL_PSI_SHIFT = 12,       // 4 bits
    CTL_DELTA = 1u << 16,
};

// Device-resident control block of one batched check.
struct alignas(64) Ctl {
    uint64_t total_units;   // sum of max(units, 1)
    uint64_t ntiles;
    uint64_t tile_units;    // units per tile actually used
    uint32_t counter[8];    // per XCD: tiles taken from its chunk beyond the first tiles
    uint64_t pad[1];
    uint32_t lds_counter[8];  // per XCD: host-source tasks taken beyond the first ones (k_host_lds)
    uint64_t pad2[4];
};
static_assert(sizeof(Ctl) == 128, "control block layout");

struct Region {
    uint64_t hb, hl;
    const uint8_t *v;
    const uint16_t *a16;   // A bitmap viewed as 16-bit words
};

struct TableView {
    const uint64_t *base, *end, *off;
    const uint64_t *top;   // base[k << top_shift], k < ntop
    uint64_t n;
    uint32_t top_shift, ntop;
};

// Device-resident view of the context (allocation table, host region, pool);
// kernels read it through a pointer so that captured graphs stay valid when
// the table changes.
struct DevState {
    TableView table;
    Region region;
    uint64_t pool;          // device address of the shadow pool
    uint64_t size_bound;    // no live allocation is larger (within a factor of two)
    uint64_t pool_len;      // bytes of the pool ever handed out (from its start)
};
static_assert(sizeof(DevState) % 8 == 0, "uploaded in 8-byte words");

struct FillRange {
    uint64_t ptr, len;
    uint32_t val, pad;
};

constexpr int kMaxTop = 1024;        // LDS-staged top level of the table
constexpr uint64_t kMinTile = 1024;  // smallest work tile, in 16-byte units
constexpr int kClassifyBlock = 256;  // records per classify block
constexpr uint64_t kScanLimit = 1ull << 62;  // byte indices scanned per record
constexpr uint64_t kSmallUnits = 8192;       // units per block of a record in a one-launch batch (k_small)

// A pitched 2D record worked as one position (check_transfers_2d): row r is
// the transfer {src + r*spitch, dst + r*dpitch, width, kind}, its units are
// [r*upr, (r+1)*upr) of the position (upr bounds the units of any row; the
// units past a row's own are empty), and the position's Desc is row 0's.
// When `uniform` is non-zero, every row lies in row 0's allocation or in the
// host region on each side, fully valid, so row r's descriptor follows from
// row 0's by the pitches (with pitches that keep the 16-byte phases, every
// row has exactly upr units); otherwise each row is looked up and classified
// where it is worked.
struct Pitch {
    uint64_t src, dst, width, rows, spitch, dpitch, upr;
    uint32_t kind, uniform;
};

// Pitch::uniform: rows follow row 0 (kRowsUniform), and also keep its 16-byte
// phases, so that every row has row 0's units and upr is that number
// (kRowsStep); or, in a check without propagation, the rows' sources (and a
// host destination) lie back to back, so that the record is worked as one
// transfer of rows * width bytes, whose descriptor is the position's and whose
// units are upr (kRowsContig): its byte indices are the record's own.
constexpr uint32_t kRowsUniform = 1u, kRowsStep = 3u, kRowsContig = 7u;
static_assert(sizeof(Pitch) == 64, "pitched record layout");

struct BatchArgs {
    const cg_transfer *recs;
    uint64_t count;
    cg_verdict *out;        // may be null (propagation only)
    uint32_t mode;          // CG_CHECK | CG_PROPAGATE
    const DevState *st;
    Desc *desc;
    uint64_t *weight;       // units per record
    uint64_t *local;        // block-local exclusive prefix of max(units, 1)
    uint64_t *bsum;         // per classify block sums
    uint64_t *boff;         // exclusive prefix of bsum
    uint64_t *prefix;       // global exclusive prefix, count + 1 entries
    uint32_t *tile_start;   // first record of each tile
    uint64_t tiles_cap;
    Ctl *ctl;
    // when not null, position t works for record perm[t]: findings go to
    // that record's verdict (descriptors, weights and prefixes are by
    // position; the positions are source-block segments, segment.hip)
    const uint32_t *perm;
    // when not null (a check-only batch worked as segments), the host-source
    // positions [lds_meta[2], lds_meta[0]) weigh 0 in the scan kernel's
    // prefix and are worked by k_host_lds from LDS
    const uint64_t *lds_meta;
    uint32_t task_pos;   // positions per task of k_host_lds (0: its default)
    // when not null, position t is the pitched 2D record pitch[t] (desc[t] is
    // its row 0; check_transfers_2d), and findings are offset by row * width
    const Pitch *pitch;
    // when not null, k_classify adds the batch's valid bytes that a shadow
    // index would answer: [0] in the host region (host sources, host
    // destinations of device-to-host records), [1] in the shadow pool (device
    // sources); the indexes' cost test (shadowindex.hip)
    uint64_t *index_bytes[2];
    // with index_bytes: per space, a byte per step of 4,096 chunks (64 KiB of
    // V bytes), set to 1 for every step the batch's valid bytes fall in
    // (mark_cap[k] steps), so that the index's counting pass reads only those
    uint8_t *index_mark[2];
    uint64_t mark_cap[2];
};

// Index of one shadow space's faulty 16-byte chunks for a check-only batch
// (shadowindex.hip).  Space 0 is the host region (V and A bits), space 1 the
// shadow pool (V only: its addressability is the allocation table's).  The
// lists hold every chunk with an undefined byte (V != 0 where A = 1), with
// its mask and the undefined bytes of all chunks before it, and every chunk
// with an unaddressable byte (A = 0), in ascending order; a record's
// findings in that space are then two searches per list instead of a scan
// of its bytes.  Only the steps of 4,096 chunks that the batch's records
// read are listed (marked by the classify kernels) and read; the list is cut
// into `grid` contiguous slices, one per block.  state = {valid bytes of the
// batch in the space, index valid, undefined-chunk entries,
// unaddressable-chunk entries, steps listed, every step wanted, 0, 0}.
struct ShadowIndex {
    uint64_t *uchunk;   // [cap_u + 1]: entry n_u holds ~0
    uint32_t *umask;    // [cap_u]
    uint64_t *ucum;     // [cap_u + 1]: entry n_u holds the total
    uint64_t *nchunk;   // [cap_n]
    uint32_t *nmask;    // [cap_n]
    uint64_t *bcnt;     // [6 * grid]: per block entries (u, n) and undefined bytes, then their offsets
    uint64_t *state;    // [8]
    uint8_t *sflag;     // [4 * steps_cap]: wave w of listed step i (4,096 chunks) met list entries
    uint8_t *smark;     // [16384 * mark_grid]: steps the batch reads (set by the classify kernels)
    uint32_t *slist;    // [steps_cap]: the steps listed, ascending
    uint64_t *mcnt;     // [mark_grid]: marked steps per block of the marking kernels
    uint64_t *read;     // bytes the counting passes read (V, and A for the host region), accumulated
    uint64_t steps_cap; // steps of the largest space indexed (a larger one is not)
    uint64_t cap_u, cap_n;
    uint32_t grid;
    uint32_t mark_grid;
    uint32_t space;     // 0 host region, 1 shadow pool
    uint32_t ratio;     // built when the batch's valid bytes in the space reach ratio * its length
};

// ShadowIndex::state slots beyond the first four
constexpr int kIdxSteps = 4, kIdxAll = 5;
constexpr uint64_t kIdxStepShift = 16;   // a step is 2^16 bytes of V (4,096 chunks)

// Cutting a batch's records into source-block segments (segment.hip).
// rdesc / wbsum come from k_classify run over the records in their given
// order; the segments become `npos` = 3 * count positions of the batch.
struct SegArgs {
    const Desc *rdesc;      // per record
    uint64_t count;         // records (at least 1)
    uint64_t npos;          // positions provided: 3 * count
    const uint64_t *wbsum;  // k_classify's block sums of the work weights
    uint64_t *first;        // per record: first segment
    uint64_t *sbsum;        // per record block: segment sums, then their prefix
    uint32_t *srec;         // per segment: its record
    uint64_t *meta;         // [0] segments, [1] log2 of the block size, [2] first host-source position
    uint32_t min_log2;      // smallest block size, log2
    uint32_t host_last;     // host-source segments sort after the others and weigh 0: k_host_lds works them
    uint32_t key_bytes;     // 4 when every block index is below 2^31 (the host bit is then bit 31), else 8
};

// Per record of a batch worked by k_small: the findings of its blocks so
// far, and how many of its blocks have finished.  Starting state (and the
// state every call leaves): first = CG_NONE, the rest 0.
struct SmallAcc {
    uint64_t first, undef;
    uint32_t flags, done;
};
static_assert(sizeof(SmallAcc) == 24, "small-batch accumulator layout");

struct LaunchShape {
    uint32_t block, unroll, grid, nontemporal;
    uint32_t tile_units;
    uint32_t cus;   // compute units of the device
    uint32_t lds_after;   // host-source positions in a kernel of their own after the scan kernel (else side by side)
};

// Merge of a table version with the frees and allocations made since
// (table.hip).  del / ins_* are sorted by base; keep / loc / bsum / boff are
// scratch sized for n_old (boff has one extra entry: the kept count).
struct MergeArgs {
    const uint64_t *old_base, *old_end, *old_off;
    uint64_t n_old;
    const uint64_t *del;
    uint64_t n_del;
    const uint64_t *ins_base, *ins_end, *ins_off;
    uint64_t n_ins;
    uint64_t *new_base, *new_end, *new_off, *new_top;
    uint32_t top_shift, ntop;
    uint8_t *keep;
    uint32_t *loc;
    uint64_t *bsum, *boff;
};
hipError_t launch_merge(const MergeArgs &m, hipStream_t s);
hipError_t launch_merge_warm(hipStream_t s);

// kernel launchers (kernels.hip); all asynchronous on `s`
hipError_t launch_classify(const BatchArgs &a, hipStream_t s);
// one lane per pitched 2D record: row 0 classified, Pitch, weight rows * upr,
// verdict before any row is worked (check_transfers_2d)
// the shadow indexes of a check-only batch worked as segments: reset before
// k_classify, build after it, then answer the records whose every space has
// a valid index and take them out of the scan (units to 0, wbsum per
// classify block adjusted)
hipError_t launch_sidx_reset(const ShadowIndex &h, const ShadowIndex &p, hipStream_t s);
// both indexes: marks, counting pass, finish
hipError_t launch_sidx_build(const ShadowIndex &h, const ShadowIndex &p, const DevState *st, hipStream_t s);
hipError_t launch_sidx_marks(const ShadowIndex &x, const DevState *st, hipStream_t s);
hipError_t launch_sidx_count(const ShadowIndex &h, const ShadowIndex &p, const DevState *st, hipStream_t s);
hipError_t launch_sidx_finish(const ShadowIndex &x, const DevState *st, hipStream_t s);
hipError_t launch_sidx_query(const BatchArgs &ar, const ShadowIndex &h, const ShadowIndex &p, uint64_t *wbsum,
                             hipStream_t s, Pitch *pitch = nullptr);   // pitch: positions are 2D records
// the block-local prefix and block sums of max(units, 1) again, after the
// shadow indexes have answered records of a batch in its given order
hipError_t launch_reweigh(const BatchArgs &a, hipStream_t s);
hipError_t launch_classify_2d(const BatchArgs &a, const cg_transfer2d *recs2d, Pitch *pitch, hipStream_t s);
hipError_t launch_scan_sums(const BatchArgs &a, uint32_t tile_units, uint32_t waves, hipStream_t s);
hipError_t launch_prefix_tiles(const BatchArgs &a, hipStream_t s);
// the persistent scan kernel, then (a.lds_meta) the host-source positions in LDS
hipError_t launch_batched(const BatchArgs &a, const LaunchShape &sh, hipStream_t s);
hipError_t launch_plain(const BatchArgs &a, uint64_t rec, uint64_t units, const LaunchShape &sh,
                        hipStream_t s);
hipError_t launch_fill(const FillRange *ranges_dev, uint64_t k, hipStream_t s);
// `bytes` (a multiple of 8) from coherent host memory (its device address) to device memory
hipError_t launch_upload(const void *src, void *dst, uint64_t bytes, hipStream_t s);
// a batch of a.count records in one launch of a.count * bpr blocks of sh.block threads
hipError_t launch_small(const BatchArgs &a, SmallAcc *acc, uint32_t bpr, const LaunchShape &sh, hipStream_t s);
hipError_t launch_small_reset(SmallAcc *acc, uint64_t n, hipStream_t s);

// segment.hip: segments of the records described by g, sorted by source
// block, written as the positions of ap (desc, weight, local, bsum) with
// perm[p] the record of position p; `sort` holds at least g.npos pairs
struct SortWs;
hipError_t launch_segments(const SegArgs &g, SortWs &sort, const BatchArgs &ap, uint32_t *perm, hipStream_t s);
hipError_t launch_2d_prefix(const cg_transfer2d *recs, uint64_t count, uint64_t *first, uint64_t *bsum,
                            uint64_t *bshort, uint64_t *total, hipStream_t s);
hipError_t launch_2d_expand(const cg_transfer2d *recs, const uint64_t *first, uint64_t count, uint64_t nrows,
                            cg_transfer *rows, uint32_t *rec_of, hipStream_t s);
hipError_t launch_2d_fold(const cg_transfer2d *recs, const uint64_t *first, uint64_t count, const uint32_t *rec_of,
                          const cg_verdict *rowv, uint64_t nrows, cg_verdict *out, hipStream_t s);
hipError_t launch_pointers(const DevState *st, const uint64_t *ptrs, uint64_t count, cg_ptr_check *out, hipStream_t s);
hipError_t launch_probe_read(const void *p, uint64_t bytes, uint64_t *sink, hipStream_t s);
hipError_t launch_probe_copy(void *d, const void *p, uint64_t bytes, hipStream_t s);
hipError_t launch_probe_l2(const void *p, uint64_t slice_bytes, uint32_t passes, uint32_t blocks, uint64_t *sink,
                           hipStream_t s);

}  // namespace xc
