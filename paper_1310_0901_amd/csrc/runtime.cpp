// Host runtime of the transfer checker: context, allocation table and its
// device mirror, shadow pool, per-stream workspaces, graph cache, plain and
// batched check paths, autotuner and the C ABI declared in xfercheck.h.
//
// Method: Cudagrind (arXiv 1310.0901).  The wrappers of Sec. 1.2 / Sec. 2 keep
// a per-context list of device allocations, updated on every allocation and
// free, and cross-check each copy against it and against host shadow memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <fstream>
#include <map>
#include <mutex>
#include <set>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "host_logic.h"
#include "race.h"
#include "sort.h"
#include "xc_internal.h"

using namespace xc;

namespace {

constexpr uint64_t kFillPiece = 1ull << 20;   // bytes per fill range
constexpr uint64_t kFillCap = 1ull << 13;     // ranges per fill launch
constexpr uint64_t kDeltaWords = 4096;        // a table delta this small is uploaded by a kernel
constexpr int kFillSlots = 8;                 // staging ring for fill ranges
constexpr uint64_t kTilesCap = 1ull << 22;    // tile-start entries per workspace
constexpr int kPooledEvents = 16;             // completion events made at set-up
// launch shape for checks of mostly short pitched rows (measured on 4 KiB and
// 512-byte rows: 20-26 % faster than the shapes tuned for long transfers)
constexpr cg_tuning kShortRowTuning = {256, 2, 16, 1u << 16, 0, {0, 0, 0}};

// largest batch worked as segments: its 3 * count positions take 96-byte
// descriptors (about 40 GB at this size); larger batches keep their order
constexpr uint64_t kSegMaxRecords = 1ull << 27;
constexpr size_t kGraphsPerWs = 16;
// batches of at most this many records are worked in one launch (k_small),
// unless XC_SMALL_MAX sets another limit
constexpr uint64_t kSmallMax = 256;
constexpr int kVersions = 4;             // table versions in the device ring

// A captured batched check.  With kernel timing on, the scan kernel is kept in
// a graph of its own so that events on the caller's stream bracket exactly it.
struct GraphEntry {
    const DevState *st;
    const void *recs;
    void *out;
    uint64_t count;
    uint32_t mode;
    cg_tuning tun;
    bool split;
    // whole check (or, split for timing: the preparation, the scan kernel);
    // a split check with shadow indexes has its preparation in three parts,
    // the indexes' counting pass alone in the middle one
    hipGraph_t graph, graph2, graph3, graph4;
    hipGraphExec_t exec, exec2, exec3, exec4;
};

void destroy_graph(GraphEntry &g)
{
    for (hipGraphExec_t x : {g.exec, g.exec2, g.exec3, g.exec4})
        if (x) (void)hipGraphExecDestroy(x);
    for (hipGraph_t x : {g.graph, g.graph2, g.graph3, g.graph4})
        if (x) (void)hipGraphDestroy(x);
}

struct Workspace {
    uint64_t cap = 0;
    Desc *desc = nullptr;
    uint64_t *weight = nullptr, *local = nullptr, *bsum = nullptr, *boff = nullptr, *prefix = nullptr;
    uint32_t *tile_start = nullptr;
    Ctl *ctl = nullptr;
    uint64_t *h_weight = nullptr;   // pinned copy of weights (plain path)
    uint64_t ctx_seen = ~0ull;      // ctx_seq when this stream last waited for ev_ctx
    SmallAcc *small = nullptr;      // small_max accumulators of the one-launch path (k_small)
    Pitch *pitch = nullptr;         // per position of a pitched 2D batch (allocated on first use)
    uint64_t pitch_cap = 0;
    hipEvent_t done = nullptr;      // recorded after every check issued on this stream
    bool used = false;
    std::vector<GraphEntry> graphs;
    // large batches worked as source-block segments (allocated on first use):
    // per record the classify output and first segment, per segment its
    // record, the sort of the segments, and per position its record
    uint64_t seg_cap = 0;    // records
    Desc *rdesc = nullptr;
    uint64_t *rweight = nullptr, *rlocal = nullptr, *rbsum = nullptr, *sfirst = nullptr, *sbsum = nullptr;
    uint64_t *meta = nullptr;
    uint32_t *srec = nullptr;
    SortWs sort;
    uint32_t *perm = nullptr;
    // shadow indexes of check-only segmented batches, host region and pool
    // (shadowindex.hip; allocated on first use)
    ShadowIndex hidx{}, pidx{};
};

struct TimingPair {
    hipEvent_t a = nullptr, b = nullptr;
};

// One version of the device table: sorted base | end | off | top arrays and
// the DevState that points at them.  `uses` holds, per stream, an event
// recorded after the last check on that stream that read this version.
struct TableVersion {
    uint64_t *tab = nullptr;
    DevState *st = nullptr;
    uint64_t n = 0;
    std::map<hipStream_t, hipEvent_t> uses;
    hipEvent_t fixed_use = nullptr;   // after the last check_transfers_noalloc call that read this version
    bool fixed_used = false;
};

// Row expansion of pitched 2D copies on one stream.
struct StridedWs {
    uint64_t rec_cap = 0, row_cap = 0;
    uint64_t *first = nullptr, *bsum = nullptr, *bshort = nullptr, *total = nullptr, *h_total = nullptr;
    cg_transfer *rows = nullptr;
    uint32_t *rec_of = nullptr;
    cg_verdict *rowv = nullptr;
};

struct Quarantined {
    uint64_t seq, off, size;   // pool block freed after check number `seq` was issued
};

struct InFlight {
    uint64_t seq;
    hipEvent_t ev;
};

bool same_tuning(const cg_tuning &x, const cg_tuning &y)
{
    return x.block == y.block && x.unroll == y.unroll && x.blocks_per_cu == y.blocks_per_cu &&
           x.tile_units == y.tile_units && x.nontemporal == y.nontemporal;
}

}  // namespace

struct cg_ctx {
    int dev = 0;
    int cu_count = 0;
    std::string arch;
    hipStream_t s = nullptr;     // the context's own stream (table and shadow updates)
    hipStream_t cap = nullptr;   // graph capture stream
    uint8_t *pool = nullptr;
    uint64_t pool_bytes = 0;
    PoolAllocator *palloc = nullptr;
    AllocTable table;
    uint64_t max_allocs = 0;
    // device table: a ring of versions; frees and allocations since the
    // current version wait in pend_del / pend_ins until the next check
    TableVersion ver[kVersions];
    int cur = 0;
    bool full_dirty = true;
    std::set<uint64_t> pend_del;
    std::map<uint64_t, AllocEntry> pend_ins;
    uint64_t *d_delta = nullptr;   // sorted deletes | inserted base | end | off
    uint8_t *m_keep = nullptr;
    uint32_t *m_loc = nullptr;
    uint64_t *m_bsum = nullptr, *m_boff = nullptr;
    uint64_t *h_stage = nullptr;   // pinned staging for table uploads and large deltas
    // coherent host staging that small uploads read from the device (k_upload):
    // a table delta of up to kDeltaWords words and the context state; m_* are
    // the device's addresses of the same memory
    uint64_t *h_delta = nullptr, *m_delta = nullptr;
    DevState *h_state = nullptr, *m_state = nullptr;
    hipEvent_t ev_stage = nullptr;
    bool stage_busy = false;
    uint64_t versions_made = 0, merges = 0, full_uploads = 0;
    // shadow-pool blocks of freed allocations wait until every check issued
    // before the free has finished
    std::deque<Quarantined> quarantine;
    std::deque<InFlight> inflight;
    std::vector<hipEvent_t> ev_pool;
    uint64_t check_seq = 0, done_seq = 0;
    Region region{0, 0, nullptr, nullptr};
    // fills: a ring of staging buffers so that a new fill rarely waits for
    // the copy of an earlier one
    FillRange *d_fill = nullptr, *h_fill = nullptr, *m_fill = nullptr;   // h_fill coherent, m_fill its device address
    hipEvent_t ev_fill[kFillSlots] = {};
    bool fill_busy[kFillSlots] = {};
    int fill_next = 0;
    // ordering
    hipEvent_t ev_ctx = nullptr;
    uint64_t ctx_seq = 0;          // records of ev_ctx so far
    std::map<hipStream_t, Workspace *> ws;
    std::map<hipStream_t, RaceWs> race_ws;   // concurrent-access joins, per stream
    uint64_t reorder_min = 16384;            // batches this large are worked as source-block segments
    uint32_t seg_min_log2 = 20;              // smallest source block of the segments, log2
    uint64_t small_max = kSmallMax;          // batches this small run in one launch (k_small); 0: never
    uint32_t task_pos = 0;                   // positions per host-source task (0: the kernel's default)
    bool pitched_2d = true;                  // 2D records as pitched positions (else rows expanded, one wait)
    int shadow_index = 1;                    // shadow indexes of check-only segmented batches: 0 off, 1 when they pay, 2 always
    uint32_t sidx_ratio = 4;                 // one pays from this many of the batch's bytes per byte of its space
    uint64_t sidx_cap = 1ull << 22;          // entries per list of a shadow index
    uint32_t sidx_blocks_per_cu = 8;         // grid of the index passes
    int host_lds = 1;                        // check-only segments of host sources worked from LDS: 1 in the
                                             // scan kernel's blocks, 2 in a kernel of their own after it, 0 not
    std::map<hipStream_t, StridedWs> strided_ws;   // row expansion of 2D copies, per stream
    cg_tuning tuning{};        // check-only launch shape
    cg_tuning tuning_prop{};   // launch shape when propagating (more registers per lane)
    // timing
    bool timing = false;
    std::vector<TimingPair> tpairs;   // pairs of the last check
    std::vector<TimingPair> ipairs;   // pairs around the indexes' counting pass
    size_t iused = 0;
    uint64_t *idx_read = nullptr;     // device: bytes the index counting passes read, [0] host region, [1] pool
    size_t tused = 0;
    std::string last_error;
};

namespace {

int fail(cg_ctx *c, int code, const std::string &msg)
{
    if (c) c->last_error = msg;
    return code;
}

int hip_fail(cg_ctx *c, const char *what, hipError_t e)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(c, CG_EHIP, m);
}

#define HIPTRY(ctx, call)                                   \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, #call, e_); \
    } while (0)

// ctx stream waits for every check issued so far
int ctx_begin(cg_ctx *c)
{
    for (auto &kv : c->ws)
        if (kv.second->used) HIPTRY(c, hipStreamWaitEvent(c->s, kv.second->done, 0));
    return CG_OK;
}

int ctx_end(cg_ctx *c)
{
    HIPTRY(c, hipEventRecord(c->ev_ctx, c->s));
    ++c->ctx_seq;
    return CG_OK;
}

// Stream s waits for the context's latest state (a table version, fills).
// Every check waits: a stream handle may be a destroyed stream's, reused.
int wait_ctx(cg_ctx *c, Workspace *w, hipStream_t s)
{
    HIPTRY(c, hipStreamWaitEvent(s, c->ev_ctx, 0));
    w->ctx_seen = c->ctx_seq;
    return CG_OK;
}

// Make a new table version if allocations, frees or the host region changed
// since the current one.  The new version goes to the next buffer of the ring
// after the checks that last read that buffer have finished; it is either a
// full upload from the host mirror or a device merge of the previous version
// with the sorted frees and allocations made since.
int materialize(cg_ctx *c)
{
    if (!c->full_dirty && c->pend_del.empty() && c->pend_ins.empty()) return CG_OK;
    if (c->stage_busy) {
        HIPTRY(c, hipEventSynchronize(c->ev_stage));
        c->stage_busy = false;
    }
    const int t = (c->cur + 1) % kVersions;
    TableVersion &nv = c->ver[t], &ov = c->ver[c->cur];
    for (auto &kv : nv.uses) HIPTRY(c, hipStreamWaitEvent(c->s, kv.second, 0));
    if (nv.fixed_used) HIPTRY(c, hipStreamWaitEvent(c->s, nv.fixed_use, 0));
    const uint64_t n = c->table.size();
    const uint64_t M = c->max_allocs;
    uint32_t shift = 0;
    while (((n + (1ull << shift) - 1) >> shift) > (uint64_t)kMaxTop) ++shift;
    const uint32_t ntop = (uint32_t)((n + (1ull << shift) - 1) >> shift);
    const uint64_t nd = c->pend_del.size(), ni = c->pend_ins.size();
    const bool full = c->full_dirty || nd + 3 * ni > 3 * M || (nd + ni) * 4 > n + 64;
    uint64_t *hs = c->h_stage;
    if (full) {
        uint64_t *hb = hs, *he = hb + M, *ho = he + M, *ht = ho + M;
        c->table.export_sorted(hb, he, ho);
        for (uint32_t k = 0; k < ntop; ++k) ht[k] = hb[(uint64_t)k << shift];
        if (n) {
            HIPTRY(c, hipMemcpyAsync(nv.tab, hb, n * 8, hipMemcpyHostToDevice, c->s));
            HIPTRY(c, hipMemcpyAsync(nv.tab + M, he, n * 8, hipMemcpyHostToDevice, c->s));
            HIPTRY(c, hipMemcpyAsync(nv.tab + 2 * M, ho, n * 8, hipMemcpyHostToDevice, c->s));
            HIPTRY(c, hipMemcpyAsync(nv.tab + 3 * M, ht, ntop * 8ull, hipMemcpyHostToDevice, c->s));
        }
        c->full_uploads++;
    } else {
        const uint64_t words = nd + 3 * ni;
        const bool small = words <= kDeltaWords;
        if (small) hs = c->h_delta;
        uint64_t *hd = hs, *hib = hd + nd, *hie = hib + ni, *hio = hie + ni;
        size_t k = 0;
        for (uint64_t b : c->pend_del) hd[k++] = b;
        k = 0;
        for (const auto &kv : c->pend_ins) {
            hib[k] = kv.first;
            hie[k] = kv.first + kv.second.size;
            hio[k] = kv.second.off;
            ++k;
        }
        if (small) HIPTRY(c, launch_upload(c->m_delta, c->d_delta, words * 8, c->s));
        else HIPTRY(c, hipMemcpyAsync(c->d_delta, hs, words * 8, hipMemcpyHostToDevice, c->s));
        MergeArgs m{};
        m.old_base = ov.tab; m.old_end = ov.tab + M; m.old_off = ov.tab + 2 * M; m.n_old = ov.n;
        m.del = c->d_delta; m.n_del = nd;
        m.ins_base = c->d_delta + nd; m.ins_end = c->d_delta + nd + ni; m.ins_off = c->d_delta + nd + 2 * ni;
        m.n_ins = ni;
        m.new_base = nv.tab; m.new_end = nv.tab + M; m.new_off = nv.tab + 2 * M; m.new_top = nv.tab + 3 * M;
        m.top_shift = shift; m.ntop = ntop;
        m.keep = c->m_keep; m.loc = c->m_loc; m.bsum = c->m_bsum; m.boff = c->m_boff;
        HIPTRY(c, launch_merge(m, c->s));
        c->merges++;
    }
    DevState &st = *c->h_state;
    st.table.base = nv.tab;
    st.table.end = nv.tab + M;
    st.table.off = nv.tab + 2 * M;
    st.table.top = nv.tab + 3 * M;
    st.table.n = n;
    st.table.top_shift = shift;
    st.table.ntop = ntop;
    st.region = c->region;
    st.pool = (uint64_t)c->pool;
    st.size_bound = c->table.size_bound();
    st.pool_len = c->palloc->high();
    HIPTRY(c, launch_upload(c->m_state, nv.st, sizeof(DevState), c->s));
    HIPTRY(c, hipEventRecord(c->ev_stage, c->s));
    c->stage_busy = true;
    nv.n = n;
    c->cur = t;
    c->pend_del.clear();
    c->pend_ins.clear();
    c->full_dirty = false;
    c->versions_made++;
    return ctx_end(c);
}

int issue_fills(cg_ctx *c, const std::vector<FillRange> &rs, bool after_checks);
void add_fill(std::vector<FillRange> &rs, uint64_t ptr, uint64_t len, uint8_t v);

// Checks that have finished, in issue order; quarantined pool blocks whose
// readers are all done go back to the allocator.
void retire(cg_ctx *c, bool wait_all)
{
    while (!c->inflight.empty()) {
        InFlight &f = c->inflight.front();
        if (wait_all) (void)hipEventSynchronize(f.ev);
        else if (hipEventQuery(f.ev) != hipSuccess) break;
        c->done_seq = f.seq;
        c->ev_pool.push_back(f.ev);
        c->inflight.pop_front();
    }
    if (c->inflight.empty()) c->done_seq = c->check_seq;
    // released blocks are cleared to 0, so that a stale shadow left in the
    // pool adds no entries to the pool's shadow index (a new allocation fills
    // its block first, later on the same stream)
    std::vector<FillRange> zero;
    while (!c->quarantine.empty() && c->quarantine.front().seq <= c->done_seq) {
        const Quarantined &q = c->quarantine.front();
        add_fill(zero, (uint64_t)c->pool + q.off, c->palloc->rounded(q.size), 0);
        c->palloc->release(q.off, q.size);
        c->quarantine.pop_front();
    }
    if (!zero.empty()) (void)issue_fills(c, zero, false);   // a failed clear only makes an index longer
}

// Issue fills of [ptr, ptr + len) with v on the context stream.  Fills of
// existing allocations (shadow_set) wait for every check issued before;
// fills of fresh allocations need not: their pool blocks are read by no check.
int issue_fills(cg_ctx *c, const std::vector<FillRange> &rs, bool after_checks)
{
    size_t i = 0;
    if (after_checks) {
        int rc = ctx_begin(c);
        if (rc) return rc;
    }
    while (i < rs.size()) {
        const int f = c->fill_next;
        c->fill_next = (f + 1) % kFillSlots;
        if (c->fill_busy[f]) {
            HIPTRY(c, hipEventSynchronize(c->ev_fill[f]));
            c->fill_busy[f] = false;
        }
        FillRange *h = c->h_fill + f * kFillCap, *d = c->d_fill + f * kFillCap;
        size_t k = 0;
        for (; i < rs.size() && k < kFillCap; ++i) h[k++] = rs[i];
        HIPTRY(c, launch_upload(c->m_fill + f * kFillCap, d, k * sizeof(FillRange), c->s));
        HIPTRY(c, launch_fill(d, k, c->s));
        HIPTRY(c, hipEventRecord(c->ev_fill[f], c->s));
        c->fill_busy[f] = true;
    }
    return ctx_end(c);
}

void add_fill(std::vector<FillRange> &rs, uint64_t ptr, uint64_t len, uint8_t v)
{
    while (len) {
        const uint64_t take = len < kFillPiece ? len : kFillPiece;
        rs.push_back(FillRange{ptr, take, v, 0});
        ptr += take;
        len -= take;
    }
}

void free_seg(Workspace *w)
{
    void *ps[] = {w->rdesc, w->rweight, w->rlocal, w->rbsum, w->sfirst, w->sbsum, w->meta, w->srec, w->perm};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    sort_release(w->sort);
    w->rdesc = nullptr;
    w->rweight = w->rlocal = w->rbsum = w->sfirst = w->sbsum = w->meta = nullptr;
    w->srec = w->perm = nullptr;
    w->seg_cap = 0;
    for (ShadowIndex *x : {&w->hidx, &w->pidx}) {
        void *hs[] = {x->uchunk, x->umask, x->ucum, x->nchunk, x->nmask, x->bcnt, x->sflag, x->state,
                      x->smark, x->slist, x->mcnt};
        for (void *p : hs)
            if (p) (void)hipFree(p);
        *x = ShadowIndex{};
    }
}

void free_ws(Workspace *w)
{
    for (auto &g : w->graphs) destroy_graph(g);
    w->graphs.clear();
    (void)hipFree(w->desc);
    (void)hipFree(w->weight);
    (void)hipFree(w->local);
    (void)hipFree(w->bsum);
    (void)hipFree(w->boff);
    (void)hipFree(w->prefix);
    (void)hipFree(w->tile_start);
    (void)hipFree(w->ctl);
    if (w->h_weight) (void)hipHostFree(w->h_weight);
    (void)hipFree(w->small);
    w->small = nullptr;
    (void)hipFree(w->pitch);
    w->pitch = nullptr;
    w->pitch_cap = 0;
    free_seg(w);
    w->desc = nullptr;
    w->weight = w->local = w->bsum = w->boff = w->prefix = nullptr;
    w->tile_start = nullptr;
    w->ctl = nullptr;
    w->h_weight = nullptr;
    w->cap = 0;
}

int get_ws(cg_ctx *c, hipStream_t s, uint64_t count, Workspace **out)
{
    Workspace *w;
    auto it = c->ws.find(s);
    if (it == c->ws.end()) {
        w = new Workspace();
        HIPTRY(c, hipEventCreateWithFlags(&w->done, hipEventDisableTiming));
        c->ws[s] = w;
    } else {
        w = it->second;
    }
    if (w->cap < count) {
        // buffers may be in use by earlier checks on this stream
        HIPTRY(c, hipStreamSynchronize(s));
        free_ws(w);
        uint64_t cap = 1024;
        while (cap < count) cap <<= 1;
        const uint64_t nb = (cap + kClassifyBlock - 1) / kClassifyBlock;
        HIPTRY(c, hipMalloc(&w->desc, cap * sizeof(Desc)));
        HIPTRY(c, hipMalloc(&w->weight, cap * 8));
        HIPTRY(c, hipMalloc(&w->local, cap * 8));
        HIPTRY(c, hipMalloc(&w->bsum, nb * 8));
        HIPTRY(c, hipMalloc(&w->boff, nb * 8));
        HIPTRY(c, hipMalloc(&w->prefix, (cap + 1) * 8));
        HIPTRY(c, hipMalloc(&w->tile_start, kTilesCap * 4));
        HIPTRY(c, hipMalloc(&w->ctl, sizeof(Ctl)));
        HIPTRY(c, hipHostMalloc(&w->h_weight, cap * 8, hipHostMallocDefault));
        HIPTRY(c, hipMalloc(&w->small, std::max<uint64_t>(c->small_max, 1) * sizeof(SmallAcc)));
        HIPTRY(c, launch_small_reset(w->small, std::max<uint64_t>(c->small_max, 1), s));
        w->cap = cap;
    }
    *out = w;
    return CG_OK;
}

BatchArgs make_args(cg_ctx *c, Workspace *w, const cg_transfer *recs, uint64_t count, cg_verdict *out,
                    uint32_t mode)
{
    BatchArgs a{};
    a.recs = recs;
    a.count = count;
    a.out = (mode & CG_CHECK) ? out : nullptr;
    a.mode = mode & (CG_CHECK | CG_PROPAGATE);
    a.st = c->ver[c->cur].st;
    a.desc = w->desc;
    a.weight = w->weight;
    a.local = w->local;
    a.bsum = w->bsum;
    a.boff = w->boff;
    a.prefix = w->prefix;
    a.tile_start = w->tile_start;
    a.tiles_cap = kTilesCap;
    a.ctl = w->ctl;
    return a;
}

LaunchShape shape_of(cg_ctx *c, const cg_tuning &t)
{
    LaunchShape sh;
    sh.block = t.block;
    sh.unroll = t.unroll;
    sh.grid = (uint32_t)c->cu_count * t.blocks_per_cu;
    sh.nontemporal = t.nontemporal;
    sh.tile_units = t.tile_units;
    sh.cus = (uint32_t)c->cu_count;
    sh.lds_after = c->host_lds == 2 ? 1u : 0u;
    return sh;
}

// A batch worked as source-block segments: k_classify over the records in
// their given order (ar), then the segments (g) as the positions of the batch.
// How a batched check is prepared beyond classify and scan: as source-block
// segments (seg; ar is then the record-level classify's arguments), and/or
// with the shadow indexes (hidx, pidx; without segments ar is the batch's own
// arguments).
struct SegPlan {
    bool seg;
    BatchArgs ar;
    SegArgs g;
    SortWs *sort;
    // not null: build the shadow indexes (host region, pool) and answer the
    // records whose spaces are indexed from them
    const ShadowIndex *hidx, *pidx;
};

// The preparation of a batched check, in three stages around the shadow
// indexes' counting pass (stage 1, empty without indexes: one launch over the
// host region's and the pool's listed steps), so that timing can bracket that
// pass.
hipError_t prepare_stage(const BatchArgs &a, const LaunchShape &sh, hipStream_t s, const SegPlan *sp, int stage)
{
    hipError_t e;
    const bool idx = sp && sp->hidx;
    if (stage == 0) {
        if (!sp) return launch_classify(a, s);
        if (idx && (e = launch_sidx_reset(*sp->hidx, *sp->pidx, s)) != hipSuccess) return e;
        if ((e = launch_classify(sp->ar, s)) != hipSuccess) return e;
        if (idx && (e = launch_sidx_marks(*sp->hidx, sp->ar.st, s)) != hipSuccess) return e;
        if (idx && (e = launch_sidx_marks(*sp->pidx, sp->ar.st, s)) != hipSuccess) return e;
        return hipSuccess;
    }
    if (stage == 1) return idx ? launch_sidx_count(*sp->hidx, *sp->pidx, sp->ar.st, s) : hipSuccess;
    if (idx) {
        if ((e = launch_sidx_finish(*sp->hidx, sp->ar.st, s)) != hipSuccess) return e;
        if ((e = launch_sidx_finish(*sp->pidx, sp->ar.st, s)) != hipSuccess) return e;
        if ((e = launch_sidx_query(sp->ar, *sp->hidx, *sp->pidx, sp->ar.bsum, s)) != hipSuccess) return e;
        // a batch in its given order: the prefix inputs again, from the units left
        if (!sp->seg && (e = launch_reweigh(a, s)) != hipSuccess) return e;
    }
    if (sp && sp->seg && (e = launch_segments(sp->g, *sp->sort, a, const_cast<uint32_t *>(a.perm), s)) != hipSuccess)
        return e;
    if ((e = launch_scan_sums(a, sh.tile_units, sh.grid * (sh.block / 64), s)) != hipSuccess) return e;
    return launch_prefix_tiles(a, s);
}

hipError_t enqueue_prepare(const BatchArgs &a, const LaunchShape &sh, hipStream_t s, const SegPlan *sp)
{
    hipError_t e;
    for (int k = 0; k < 3; ++k)
        if ((e = prepare_stage(a, sh, s, sp, k)) != hipSuccess) return e;
    return hipSuccess;
}

// The whole check; with tp, events around the scan kernel, and with ip
// around the indexes' counting pass.
hipError_t enqueue_batched(const BatchArgs &a, const LaunchShape &sh, hipStream_t s, TimingPair *tp,
                           const SegPlan *sp, TimingPair *ip = nullptr)
{
    hipError_t e;
    if ((e = prepare_stage(a, sh, s, sp, 0)) != hipSuccess) return e;
    if (ip && (e = hipEventRecord(ip->a, s)) != hipSuccess) return e;
    if ((e = prepare_stage(a, sh, s, sp, 1)) != hipSuccess) return e;
    if (ip && (e = hipEventRecord(ip->b, s)) != hipSuccess) return e;
    if ((e = prepare_stage(a, sh, s, sp, 2)) != hipSuccess) return e;
    if (tp && (e = hipEventRecord(tp->a, s)) != hipSuccess) return e;
    if ((e = launch_batched(a, sh, s)) != hipSuccess) return e;
    if (tp && (e = hipEventRecord(tp->b, s)) != hipSuccess) return e;
    return hipSuccess;
}

int capture(cg_ctx *c, hipGraph_t *g, hipGraphExec_t *x, const BatchArgs &a, const LaunchShape &sh, int part,
            const SegPlan *sp);

// The cached graph of this batched check (keyed by table version, buffers,
// count, mode and launch shape), captured on first use.
int find_graph(cg_ctx *c, Workspace *w, const BatchArgs &a, const SegPlan *sp, const LaunchShape &sh,
               const cg_tuning &tun, bool split, hipStream_t s, GraphEntry **out)
{
    // (the segment keys' width follows the shadow's addresses, which a new
    // host region may change)
    const uint32_t mode = (a.mode & 3u) | (a.perm ? 4u : 0u) | (sp && sp->seg && sp->g.key_bytes == 8 ? 8u : 0u);
    for (auto &g : w->graphs)
        if (g.st == a.st && g.recs == a.recs && g.count == a.count && g.mode == mode && same_tuning(g.tun, tun) &&
            g.split == split && g.out == a.out) {
            *out = &g;
            return CG_OK;
        }
    if (w->graphs.size() >= kGraphsPerWs) {
        HIPTRY(c, hipStreamSynchronize(s));
        destroy_graph(w->graphs.front());
        w->graphs.erase(w->graphs.begin());
    }
    GraphEntry g{a.st, a.recs, a.out, a.count, mode, tun, split, nullptr, nullptr, nullptr, nullptr,
                 nullptr, nullptr, nullptr, nullptr};
    const bool three = split && sp && sp->pidx;
    int rc = capture(c, &g.graph, &g.exec, a, sh, !split ? 0 : three ? 3 : 1, sp);
    if (!rc && split) rc = capture(c, &g.graph2, &g.exec2, a, sh, 2, sp);
    if (!rc && three) rc = capture(c, &g.graph3, &g.exec3, a, sh, 4, sp);
    if (!rc && three) rc = capture(c, &g.graph4, &g.exec4, a, sh, 5, sp);
    if (rc) {
        destroy_graph(g);
        return rc;
    }
    w->graphs.push_back(g);
    *out = &w->graphs.back();
    return CG_OK;
}

TimingPair *next_pair(cg_ctx *c)
{
    if (c->tused == c->tpairs.size()) {
        TimingPair p;
        (void)hipEventCreate(&p.a);
        (void)hipEventCreate(&p.b);
        c->tpairs.push_back(p);
    }
    return &c->tpairs[c->tused++];
}

TimingPair *next_ipair(cg_ctx *c)
{
    if (c->iused == c->ipairs.size()) {
        TimingPair p;
        (void)hipEventCreate(&p.a);
        (void)hipEventCreate(&p.b);
        c->ipairs.push_back(p);
    }
    return &c->ipairs[c->iused++];
}

int valid_tuning(const cg_tuning &t)
{
    const bool u_ok = t.unroll == 1 || t.unroll == 2 || t.unroll == 4 || t.unroll == 8;
    const bool b_ok = t.block == 256 || t.block == 512;
    const bool tu_ok = t.tile_units >= 4096 && (t.tile_units & (t.tile_units - 1)) == 0;
    return u_ok && b_ok && tu_ok && t.blocks_per_cu >= 1 && t.blocks_per_cu <= 16;
}

// Host-side verification of the no-conflict rule for propagation: no
// record's destination shadow bytes may meet another record's source or
// destination shadow bytes.
int debug_conflicts(cg_ctx *c, const cg_transfer *recs_dev, uint64_t count, hipStream_t s)
{
    std::vector<cg_transfer> h(count);
    HIPTRY(c, hipMemcpyAsync(h.data(), recs_dev, count * sizeof(cg_transfer), hipMemcpyDeviceToHost, s));
    HIPTRY(c, hipStreamSynchronize(s));
    struct Iv {
        uint64_t a, b;   // shadow byte interval in a unified space
        uint64_t rec;
        bool write;
    };
    std::vector<Iv> iv;
    // unified shadow space: host region at [0, hl), pool at [2^63, 2^63 + pool)
    const uint64_t POOL = 1ull << 63;
    auto host_iv = [&](uint64_t p, uint64_t n, uint64_t *a, uint64_t *b) {
        const uint64_t hb = c->region.hb, hl = c->region.hl;
        uint64_t lo = std::max<uint64_t>(p, hb), hi = std::min<uint64_t>(p + n < p ? ~0ull : p + n, hb + hl);
        if (hi <= lo) return false;
        *a = lo - hb;
        *b = hi - hb;
        return true;
    };
    auto dev_iv = [&](uint64_t p, uint64_t n, uint64_t *a, uint64_t *b) {
        uint64_t base;
        const AllocEntry *e = c->table.find(p, &base);
        if (!e) return false;
        const uint64_t avail = base + e->size - p;
        *a = POOL + e->off + (p - base);
        *b = *a + std::min(n, avail);
        return true;
    };
    for (uint64_t t = 0; t < count; ++t) {
        const cg_transfer &r = h[t];
        if (r.kind > CG_D2D || r.n == 0) continue;
        if (r.kind == CG_D2D) {
            const bool ov = (r.src < r.dst) ? (r.dst - r.src < r.n) : (r.src - r.dst < r.n);
            if (ov) {
                uint64_t a, b;
                if (dev_iv(r.src, r.n, &a, &b)) iv.push_back({a, b, t, false});
                continue;   // not propagated
            }
        }
        uint64_t a, b;
        const bool sh = r.kind == CG_H2D, dh = r.kind == CG_D2H;
        if (sh ? host_iv(r.src, r.n, &a, &b) : dev_iv(r.src, r.n, &a, &b)) iv.push_back({a, b, t, false});
        if (dh ? host_iv(r.dst, r.n, &a, &b) : dev_iv(r.dst, r.n, &a, &b)) iv.push_back({a, b, t, true});
    }
    std::sort(iv.begin(), iv.end(), [](const Iv &x, const Iv &y) { return x.a < y.a; });
    // sweep by start: keep, for reads and for writes separately, the two
    // furthest-reaching intervals of distinct records seen so far
    struct Best {
        uint64_t end1 = 0, rec1 = ~0ull, end2 = 0;
        uint64_t reach_other(uint64_t rec) const { return rec1 != rec ? end1 : end2; }
        void add(uint64_t end, uint64_t rec)
        {
            if (rec == rec1) { end1 = std::max(end1, end); return; }
            if (end > end1) { end2 = end1; end1 = end; rec1 = rec; }
            else if (end > end2) end2 = end;
        }
    } rd, wr;
    for (const Iv &x : iv) {
        if (x.a < wr.reach_other(x.rec) || (x.write && x.a < rd.reach_other(x.rec)))
            return fail(c, CG_ECONFLICT, "record " + std::to_string(x.rec) +
                                             " touches shadow bytes another record of the batch writes or reads");
        (x.write ? wr : rd).add(x.b, x.rec);
    }
    return CG_OK;
}

int note_use(cg_ctx *c, hipStream_t s);

// Batches of at least reorder_min records and at most kSegMaxRecords are
// worked as source-block segments unless the caller keeps the given order.
bool segmented(const cg_ctx *c, uint64_t count, uint32_t mode)
{
    return !(mode & (CG_PLAIN | CG_KEEP_ORDER)) && count >= 1 && count >= c->reorder_min && count <= kSegMaxRecords;
}

// Segment buffers for `count` records; the positions (w->cap) are already
// at least 3 * count.
int reserve_segments(cg_ctx *c, Workspace *w, uint64_t count, hipStream_t s)
{
    if (w->seg_cap >= count && w->sort.cap >= w->cap) return CG_OK;
    HIPTRY(c, hipStreamSynchronize(s));   // the old buffers may still be in use
    for (auto &g : w->graphs) destroy_graph(g);
    w->graphs.clear();
    free_seg(w);
    uint64_t cap = 1024;
    while (cap < count) cap <<= 1;
    const uint64_t nb = (cap + kClassifyBlock - 1) / kClassifyBlock;
    HIPTRY(c, hipMalloc(&w->rdesc, cap * sizeof(Desc)));
    HIPTRY(c, hipMalloc(&w->rweight, cap * 8));
    HIPTRY(c, hipMalloc(&w->rlocal, cap * 8));
    HIPTRY(c, hipMalloc(&w->sfirst, cap * 8));
    HIPTRY(c, hipMalloc(&w->rbsum, nb * 8));
    HIPTRY(c, hipMalloc(&w->sbsum, nb * 8));
    HIPTRY(c, hipMalloc(&w->meta, 64));
    HIPTRY(c, hipMalloc(&w->srec, w->cap * 4));
    HIPTRY(c, hipMalloc(&w->perm, w->cap * 4));
    const hipError_t e = sort_reserve(w->sort, w->cap);
    if (e != hipSuccess) return hip_fail(c, "segment sort work space", e);
    w->seg_cap = cap;
    return CG_OK;
}

// The shadow indexes' buffers: lists of sidx_cap entries (the pool's
// unaddressable list stays empty: one entry), block counts for a grid of 8
// blocks per CU.
int reserve_sidx(cg_ctx *c, Workspace *w)
{
    if (w->pidx.state) return CG_OK;
    if (!c->idx_read) {
        HIPTRY(c, hipMalloc(&c->idx_read, 2 * 8));
        HIPTRY(c, hipMemset(c->idx_read, 0, 2 * 8));
    }
    for (uint32_t space : {0u, 1u}) {
        ShadowIndex &x = space ? w->pidx : w->hidx;
        x.space = space;
        x.cap_u = c->sidx_cap;
        x.cap_n = space ? 1 : c->sidx_cap;
        x.grid = (uint32_t)std::max(c->cu_count, 1) * c->sidx_blocks_per_cu;
        HIPTRY(c, hipMalloc(&x.uchunk, (x.cap_u + 1) * 8));
        HIPTRY(c, hipMalloc(&x.umask, x.cap_u * 4));
        HIPTRY(c, hipMalloc(&x.ucum, (x.cap_u + 1) * 8));
        HIPTRY(c, hipMalloc(&x.nchunk, x.cap_n * 8));
        HIPTRY(c, hipMalloc(&x.nmask, x.cap_n * 4));
        HIPTRY(c, hipMalloc(&x.bcnt, 6ull * x.grid * 8));
        // a mark, a list entry and 4 flags per step of 4,096 chunks (64 KiB) of
        // the pool, or of a host region of up to 64 GiB; a larger one is not indexed
        const uint64_t len = space ? c->palloc->capacity() : std::max<uint64_t>(c->region.hl, 64ull << 30);
        x.steps_cap = (len >> kIdxStepShift) + 1;
        x.mark_grid = (uint32_t)((x.steps_cap + 16383) / 16384);
        HIPTRY(c, hipMalloc(&x.sflag, 4 * x.steps_cap));
        HIPTRY(c, hipMalloc(&x.slist, 4 * x.steps_cap));
        HIPTRY(c, hipMalloc(&x.smark, 16384ull * x.mark_grid));
        HIPTRY(c, hipMemset(x.smark, 0, 16384ull * x.mark_grid));   // the marking kernels clear what they read
        HIPTRY(c, hipMalloc(&x.mcnt, 8ull * x.mark_grid));
        HIPTRY(c, hipMalloc(&x.state, 8 * 8));
        x.read = c->idx_read + space;
    }
    return CG_OK;
}

// a batch's classify kernels feed the workspace's indexes: bytes per space and step marks
void set_index_args(BatchArgs &a, const Workspace *w)
{
    const ShadowIndex *xs[2] = {&w->hidx, &w->pidx};
    for (int k = 0; k < 2; ++k) {
        a.index_bytes[k] = xs[k]->state;
        a.index_mark[k] = xs[k]->smark;
        a.mark_cap[k] = xs[k]->steps_cap;
    }
}

// Blocks per record of a small batch, at most: `hint`, or else about 8
// blocks of 256 threads per CU over the whole batch (a record uses fewer
// when it is small, k_small).
uint32_t small_bpr(const cg_ctx *c, uint64_t count, const LaunchShape &sh, uint32_t hint)
{
    const uint64_t grid = (uint64_t)c->cu_count * 8 * 256 / (sh.block ? sh.block : 256);
    uint64_t bpr = hint ? hint : grid / (count ? count : 1);
    if (bpr < 1) bpr = 1;
    if (bpr > grid) bpr = grid;
    return (uint32_t)bpr;
}

// With `after`, a one-launch batch records that event right after its launch,
// before the bookkeeping events (a caller timing the batch's completion).
int run_check(cg_ctx *c, const cg_transfer *recs, uint64_t count, cg_verdict *out, uint32_t mode,
              hipStream_t s, const cg_tuning &tun, uint32_t bpr = 0, hipEvent_t after = nullptr)
{
    Workspace *w;
    const bool seg = segmented(c, count, mode);
    const uint64_t npos = seg ? 3 * count : count;   // positions of the batch
    int rc = get_ws(c, s, npos, &w);
    if (rc) return rc;
    rc = materialize(c);
    if (rc) return rc;
    rc = wait_ctx(c, w, s);
    if (rc) return rc;
    if ((mode & CG_DEBUG_CONFLICTS) && (mode & CG_PROPAGATE)) {
        rc = debug_conflicts(c, recs, count, s);
        if (rc) return rc;
    }
    BatchArgs a = make_args(c, w, recs, npos, out, mode);
    SegPlan plan{};
    const SegPlan *sp = nullptr;
    if (seg) {
        // the work on each block of source memory runs together, so that
        // re-reads of the same bytes hit in cache
        rc = reserve_segments(c, w, count, s);
        if (rc) return rc;
        plan.ar = make_args(c, w, recs, count, out, mode);
        plan.ar.desc = w->rdesc;
        plan.ar.weight = w->rweight;
        plan.ar.local = w->rlocal;
        plan.ar.bsum = w->rbsum;
        plan.ar.boff = nullptr;
        plan.ar.prefix = nullptr;
        plan.ar.tile_start = nullptr;
        plan.ar.ctl = nullptr;
        // check-only: the host-source segments sort last and are worked from LDS
        const bool host_last = c->host_lds && (mode & (CG_CHECK | CG_PROPAGATE)) == CG_CHECK;
        // the segments' block indices (shadow address >> log2 B, B >= 2^seg_min_log2)
        // fit 31 bits, and the keys 4 bytes, when the shadow's highest address does
        const uint64_t top = std::max<uint64_t>((uint64_t)c->pool + c->palloc->capacity(),
                                                (uint64_t)c->region.v + c->region.hl);
        const uint32_t key_bytes = (top >> c->seg_min_log2) < (1ull << 31) ? 4u : 8u;
        plan.g = SegArgs{w->rdesc, count, npos, w->rbsum, w->sfirst, w->sbsum, w->srec, w->meta, c->seg_min_log2,
                         host_last ? 1u : 0u, key_bytes};
        plan.sort = &w->sort;
        plan.seg = true;
        a.perm = w->perm;
        a.lds_meta = host_last ? w->meta : nullptr;
        a.task_pos = c->task_pos;
        sp = &plan;
    }
    // a check without propagation, of more records than one launch takes and
    // not kept in its order: the shadow indexes answer what they can
    if (c->shadow_index && (mode & (CG_CHECK | CG_PROPAGATE | CG_PLAIN | CG_KEEP_ORDER)) == CG_CHECK &&
        count > c->small_max) {
        rc = reserve_sidx(c, w);
        if (rc) return rc;
        w->hidx.ratio = w->pidx.ratio = c->shadow_index == 2 ? 0u : c->sidx_ratio;
        if (!seg) {
            plan.seg = false;
            plan.ar = a;
        }
        plan.hidx = &w->hidx;
        plan.pidx = &w->pidx;
        set_index_args(plan.ar, w);
        if (!seg) a = plan.ar;
        sp = &plan;
    }
    const LaunchShape sh = shape_of(c, tun);
    if (!(mode & CG_PLAIN) && count <= c->small_max) {
        // few records: one launch, no preparation kernels
        TimingPair *tp = c->timing ? next_pair(c) : nullptr;
        if (tp) HIPTRY(c, hipEventRecord(tp->a, s));
        HIPTRY(c, launch_small(a, w->small, small_bpr(c, count, sh, bpr), sh, s));
        if (tp) HIPTRY(c, hipEventRecord(tp->b, s));
        if (after) HIPTRY(c, hipEventRecord(after, s));
    } else if (mode & CG_PLAIN) {
        HIPTRY(c, launch_classify(a, s));
        HIPTRY(c, hipMemcpyAsync(w->h_weight, w->weight, count * 8, hipMemcpyDeviceToHost, s));
        HIPTRY(c, hipStreamSynchronize(s));
        TimingPair *tp = c->timing ? next_pair(c) : nullptr;
        if (tp) HIPTRY(c, hipEventRecord(tp->a, s));
        for (uint64_t t = 0; t < count; ++t) {
            const uint64_t u = w->h_weight[t];
            if (u) HIPTRY(c, launch_plain(a, t, u, sh, s));
        }
        if (tp) HIPTRY(c, hipEventRecord(tp->b, s));
    } else if (mode & CG_EAGER) {
        TimingPair *tp = c->timing ? next_pair(c) : nullptr;
        TimingPair *ip = c->timing && sp && sp->pidx ? next_ipair(c) : nullptr;
        HIPTRY(c, enqueue_batched(a, sh, s, tp, sp, ip));
    } else {
        const bool split = c->timing;
        GraphEntry *ge = nullptr;
        rc = find_graph(c, w, a, sp, sh, tun, split, s, &ge);
        if (rc) return rc;
        if (split) {
            TimingPair *tp = next_pair(c);
            HIPTRY(c, hipGraphLaunch(ge->exec, s));
            if (ge->exec3) {
                TimingPair *ip = next_ipair(c);
                HIPTRY(c, hipEventRecord(ip->a, s));
                HIPTRY(c, hipGraphLaunch(ge->exec3, s));
                HIPTRY(c, hipEventRecord(ip->b, s));
                HIPTRY(c, hipGraphLaunch(ge->exec4, s));
            }
            HIPTRY(c, hipEventRecord(tp->a, s));
            HIPTRY(c, hipGraphLaunch(ge->exec2, s));
            HIPTRY(c, hipEventRecord(tp->b, s));
        } else {
            HIPTRY(c, hipGraphLaunch(ge->exec, s));
        }
    }
    HIPTRY(c, hipEventRecord(w->done, s));
    w->used = true;
    return note_use(c, s);
}

// Bookkeeping after work on stream s that reads the current table version:
// the version's ring slot is not overwritten, and pool blocks freed later are
// not reused, before that work has finished.
int note_use(cg_ctx *c, hipStream_t s)
{
    hipEvent_t &vu = c->ver[c->cur].uses[s];
    if (!vu) HIPTRY(c, hipEventCreateWithFlags(&vu, hipEventDisableTiming));
    HIPTRY(c, hipEventRecord(vu, s));
    hipEvent_t ev;
    if (c->ev_pool.empty()) HIPTRY(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    else { ev = c->ev_pool.back(); c->ev_pool.pop_back(); }
    HIPTRY(c, hipEventRecord(ev, s));
    c->inflight.push_back(InFlight{++c->check_seq, ev});
    if (c->inflight.size() > 256) retire(c, false);
    return CG_OK;
}

// Capture part 0 (the whole batched check), 1 (the preparation kernels) or
// 2 (the scan kernel) into an executable graph.
int capture(cg_ctx *c, hipGraph_t *g, hipGraphExec_t *x, const BatchArgs &a, const LaunchShape &sh, int part,
            const SegPlan *sp)
{
    HIPTRY(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    // 0: all; 1: the preparation; 2: the scan kernel; 3, 4, 5: the
    // preparation's stages 0, 1 (the indexes' counting pass), 2
    hipError_t e = part == 0 ? enqueue_batched(a, sh, c->cap, nullptr, sp)
                 : part == 1 ? enqueue_prepare(a, sh, c->cap, sp)
                 : part == 2 ? launch_batched(a, sh, c->cap)
                             : prepare_stage(a, sh, c->cap, sp, part - 3);
    hipError_t e2 = hipStreamEndCapture(c->cap, g);
    if (e != hipSuccess) return hip_fail(c, "graph capture", e);
    if (e2 != hipSuccess) return hip_fail(c, "hipStreamEndCapture", e2);
    HIPTRY(c, hipGraphInstantiate(x, *g, nullptr, nullptr, 0));
    return CG_OK;
}

std::string tuning_json(const cg_tuning &t)
{
    std::ostringstream o;
    o << "\"block\": " << t.block << ", \"unroll\": " << t.unroll << ", \"blocks_per_cu\": " << t.blocks_per_cu
      << ", \"tile_units\": " << t.tile_units << ", \"nontemporal\": " << t.nontemporal;
    return o.str();
}

bool parse_field(const std::string &line, const char *name, uint32_t *v)
{
    const std::string key = std::string("\"") + name + "\": ";
    const size_t p = line.find(key);
    if (p == std::string::npos) return false;
    *v = (uint32_t)std::stoul(line.substr(p + key.size()));
    return true;
}

}  // namespace

// ---- the no-allocation entry point's device array -----------------------------
// Accumulators of check_transfers_noalloc: a fixed array on every GPU the
// library runs on, held until the process ends.  In host code `scratch` is
// only a stand-in for the array; its device address on each GPU comes from
// hipGetSymbolAddress, taken once per device at set-up with that device
// current, and is the only thing passed to kernels.
static __device__ __align__(256) SmallAcc scratch[CG_NOALLOC_MAX];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
SmallAcc *g_scratch[kMaxDevices] = {};

// Once per device, with that device current: the array's address there, and
// every accumulator put in its starting state.
int scratch_setup(cg_ctx *c)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (c->dev < 0 || c->dev >= kMaxDevices) return fail(c, CG_EINVAL, "device index above 63");
    if (g_scratch[c->dev]) return CG_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(c, "hipGetSymbolAddress(scratch)", e != hipSuccess ? e : hipErrorUnknown);
    e = launch_small_reset(static_cast<SmallAcc *>(p), CG_NOALLOC_MAX, c->s);
    if (e == hipSuccess) e = hipStreamSynchronize(c->s);
    if (e != hipSuccess) return hip_fail(c, "scratch reset", e);
    g_scratch[c->dev] = static_cast<SmallAcc *>(p);
    return CG_OK;
}

SmallAcc *scratch_of(int dev)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return dev >= 0 && dev < kMaxDevices ? g_scratch[dev] : nullptr;
}

// note_use for check_transfers_noalloc: the version's own event, and an event
// from the pool (made by cg_create) for the pool blocks' quarantine; when the
// pool is empty, finished checks give theirs back first
int note_use_fixed(cg_ctx *c, hipStream_t s)
{
    TableVersion &v = c->ver[c->cur];
    HIPTRY(c, hipEventRecord(v.fixed_use, s));
    v.fixed_used = true;
    if (c->ev_pool.empty()) retire(c, false);
    if (c->ev_pool.empty()) retire(c, true);
    if (c->ev_pool.empty()) return fail(c, CG_ESTATE, "no pooled event");
    const hipEvent_t ev = c->ev_pool.back();
    c->ev_pool.pop_back();
    HIPTRY(c, hipEventRecord(ev, s));
    c->inflight.push_back(InFlight{++c->check_seq, ev});
    if (c->inflight.size() > 256) retire(c, false);
    return CG_OK;
}
}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *cg_strerror(int status)
{
    switch (status) {
    case CG_OK: return "ok";
    case CG_EINVAL: return "invalid argument";
    case CG_ENOMEM: return "out of shadow or device memory";
    case CG_EOVERLAP: return "allocation overlaps a live allocation";
    case CG_ENOTFOUND: return "not a live device allocation";
    case CG_ECONFLICT: return "records of one batch touch the same shadow bytes";
    case CG_ECAPACITY: return "allocation table is full";
    case CG_EHIP: return "HIP runtime error";
    case CG_ESTATE: return "call not valid in the current state";
    default: return "unknown status";
    }
}

const char *cg_last_error(cg_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int cg_create(cg_ctx **out, int hip_device, uint64_t shadow_pool_bytes, uint64_t max_allocs)
{
    if (!out || shadow_pool_bytes == 0 || max_allocs == 0) return CG_EINVAL;
    *out = nullptr;
    cg_ctx *c = new cg_ctx();
    c->dev = hip_device;
    c->max_allocs = max_allocs;
    auto bail = [&](int rc) {
        cg_destroy(c);
        return rc;
    };
    if (hipSetDevice(hip_device) != hipSuccess) return bail(CG_EHIP);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return bail(CG_EHIP);
    c->cu_count = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    if (hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking) != hipSuccess) return bail(CG_EHIP);
    if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) return bail(CG_EHIP);
    const uint64_t pool = (shadow_pool_bytes + 255) / 256 * 256;
    if (hipMalloc(&c->pool, pool) != hipSuccess) return bail(CG_ENOMEM);
    c->pool_bytes = pool;
    c->palloc = new PoolAllocator(pool, 256);
    for (auto &v : c->ver) {
        if (hipMalloc(&v.tab, (3 * max_allocs + kMaxTop) * 8) != hipSuccess) return bail(CG_ENOMEM);
        if (hipMalloc(&v.st, sizeof(DevState)) != hipSuccess) return bail(CG_ENOMEM);
    }
    if (hipMalloc(&c->d_delta, (3 * max_allocs + kMaxTop) * 8) != hipSuccess) return bail(CG_ENOMEM);
    if (hipMalloc(&c->m_keep, max_allocs) != hipSuccess) return bail(CG_ENOMEM);
    if (hipMalloc(&c->m_loc, max_allocs * 4) != hipSuccess) return bail(CG_ENOMEM);
    if (hipMalloc(&c->m_bsum, (max_allocs / 256 + 2) * 8) != hipSuccess) return bail(CG_ENOMEM);
    if (hipMalloc(&c->m_boff, (max_allocs / 256 + 2) * 8) != hipSuccess) return bail(CG_ENOMEM);
    if (hipHostMalloc(&c->h_stage, (3 * max_allocs + kMaxTop) * 8, hipHostMallocDefault) != hipSuccess)
        return bail(CG_ENOMEM);
    const unsigned coh = hipHostMallocMapped | hipHostMallocCoherent;
    if (hipHostMalloc(&c->h_state, sizeof(DevState), coh) != hipSuccess ||
        hipHostGetDevicePointer((void **)&c->m_state, c->h_state, 0) != hipSuccess)
        return bail(CG_ENOMEM);
    if (hipHostMalloc(&c->h_delta, kDeltaWords * 8, coh) != hipSuccess ||
        hipHostGetDevicePointer((void **)&c->m_delta, c->h_delta, 0) != hipSuccess)
        return bail(CG_ENOMEM);
    if (hipMalloc(&c->d_fill, kFillSlots * kFillCap * sizeof(FillRange)) != hipSuccess) return bail(CG_ENOMEM);
    if (hipHostMalloc(&c->h_fill, kFillSlots * kFillCap * sizeof(FillRange), coh) != hipSuccess ||
        hipHostGetDevicePointer((void **)&c->m_fill, c->h_fill, 0) != hipSuccess)
        return bail(CG_ENOMEM);
    if (hipEventCreateWithFlags(&c->ev_stage, hipEventDisableTiming) != hipSuccess) return bail(CG_EHIP);
    for (auto &e : c->ev_fill)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return bail(CG_EHIP);
    if (hipEventCreateWithFlags(&c->ev_ctx, hipEventDisableTiming) != hipSuccess) return bail(CG_EHIP);
    c->tuning.block = 256;
    c->tuning.unroll = 4;
    c->tuning.blocks_per_cu = 4;
    c->tuning.tile_units = 1u << 16;
    c->tuning.nontemporal = 1;
    if (const char *e = getenv("XC_UNROLL")) c->tuning.unroll = (uint32_t)atoi(e);
    if (const char *e = getenv("XC_BLOCK")) c->tuning.block = (uint32_t)atoi(e);
    if (const char *e = getenv("XC_BLOCKS_PER_CU")) c->tuning.blocks_per_cu = (uint32_t)atoi(e);
    if (const char *e = getenv("XC_TILE_UNITS")) c->tuning.tile_units = (uint32_t)atoi(e);
    if (const char *e = getenv("XC_NONTEMPORAL")) c->tuning.nontemporal = (uint32_t)atoi(e);
    if (const char *e = getenv("XC_REORDER_MIN")) c->reorder_min = strtoull(e, nullptr, 0);
    if (const char *e = getenv("XC_SEG_MIN_LOG2")) c->seg_min_log2 = (uint32_t)atoi(e);
    if (const char *e = getenv("XC_SMALL_MAX")) c->small_max = std::min<uint64_t>(strtoull(e, nullptr, 0), 1ull << 20);
    if (const char *e = getenv("XC_HOST_LDS")) c->host_lds = atoi(e);
    if (const char *e = getenv("XC_TASK_POS")) c->task_pos = std::min<uint32_t>((uint32_t)atoi(e), 256);
    if (const char *e = getenv("XC_PITCHED_2D")) c->pitched_2d = atoi(e) != 0;
    if (const char *e = getenv("XC_SHADOW_INDEX")) c->shadow_index = std::min(std::max(atoi(e), 0), 2);
    if (const char *e = getenv("XC_SIDX_CAP")) c->sidx_cap = std::max<uint64_t>(strtoull(e, nullptr, 0), 1);
    if (const char *e = getenv("XC_SIDX_BLOCKS")) c->sidx_blocks_per_cu = std::min(std::max(atoi(e), 1), 64);
    if (c->seg_min_log2 < 4 || c->seg_min_log2 > 40) return bail(CG_EINVAL);
    if (!valid_tuning(c->tuning)) return bail(CG_EINVAL);
    c->tuning_prop = c->tuning;
    c->tuning_prop.unroll = 2;
    // events that check_transfers_noalloc records, made here so that it makes none
    for (auto &v : c->ver)
        if (hipEventCreateWithFlags(&v.fixed_use, hipEventDisableTiming) != hipSuccess) return bail(CG_EHIP);
    for (int k = 0; k < kPooledEvents; ++k) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return bail(CG_EHIP);
        c->ev_pool.push_back(e);
    }
    if (scratch_setup(c) != CG_OK) return bail(CG_EHIP);
    // an empty table and region, so that checks before any allocation work
    if (materialize(c) != CG_OK) return bail(CG_EHIP);
    if (hipStreamSynchronize(c->s) != hipSuccess) return bail(CG_EHIP);
    *out = c;
    return CG_OK;
}

int cg_destroy(cg_ctx *c)
{
    if (!c) return CG_EINVAL;
    (void)hipSetDevice(c->dev);
    (void)hipDeviceSynchronize();
    for (auto &kv : c->ws) {
        free_ws(kv.second);
        if (kv.second->done) (void)hipEventDestroy(kv.second->done);
        delete kv.second;
    }
    for (auto &kv : c->race_ws) race_release(kv.second);
    for (auto &kv : c->strided_ws) {
        StridedWs &w = kv.second;
        (void)hipFree(w.first);
        (void)hipFree(w.bsum);
        (void)hipFree(w.bshort);
        (void)hipFree(w.total);
        (void)hipFree(w.rows);
        (void)hipFree(w.rec_of);
        (void)hipFree(w.rowv);
        if (w.h_total) (void)hipHostFree(w.h_total);
    }
    for (auto *v : {&c->tpairs, &c->ipairs})
        for (auto &p : *v) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
    (void)hipFree(c->idx_read);
    if (c->s) (void)hipStreamDestroy(c->s);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    (void)hipFree(c->pool);
    for (auto &v : c->ver) {
        (void)hipFree(v.tab);
        (void)hipFree(v.st);
        for (auto &kv : v.uses) (void)hipEventDestroy(kv.second);
        if (v.fixed_use) (void)hipEventDestroy(v.fixed_use);
    }
    for (auto &f : c->inflight) (void)hipEventDestroy(f.ev);
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    (void)hipFree(c->d_delta);
    (void)hipFree(c->m_keep);
    (void)hipFree(c->m_loc);
    (void)hipFree(c->m_bsum);
    (void)hipFree(c->m_boff);
    (void)hipFree(c->d_fill);
    if (c->h_stage) (void)hipHostFree(c->h_stage);
    if (c->h_state) (void)hipHostFree(c->h_state);
    if (c->h_delta) (void)hipHostFree(c->h_delta);
    if (c->h_fill) (void)hipHostFree(c->h_fill);
    if (c->ev_stage) (void)hipEventDestroy(c->ev_stage);
    for (auto e : c->ev_fill)
        if (e) (void)hipEventDestroy(e);
    if (c->ev_ctx) (void)hipEventDestroy(c->ev_ctx);
    delete c->palloc;
    delete c;
    return CG_OK;
}

int cg_host_register(cg_ctx *c, uint64_t host_base, uint64_t len, uint8_t *v_dev, uint64_t *a_bits_dev)
{
    if (!c) return CG_EINVAL;
    if (len == 0 || !v_dev || !a_bits_dev) return fail(c, CG_EINVAL, "host region: null buffer or zero length");
    if (((uint64_t)v_dev & 15u) || ((uint64_t)a_bits_dev & 7u))
        return fail(c, CG_EINVAL, "host region: V must be 16-byte and A 8-byte aligned");
    if (host_base + len < host_base) return fail(c, CG_EINVAL, "host region wraps the address space");
    c->region.hb = host_base;
    c->region.hl = len;
    c->region.v = v_dev;
    c->region.a16 = reinterpret_cast<const uint16_t *>(a_bits_dev);
    c->full_dirty = true;
    return CG_OK;
}

static int alloc_one(cg_ctx *c, uint64_t addr, uint64_t size, std::vector<FillRange> &fills)
{
    int rc = c->table.check_insert(addr, size);
    if (rc == CG_EINVAL) return fail(c, rc, "shadow_alloc: size 0 or range wraps");
    if (rc == CG_EOVERLAP) return fail(c, rc, "shadow_alloc: range intersects a live allocation");
    if (c->table.size() >= c->max_allocs) return fail(c, CG_ECAPACITY, "shadow_alloc: table full");
    uint64_t off;
    retire(c, false);
    if (!c->palloc->alloc(size, &off)) {
        if (c->quarantine.empty()) return fail(c, CG_ENOMEM, "shadow_alloc: shadow pool exhausted");
        retire(c, true);   // wait for the readers of freed blocks
        if (!c->palloc->alloc(size, &off)) return fail(c, CG_ENOMEM, "shadow_alloc: shadow pool exhausted");
    }
    c->table.insert(addr, size, off);
    c->pend_ins[addr] = AllocEntry{size, off};
    add_fill(fills, (uint64_t)c->pool + off, size, 0xFF);
    return CG_OK;
}

int shadow_alloc(cg_ctx *c, uint64_t dev_addr, uint64_t size)
{
    if (!c) return CG_EINVAL;
    std::vector<FillRange> fills;
    int rc = alloc_one(c, dev_addr, size, fills);
    if (rc) return rc;
    return issue_fills(c, fills, false);
}

int shadow_alloc_batch(cg_ctx *c, const uint64_t *addr, const uint64_t *size, uint64_t k)
{
    if (!c || (k && (!addr || !size))) return CG_EINVAL;
    std::vector<FillRange> fills;
    int rc = CG_OK;
    for (uint64_t i = 0; i < k && rc == CG_OK; ++i) rc = alloc_one(c, addr[i], size[i], fills);
    int rc2 = issue_fills(c, fills, false);
    return rc ? rc : rc2;
}

static int free_one(cg_ctx *c, uint64_t addr)
{
    AllocEntry e;
    if (c->table.erase(addr, &e) != CG_OK) return fail(c, CG_ENOTFOUND, "shadow_free: not the base of a live allocation");
    // the block may still be read by checks issued before this free
    c->quarantine.push_back(Quarantined{c->check_seq, e.off, e.size});
    auto it = c->pend_ins.find(addr);
    if (it != c->pend_ins.end()) c->pend_ins.erase(it);   // never reached the device table
    else c->pend_del.insert(addr);
    return CG_OK;
}

int shadow_free(cg_ctx *c, uint64_t dev_addr)
{
    if (!c) return CG_EINVAL;
    return free_one(c, dev_addr);
}

int shadow_free_batch(cg_ctx *c, const uint64_t *addr, uint64_t k)
{
    if (!c || (k && !addr)) return CG_EINVAL;
    for (uint64_t i = 0; i < k; ++i) {
        int rc = free_one(c, addr[i]);
        if (rc) return rc;
    }
    return CG_OK;
}

static int set_one(cg_ctx *c, uint64_t addr, uint64_t n, uint8_t v, std::vector<FillRange> &fills)
{
    if (n == 0) return CG_OK;
    uint64_t base;
    const AllocEntry *e = c->table.find(addr, &base);
    if (!e) return fail(c, CG_ENOTFOUND, "shadow_set: address is in no live allocation");
    if (n > base + e->size - addr) return fail(c, CG_EINVAL, "shadow_set: range leaves the allocation");
    add_fill(fills, (uint64_t)c->pool + e->off + (addr - base), n, v);
    return CG_OK;
}

int shadow_set(cg_ctx *c, uint64_t dev_addr, uint64_t n, uint8_t v)
{
    if (!c) return CG_EINVAL;
    std::vector<FillRange> fills;
    int rc = set_one(c, dev_addr, n, v, fills);
    if (rc) return rc;
    return issue_fills(c, fills, true);
}

int shadow_set_batch(cg_ctx *c, const uint64_t *addr, const uint64_t *n, const uint8_t *v, uint64_t k)
{
    if (!c || (k && (!addr || !n || !v))) return CG_EINVAL;
    std::vector<FillRange> fills;
    int rc = CG_OK;
    for (uint64_t i = 0; i < k && rc == CG_OK; ++i) rc = set_one(c, addr[i], n[i], v[i], fills);
    int rc2 = issue_fills(c, fills, true);
    return rc ? rc : rc2;
}

int shadow_ptr(cg_ctx *c, uint64_t dev_addr, uint8_t **v_dev)
{
    if (!c || !v_dev) return CG_EINVAL;
    uint64_t base;
    const AllocEntry *e = c->table.find(dev_addr, &base);
    if (!e) return fail(c, CG_ENOTFOUND, "shadow_ptr: address is in no live allocation");
    *v_dev = c->pool + e->off + (dev_addr - base);
    return CG_OK;
}

int check_transfers(cg_ctx *c, const cg_transfer *recs_dev, uint64_t count, cg_verdict *out_dev, uint32_t mode,
                    void *hip_stream)
{
    if (!c) return CG_EINVAL;
    if (!(mode & (CG_CHECK | CG_PROPAGATE))) return fail(c, CG_EINVAL, "mode needs CG_CHECK or CG_PROPAGATE");
    if (mode & ~(CG_CHECK | CG_PROPAGATE | CG_PLAIN | CG_DEBUG_CONFLICTS | CG_EAGER | CG_KEEP_ORDER))
        return fail(c, CG_EINVAL, "unknown mode bits");
    if (count == 0) return CG_OK;
    if (!recs_dev) return fail(c, CG_EINVAL, "null records");
    if ((mode & CG_CHECK) && !out_dev) return fail(c, CG_EINVAL, "null verdicts with CG_CHECK");
    // one lane per record in the classify grid, whose size must fit in 32 bits
    if (count > (1ull << 32) - 1024) return fail(c, CG_EINVAL, "at most 2^32 - 1024 records per call");
    if (hipSetDevice(c->dev) != hipSuccess) return fail(c, CG_EHIP, "hipSetDevice");
    return run_check(c, recs_dev, count, out_dev, mode, (hipStream_t)hip_stream,
                     (mode & CG_PROPAGATE) ? c->tuning_prop : c->tuning);
}

int check_transfers_noalloc(cg_ctx *c, const cg_transfer *recs_dev, uint64_t count, cg_verdict *out_dev,
                            uint32_t mode, void *hip_stream)
{
    if (!c) return CG_EINVAL;
    if (!(mode & (CG_CHECK | CG_PROPAGATE))) return fail(c, CG_EINVAL, "mode needs CG_CHECK or CG_PROPAGATE");
    if (mode & ~(CG_CHECK | CG_PROPAGATE | CG_EAGER | CG_KEEP_ORDER))
        return fail(c, CG_EINVAL, "check_transfers_noalloc: mode bits other than CG_CHECK, CG_PROPAGATE, CG_EAGER, "
                                  "CG_KEEP_ORDER");
    if (count > CG_NOALLOC_MAX) return fail(c, CG_EINVAL, "check_transfers_noalloc: more than CG_NOALLOC_MAX records");
    if (count == 0) return CG_OK;
    if (!recs_dev) return fail(c, CG_EINVAL, "null records");
    if ((mode & CG_CHECK) && !out_dev) return fail(c, CG_EINVAL, "null verdicts with CG_CHECK");
    SmallAcc *acc = scratch_of(c->dev);
    if (!acc) return fail(c, CG_ESTATE, "check_transfers_noalloc: no device array for this device");
    if (hipSetDevice(c->dev) != hipSuccess) return fail(c, CG_EHIP, "hipSetDevice");
    const hipStream_t s = (hipStream_t)hip_stream;
    int rc = materialize(c);
    if (rc) return rc;
    HIPTRY(c, hipStreamWaitEvent(s, c->ev_ctx, 0));
    BatchArgs a{};
    a.recs = recs_dev;
    a.count = count;
    a.out = (mode & CG_CHECK) ? out_dev : nullptr;
    a.mode = mode & (CG_CHECK | CG_PROPAGATE);
    a.st = c->ver[c->cur].st;
    const LaunchShape sh = shape_of(c, (mode & CG_PROPAGATE) ? c->tuning_prop : c->tuning);
    HIPTRY(c, launch_small(a, acc, small_bpr(c, count, sh, 0), sh, s));
    return note_use_fixed(c, s);
}

int propagate_shadow(cg_ctx *c, const cg_transfer *recs_dev, uint64_t count, void *hip_stream)
{
    return check_transfers(c, recs_dev, count, nullptr, CG_PROPAGATE, hip_stream);
}

// check_transfers_2d without a wait: every 2D record is one position whose
// units step through its rows (k_classify_2d, then the scan kernel over
// pitched positions); no row count is needed on the host.  Under a caller's
// stream capture only the four kernels are enqueued: the stream must already
// wait for every table upload (an eager call on it since the last change),
// and the bookkeeping events are left out (a replay reads the table of the
// capture's time).
int check_2d_pitched(cg_ctx *c, const cg_transfer2d *recs_dev, uint64_t count, cg_verdict *out_dev, uint32_t mode,
                     hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPTRY(c, hipStreamIsCapturing(s, &cs));
    const bool capturing = cs != hipStreamCaptureStatusNone;
    Workspace *w;
    auto it = c->ws.find(s);
    if (capturing && (it == c->ws.end() || it->second->cap < count || it->second->pitch_cap < it->second->cap))
        return fail(c, CG_ESTATE, "check_transfers_2d under capture: make one call of this size on the stream first");
    int rc = get_ws(c, s, count, &w);
    if (rc) return rc;
    if (w->pitch_cap < w->cap) {
        if (w->pitch) HIPTRY(c, hipStreamSynchronize(s));   // an earlier call on this stream may still read it
        (void)hipFree(w->pitch);
        w->pitch = nullptr;
        w->pitch_cap = 0;
        HIPTRY(c, hipMalloc(&w->pitch, w->cap * sizeof(Pitch)));
        w->pitch_cap = w->cap;
    }
    if (capturing) {
        if (c->full_dirty || !c->pend_del.empty() || !c->pend_ins.empty() || w->ctx_seen != c->ctx_seq)
            return fail(c, CG_ESTATE, "check_transfers_2d under capture: the table changed since the last call on "
                                      "this stream; make one call outside the capture first");
    } else {
        rc = materialize(c);
        if (rc) return rc;
        rc = wait_ctx(c, w, s);
        if (rc) return rc;
    }
    BatchArgs a = make_args(c, w, nullptr, count, out_dev, mode);
    a.pitch = w->pitch;
    const cg_tuning &tun = (mode & CG_PROPAGATE) ? c->tuning_prop : c->tuning;
    const LaunchShape sh = shape_of(c, tun);
    // a check without propagation: records worked as one transfer each (rows
    // back to back) are answered by the shadow indexes when they pay
    const bool idx = c->shadow_index && mode == CG_CHECK;
    if (idx) {
        if (capturing && !w->pidx.state)
            return fail(c, CG_ESTATE, "check_transfers_2d under capture: make one call on this stream first");
        rc = reserve_sidx(c, w);
        if (rc) return rc;
        w->hidx.ratio = w->pidx.ratio = c->shadow_index == 2 ? 0u : c->sidx_ratio;
        set_index_args(a, w);
        HIPTRY(c, launch_sidx_reset(w->hidx, w->pidx, s));
    }
    HIPTRY(c, launch_classify_2d(a, recs_dev, w->pitch, s));
    if (idx) {
        HIPTRY(c, launch_sidx_build(w->hidx, w->pidx, a.st, s));
        HIPTRY(c, launch_sidx_query(a, w->hidx, w->pidx, a.bsum, s, w->pitch));
        HIPTRY(c, launch_reweigh(a, s));
    }
    HIPTRY(c, launch_scan_sums(a, sh.tile_units, sh.grid * (sh.block / 64), s));
    HIPTRY(c, launch_prefix_tiles(a, s));
    if (capturing) {
        HIPTRY(c, launch_batched(a, sh, s));
        return CG_OK;
    }
    TimingPair *tp = c->timing ? next_pair(c) : nullptr;
    if (tp) HIPTRY(c, hipEventRecord(tp->a, s));
    HIPTRY(c, launch_batched(a, sh, s));
    if (tp) HIPTRY(c, hipEventRecord(tp->b, s));
    HIPTRY(c, hipEventRecord(w->done, s));
    w->used = true;
    return note_use(c, s);
}

int check_transfers_2d(cg_ctx *c, const cg_transfer2d *recs_dev, uint64_t count, cg_verdict *out_dev, uint32_t mode,
                       void *hip_stream)
{
    if (!c) return CG_EINVAL;
    if (!(mode & (CG_CHECK | CG_PROPAGATE))) return fail(c, CG_EINVAL, "mode needs CG_CHECK or CG_PROPAGATE");
    if (mode & ~(CG_CHECK | CG_PROPAGATE | CG_PLAIN | CG_DEBUG_CONFLICTS | CG_EAGER | CG_KEEP_ORDER))
        return fail(c, CG_EINVAL, "unknown mode bits");
    if (count == 0) return CG_OK;
    if (!recs_dev) return fail(c, CG_EINVAL, "null records");
    if ((mode & CG_CHECK) && !out_dev) return fail(c, CG_EINVAL, "null verdicts with CG_CHECK");
    if (count >= (1ull << 31)) return fail(c, CG_EINVAL, "at most 2^31 - 1 records per call");
    if (hipSetDevice(c->dev) != hipSuccess) return fail(c, CG_EHIP, "hipSetDevice");
    const hipStream_t s = (hipStream_t)hip_stream;
    // the plain path (a launch per row) and the host-side conflict check need
    // the rows themselves: those modes expand them, after one wait for the count
    if (!(mode & (CG_PLAIN | CG_DEBUG_CONFLICTS)) && c->pitched_2d)
        return check_2d_pitched(c, recs_dev, count, out_dev, mode & (CG_CHECK | CG_PROPAGATE), s);
    StridedWs &w = c->strided_ws[s];
    if (w.rec_cap < count) {
        // the buffers may still be in use by an earlier call on this stream
        HIPTRY(c, hipStreamSynchronize(s));
        (void)hipFree(w.first);
        (void)hipFree(w.bsum);
        (void)hipFree(w.bshort);
        w.first = w.bsum = w.bshort = nullptr;
        w.rec_cap = 0;
        uint64_t cap = 1024;
        while (cap < count) cap <<= 1;
        HIPTRY(c, hipMalloc(&w.first, cap * 8));
        HIPTRY(c, hipMalloc(&w.bsum, (cap / 256 + 1) * 8));
        HIPTRY(c, hipMalloc(&w.bshort, (cap / 256 + 1) * 8));
        if (!w.total) HIPTRY(c, hipMalloc(&w.total, 16));
        if (!w.h_total) HIPTRY(c, hipHostMalloc(&w.h_total, 16, hipHostMallocDefault));
        w.rec_cap = cap;
    }
    HIPTRY(c, launch_2d_prefix(recs_dev, count, w.first, w.bsum, w.bshort, w.total, s));
    HIPTRY(c, hipMemcpyAsync(w.h_total, w.total, 16, hipMemcpyDeviceToHost, s));
    HIPTRY(c, hipStreamSynchronize(s));
    const uint64_t nrows = w.h_total[0], nshort = w.h_total[1];
    if (nrows > (1ull << 32) - 1024) return fail(c, CG_EINVAL, "at most 2^32 - 1024 rows per call");
    if (nrows) {
        if (w.row_cap < nrows) {
            (void)hipFree(w.rows);
            (void)hipFree(w.rec_of);
            (void)hipFree(w.rowv);
            w.rows = nullptr;
            w.rec_of = nullptr;
            w.rowv = nullptr;
            w.row_cap = 0;
            uint64_t cap = 1024;
            while (cap < nrows) cap <<= 1;
            HIPTRY(c, hipMalloc(&w.rows, cap * sizeof(cg_transfer)));
            HIPTRY(c, hipMalloc(&w.rec_of, cap * 4));
            HIPTRY(c, hipMalloc(&w.rowv, cap * sizeof(cg_verdict)));
            w.row_cap = cap;
        }
        HIPTRY(c, launch_2d_expand(recs_dev, w.first, count, nrows, w.rows, w.rec_of, s));
        // the rows keep their order (each record's rows ascend in memory):
        // cutting millions of short rows into source-block segments costs
        // more than the cache reuse it could bring
        // mostly short rows (16 KiB or less) are checked with more waves in
        // flight and a shorter loop: their work per row is latency, not bytes
        cg_tuning tun = (mode & CG_PROPAGATE) ? c->tuning_prop : c->tuning;
        if (!(mode & CG_PROPAGATE) && 2 * nshort >= nrows) tun = kShortRowTuning;
        const int rc = run_check(c, w.rows, nrows, (mode & CG_CHECK) ? w.rowv : nullptr, mode | CG_KEEP_ORDER, s, tun);
        if (rc) return rc;
    }
    if (mode & CG_CHECK) HIPTRY(c, launch_2d_fold(recs_dev, w.first, count, w.rec_of, w.rowv, nrows, out_dev, s));
    return CG_OK;
}

int check_pointers(cg_ctx *c, const uint64_t *ptrs_dev, uint64_t count, cg_ptr_check *out_dev, void *hip_stream)
{
    if (!c) return CG_EINVAL;
    if (count == 0) return CG_OK;
    if (!ptrs_dev || !out_dev) return fail(c, CG_EINVAL, "null pointers or results");
    if (count >= (1ull << 31)) return fail(c, CG_EINVAL, "at most 2^31 - 1 pointers per call");
    if (hipSetDevice(c->dev) != hipSuccess) return fail(c, CG_EHIP, "hipSetDevice");
    const hipStream_t s = (hipStream_t)hip_stream;
    int rc = materialize(c);
    if (rc) return rc;
    HIPTRY(c, hipStreamWaitEvent(s, c->ev_ctx, 0));
    HIPTRY(c, launch_pointers(c->ver[c->cur].st, ptrs_dev, count, out_dev, s));
    return note_use(c, s);
}

int check_concurrent(cg_ctx *c, const cg_transfer *recs_dev, const uint32_t *streams_dev, const uint32_t *epochs_dev,
                     uint64_t count, cg_race *out_dev, void *hip_stream)
{
    if (!c) return CG_EINVAL;
    if (count == 0) return CG_OK;
    if (!recs_dev || !streams_dev || !out_dev) return fail(c, CG_EINVAL, "null records, streams or results");
    if (count > (1ull << 30)) return fail(c, CG_EINVAL, "at most 2^30 records per join");
    if (hipSetDevice(c->dev) != hipSuccess) return fail(c, CG_EHIP, "hipSetDevice");
    const hipStream_t s = (hipStream_t)hip_stream;
    RaceWs &w = c->race_ws[s];
    if (w.cap < 2 * count) {
        // the buffers may still be read by an earlier join on this stream
        HIPTRY(c, hipStreamSynchronize(s));
        uint64_t cap = 1u << 12;
        while (cap < 2 * count) cap <<= 1;
        const hipError_t e = race_reserve(w, cap);
        if (e == hipErrorOutOfMemory) return fail(c, CG_ENOMEM, "join work space");
        if (e != hipSuccess) return fail(c, CG_EHIP, std::string("join work space: ") + hipGetErrorString(e));
    }
    const hipError_t e = race_launch(w, recs_dev, streams_dev, epochs_dev, count, out_dev, s);
    if (e != hipSuccess) return fail(c, CG_EHIP, std::string("join launch: ") + hipGetErrorString(e));
    return CG_OK;
}

int cg_sync(cg_ctx *c)
{
    if (!c) return CG_EINVAL;
    HIPTRY(c, hipStreamSynchronize(c->s));
    return CG_OK;
}

int cg_stats(cg_ctx *c, uint64_t *live, uint64_t *used)
{
    if (!c) return CG_EINVAL;
    if (live) *live = c->table.size();
    if (used) *used = c->palloc->used();
    return CG_OK;
}

int cg_table_read(cg_ctx *c, uint64_t *base, uint64_t *end, uint64_t *off, uint64_t cap, uint64_t *n, uint64_t *top,
                  uint32_t top_cap, uint32_t *ntop, uint32_t *shift, uint64_t *pool, uint64_t *merges,
                  uint64_t *full_uploads)
{
    if (!c || !base || !end || !off || !n || !top || !ntop || !shift) return CG_EINVAL;
    int rc = ctx_begin(c);
    if (!rc) rc = materialize(c);
    if (rc) return rc;
    const TableVersion &v = c->ver[c->cur];
    const DevState &st = *c->h_state;
    const uint64_t M = c->max_allocs;
    if (v.n > cap || st.table.ntop > top_cap) return fail(c, CG_EINVAL, "cg_table_read: buffers too small");
    HIPTRY(c, hipStreamSynchronize(c->s));
    if (v.n) {
        HIPTRY(c, hipMemcpy(base, v.tab, v.n * 8, hipMemcpyDeviceToHost));
        HIPTRY(c, hipMemcpy(end, v.tab + M, v.n * 8, hipMemcpyDeviceToHost));
        HIPTRY(c, hipMemcpy(off, v.tab + 2 * M, v.n * 8, hipMemcpyDeviceToHost));
        HIPTRY(c, hipMemcpy(top, v.tab + 3 * M, st.table.ntop * 8ull, hipMemcpyDeviceToHost));
    }
    *n = v.n;
    *ntop = v.n ? st.table.ntop : 0;
    *shift = st.table.top_shift;
    if (pool) *pool = (uint64_t)c->pool;
    if (merges) *merges = c->merges;
    if (full_uploads) *full_uploads = c->full_uploads;
    return CG_OK;
}

int cg_get_tuning(cg_ctx *c, cg_tuning *t)
{
    if (!c || !t) return CG_EINVAL;
    *t = c->tuning;
    return CG_OK;
}

int cg_set_tuning(cg_ctx *c, const cg_tuning *t)
{
    if (!c || !t) return CG_EINVAL;
    if (!valid_tuning(*t)) return fail(c, CG_EINVAL, "tuning out of range");
    c->tuning = *t;
    c->tuning_prop = *t;
    return CG_OK;
}

int cg_timing(cg_ctx *c, int enable)
{
    if (!c) return CG_EINVAL;
    c->timing = enable != 0;
    return CG_OK;
}

int cg_kernel_ms(cg_ctx *c, double *ms, uint64_t *launches)
{
    if (!c || !ms) return CG_EINVAL;
    double sum = 0;
    for (size_t i = 0; i < c->tused; ++i) {
        HIPTRY(c, hipEventSynchronize(c->tpairs[i].b));
        float x = 0;
        HIPTRY(c, hipEventElapsedTime(&x, c->tpairs[i].a, c->tpairs[i].b));
        sum += x;
    }
    *ms = sum;
    if (launches) *launches = c->tused;
    c->tused = 0;
    return CG_OK;
}

int cg_index_ms(cg_ctx *c, double *ms, uint64_t *launches, uint64_t *bytes)
{
    if (!c || !ms) return CG_EINVAL;
    double sum = 0;
    for (size_t i = 0; i < c->iused; ++i) {
        HIPTRY(c, hipEventSynchronize(c->ipairs[i].b));
        float x = 0;
        HIPTRY(c, hipEventElapsedTime(&x, c->ipairs[i].a, c->ipairs[i].b));
        sum += x;
    }
    *ms = sum;
    if (launches) *launches = c->iused;
    c->iused = 0;
    if (bytes) {
        bytes[0] = bytes[1] = 0;
        if (c->idx_read) {
            if (hipSetDevice(c->dev) != hipSuccess) return fail(c, CG_EHIP, "hipSetDevice");
            HIPTRY(c, hipDeviceSynchronize());
            HIPTRY(c, hipMemcpy(bytes, c->idx_read, 2 * 8, hipMemcpyDeviceToHost));
            HIPTRY(c, hipMemset(c->idx_read, 0, 2 * 8));
        }
    }
    return CG_OK;
}

int cg_autotune(cg_ctx *c, const cg_transfer *recs_dev, uint64_t count, cg_verdict *out_dev, uint32_t mode,
                void *hip_stream, const char *cache_path, cg_tuning *best)
{
    if (!c || !recs_dev || !count) return CG_EINVAL;
    if ((mode & CG_CHECK) && !out_dev) return CG_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    const uint32_t keep = mode & CG_KEEP_ORDER;
    mode &= (CG_CHECK | CG_PROPAGATE);
    if (!mode) return CG_EINVAL;
    // the batch is worked as source-block segments unless kept (as run_check decides)
    const bool reordered = segmented(c, count, mode | keep);
    cg_tuning &target = (mode & CG_PROPAGATE) ? c->tuning_prop : c->tuning;
    // workload signature: count and log2 of the total units, from a first run
    const bool was_timing = c->timing;
    c->timing = true;
    c->tused = 0;
    int rc = run_check(c, recs_dev, count, out_dev, mode | CG_EAGER | keep, s, target);
    if (rc) { c->timing = was_timing; return rc; }
    HIPTRY(c, hipStreamSynchronize(s));
    c->tused = 0;
    c->iused = 0;
    Ctl ctl;
    HIPTRY(c, hipMemcpy(&ctl, c->ws[s]->ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    if (ctl.total_units <= count) {
        // no record left to scan (the shadow indexes answered them, or they
        // are empty): the launch shape does not matter; keep it
        c->timing = was_timing;
        if (best) *best = target;
        return CG_OK;
    }
    uint32_t lg = 0;
    while ((1ull << lg) < ctl.total_units) ++lg;
    std::ostringstream key;
    key << c->arch << "/cu" << c->cu_count << "/n" << count << "/u2^" << lg << "/m" << mode << (reordered ? "/o" : "");
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            if (line.find("\"key\": \"" + key.str() + "\"") == std::string::npos) continue;
            cg_tuning t = target;
            if (parse_field(line, "block", &t.block) && parse_field(line, "unroll", &t.unroll) &&
                parse_field(line, "blocks_per_cu", &t.blocks_per_cu) && parse_field(line, "tile_units", &t.tile_units) &&
                parse_field(line, "nontemporal", &t.nontemporal) && valid_tuning(t)) {
                target = t;
                c->timing = was_timing;
                if (best) *best = t;
                return CG_OK;
            }
        }
    }
    auto measure = [&](const cg_tuning &t, double *ms) -> int {
        double sum = 0;
        for (int rep = 0; rep < 3; ++rep) {
            int r = run_check(c, recs_dev, count, out_dev, mode | CG_EAGER | keep, s, t);
            if (r) return r;
            double x;
            uint64_t l;
            r = cg_kernel_ms(c, &x, &l);
            if (r) return r;
            if (rep) sum += x;   // first run warms caches / code
        }
        *ms = sum / 2;
        return CG_OK;
    };
    cg_tuning cur = target;
    double cur_ms;
    rc = measure(cur, &cur_ms);
    if (rc) { c->timing = was_timing; return rc; }
    auto try_set = [&](std::vector<cg_tuning> cands) -> int {
        for (const auto &t : cands) {
            if (!valid_tuning(t) || same_tuning(t, cur)) continue;
            double ms;
            int r = measure(t, &ms);
            if (r) return r;
            if (ms < cur_ms) { cur = t; cur_ms = ms; }
        }
        return CG_OK;
    };
    std::vector<cg_tuning> cands;
    for (uint32_t u : {2u, 4u, 8u})
        for (uint32_t nt : {0u, 1u}) { cg_tuning t = cur; t.unroll = u; t.nontemporal = nt; cands.push_back(t); }
    rc = try_set(cands);
    if (!rc) {
        cands.clear();
        for (uint32_t b : {256u, 512u})
            for (uint32_t bpc : {1u, 2u, 3u, 4u, 6u, 8u}) {
                cg_tuning t = cur;
                t.block = b;
                t.blocks_per_cu = bpc;
                cands.push_back(t);
            }
        rc = try_set(cands);
    }
    if (!rc) {
        cands.clear();
        for (uint32_t tu : {1u << 12, 1u << 13, 1u << 14, 1u << 15, 1u << 16, 1u << 18}) {
            cg_tuning t = cur;
            t.tile_units = tu;
            cands.push_back(t);
        }
        rc = try_set(cands);
    }
    if (!rc) {
        // the occupancy that suits a tile size may differ from the first pick
        cands.clear();
        for (uint32_t b : {256u, 512u})
            for (uint32_t bpc : {1u, 2u, 3u, 4u, 6u, 8u}) {
                cg_tuning t = cur;
                t.block = b;
                t.blocks_per_cu = bpc;
                cands.push_back(t);
            }
        rc = try_set(cands);
    }
    if (!rc) {
        // batches of short records are per-record latency: many waves with a
        // short loop can beat deep unrolling (measured on 4 KiB rows: -20 %)
        cands.clear();
        for (uint32_t u : {1u, 2u})
            for (uint32_t bpc : {8u, 16u}) {
                cg_tuning t = cur;
                t.block = 256;
                t.unroll = u;
                t.blocks_per_cu = bpc;
                cands.push_back(t);
            }
        rc = try_set(cands);
    }
    c->timing = was_timing;
    if (rc) return rc;
    target = cur;
    if (best) *best = cur;
    if (cache_path) {
        std::ofstream o(cache_path, std::ios::app);
        o << "{\"key\": \"" << key.str() << "\", " << tuning_json(cur) << ", \"ms\": " << cur_ms << "}\n";
    }
    return CG_OK;
}

int cg_probe_read(const void *dev, uint64_t bytes, uint64_t *sink_dev, void *hip_stream)
{
    if (!dev || !sink_dev || (bytes & 15u) || ((uint64_t)dev & 15u)) return CG_EINVAL;
    return launch_probe_read(dev, bytes, sink_dev, (hipStream_t)hip_stream) == hipSuccess ? CG_OK : CG_EHIP;
}

int cg_probe_l2(const void *dev, uint64_t slice_bytes, uint32_t passes, uint32_t blocks, uint64_t *sink_dev,
                void *hip_stream)
{
    if (!dev || !sink_dev || ((uint64_t)dev & 15u) || slice_bytes < 16384 || (slice_bytes & 16383u) || passes == 0 ||
        blocks == 0)
        return CG_EINVAL;
    return launch_probe_l2(dev, slice_bytes, passes, blocks, sink_dev, (hipStream_t)hip_stream) == hipSuccess ? CG_OK
                                                                                                           : CG_EHIP;
}

int cg_probe_copy(void *dst, const void *src, uint64_t bytes, void *hip_stream)
{
    if (!dst || !src || (bytes & 15u) || ((uint64_t)dst & 15u) || ((uint64_t)src & 15u)) return CG_EINVAL;
    return launch_probe_copy(dst, src, bytes, (hipStream_t)hip_stream) == hipSuccess ? CG_OK : CG_EHIP;
}

}  // extern "C"

// ===========================================================================
// serving loop
// ===========================================================================
namespace {

struct Slot {
    hipStream_t s = nullptr;
    cg_transfer *d_recs = nullptr, *h_recs = nullptr;
    cg_verdict *d_out = nullptr, *h_out = nullptr;
    // the device's addresses of h_recs / h_out (coherent host memory): a
    // micro-batch worked in one launch reads its records and writes its
    // verdicts there, with no copy on either side
    cg_transfer *m_recs = nullptr;
    cg_verdict *m_out = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    uint64_t bytes = 0;
    uint32_t filled = 0;                // records written in h_recs (rest padded)
    std::vector<uint64_t> reqs;         // result indices of the batch
};

// algorithmic shadow bytes of a request: V bytes plus, for a host side, its A bits
uint64_t footprint(const cg_transfer &r)
{
    return r.kind == CG_D2D ? r.n : r.n + (r.n + 7) / 8;
}

void free_slots(std::vector<Slot> &slots)
{
    for (auto &sl : slots) {
        if (sl.s) (void)hipStreamSynchronize(sl.s);
        (void)hipFree(sl.d_recs);
        (void)hipFree(sl.d_out);
        if (sl.h_recs) (void)hipHostFree(sl.h_recs);
        if (sl.h_out) (void)hipHostFree(sl.h_out);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.s) (void)hipStreamDestroy(sl.s);
    }
}

}  // namespace

// Before the clock starts: the slot's workspace and one captured graph per
// table version of the ring, so that no allocation or capture happens while
// requests wait.
int prewarm(cg_ctx *c, hipStream_t s, const cg_transfer *recs, uint64_t count, cg_verdict *out, const cg_tuning &tun)
{
    Workspace *w;
    int rc = get_ws(c, s, count, &w);
    if (rc) return rc;
    // micro-batches of this size run in one launch: run it once on the
    // padding records (bad kinds), so that its code is on the device
    if (count <= c->small_max) return run_check(c, recs, count, out, CG_CHECK | CG_KEEP_ORDER, s, tun, 1);
    const LaunchShape sh = shape_of(c, tun);
    for (int v = 0; v < kVersions && !rc; ++v) {
        BatchArgs a = make_args(c, w, recs, count, out, CG_CHECK);
        a.st = c->ver[v].st;
        GraphEntry *ge;
        rc = find_graph(c, w, a, nullptr, sh, tun, false, s, &ge);
    }
    return rc;
}

extern "C" int cg_serve_run(cg_ctx *c, const cg_serve_event *ev, uint64_t n, const cg_serve_config *cfg,
                            cg_serve_result *res, cg_serve_stats *stats)
{
    if (!c || (n && (!ev || !res)) || !cfg) return CG_EINVAL;
    const uint32_t S = cfg->plain ? 1u : cfg->streams;
    const uint32_t B = cfg->plain ? 1u : cfg->max_batch;
    if (S < 1 || S > 16 || B < 1 || B > 65536 || cfg->mem_cap == 0) return fail(c, CG_EINVAL, "serve: bad config");
    HIPTRY(c, hipSetDevice(c->dev));
    cg_tuning tun = c->tuning;
    tun.blocks_per_cu = cfg->blocks_per_cu ? cfg->blocks_per_cu : 1;
    if (!valid_tuning(tun)) return fail(c, CG_EINVAL, "serve: bad blocks_per_cu");

    std::vector<Slot> slots(S);
    auto bail = [&](int rc) { free_slots(slots); return rc; };
    for (auto &sl : slots) {
        if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess ||
            hipMalloc(&sl.d_recs, B * sizeof(cg_transfer)) != hipSuccess ||
            hipMalloc(&sl.d_out, B * sizeof(cg_verdict)) != hipSuccess ||
            hipHostMalloc(&sl.h_recs, B * sizeof(cg_transfer), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
            hipHostMalloc(&sl.h_out, B * sizeof(cg_verdict), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
            hipHostGetDevicePointer((void **)&sl.m_recs, sl.h_recs, 0) != hipSuccess ||
            hipHostGetDevicePointer((void **)&sl.m_out, sl.h_out, 0) != hipSuccess ||
            hipEventCreate(&sl.done) != hipSuccess)
            return bail(fail(c, CG_ENOMEM, "serve: slot buffers"));
        for (uint32_t k = 0; k < B; ++k) sl.h_recs[k] = cg_transfer{0, 0, 0, 0xFFFFFFFFu, 0};
        sl.filled = B;
        if (hipMemcpy(sl.d_recs, sl.h_recs, B * sizeof(cg_transfer), hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(c, CG_EHIP, "serve: slot records"));
    }
    {
        // the table as it stands now, and the code of every kernel the loop
        // launches, are on the device before the clock starts
        int rc0 = materialize(c);
        if (!rc0 && launch_merge_warm(c->s) != hipSuccess) rc0 = fail(c, CG_EHIP, "serve: warm-up launch");
        for (auto &sl : slots)
            if (!rc0 && !cfg->plain) rc0 = prewarm(c, sl.s, sl.d_recs, B, sl.d_out, tun);
        if (!rc0 && hipStreamSynchronize(c->s) != hipSuccess) rc0 = fail(c, CG_EHIP, "serve: warm-up sync");
        if (rc0) return bail(rc0);
    }
    // result index of every check event
    std::vector<uint64_t> ridx(n);
    uint64_t nreq = 0;
    for (uint64_t i = 0; i < n; ++i) ridx[i] = ev[i].type == CG_EV_CHECK ? nreq++ : ~0ull;

    // Completion times are GPU event times after ev0; arrival times are host
    // times after T0.  Every slot stream has run a command before (so no
    // first-use set-up delays ev0), and T0 is taken once the device has
    // executed ev0: the device clock cannot start after the host clock, and
    // a latency is at most overstated by the few microseconds of that wait.
    for (auto &sl : slots)
        if (hipEventRecord(sl.done, sl.s) != hipSuccess || hipEventSynchronize(sl.done) != hipSuccess)
            return bail(fail(c, CG_EHIP, "serve: stream warm-up"));
    hipEvent_t ev0;
    if (hipEventCreate(&ev0) != hipSuccess) return bail(fail(c, CG_EHIP, "serve: event"));
    using clk = std::chrono::steady_clock;
    if (hipEventRecord(ev0, slots[0].s) != hipSuccess || hipEventSynchronize(ev0) != hipSuccess) {
        (void)hipEventDestroy(ev0);
        return bail(fail(c, CG_EHIP, "serve: clock start"));
    }
    const auto T0 = clk::now();
    auto now = [&] { return std::chrono::duration<double>(clk::now() - T0).count(); };

    std::deque<uint64_t> fifo;
    uint64_t next = 0, epoch = 0, batches = 0, nevents = 0, admitted = 0;
    uint64_t inflight = 0, max_inflight = 0;   // exact integers: the loop waits for zero
    const uint64_t versions0 = c->versions_made;
    int rc = CG_OK;
    double last_progress = 0;
    while (rc == CG_OK) {
        bool progress = false;
        const double t = now();
        while (next < n && (!cfg->open_loop || ev[next].t <= t)) {
            if (ev[next].type == CG_EV_CHECK) res[ridx[next]].t_arrive = cfg->open_loop ? ev[next].t : 0.0;
            fifo.push_back(next++);
            progress = true;
        }
        // finished micro-batches
        for (uint32_t k = 0; k < S; ++k) {
            Slot &sl = slots[k];
            if (!sl.busy || hipEventQuery(sl.done) != hipSuccess) continue;
            float ms = 0;
            (void)hipEventElapsedTime(&ms, ev0, sl.done);
            for (size_t q = 0; q < sl.reqs.size(); ++q) {
                res[sl.reqs[q]].v = sl.h_out[q];
                res[sl.reqs[q]].t_done = ms / 1e3;
            }
            inflight -= sl.bytes;
            sl.busy = false;
            progress = true;
        }
        // allocation events at the head apply at once: every request before
        // them has been issued already
        while (!fifo.empty() && ev[fifo.front()].type != CG_EV_CHECK) {
            const cg_serve_event &e = ev[fifo.front()];
            if (e.type == CG_EV_ALLOC) {
                std::vector<FillRange> fills;
                rc = alloc_one(c, e.rec.dst, e.rec.n, fills);
                if (!rc) rc = issue_fills(c, fills, false);
            } else if (e.type == CG_EV_FREE) {
                rc = free_one(c, e.rec.dst);
            } else {
                rc = fail(c, CG_EINVAL, "serve: unknown event type");
            }
            if (rc) break;
            ++epoch;
            ++nevents;
            fifo.pop_front();
            progress = true;
        }
        if (rc) break;
        // continuous batching into free slots
        for (uint32_t k = 0; k < S && !fifo.empty() && rc == CG_OK; ++k) {
            Slot &sl = slots[k];
            if (sl.busy || ev[fifo.front()].type != CG_EV_CHECK) continue;
            sl.reqs.clear();
            uint64_t bytes = 0;
            while (!fifo.empty() && sl.reqs.size() < B) {
                const cg_serve_event &e = ev[fifo.front()];
                if (e.type != CG_EV_CHECK) break;
                const uint64_t fp = footprint(e.rec);
                // admit while under the cap; a request alone in flight is always admitted
                if (inflight + bytes + fp > cfg->mem_cap && inflight + bytes > 0) break;
                const uint64_t r = ridx[fifo.front()];
                sl.h_recs[sl.reqs.size()] = e.rec;
                res[r].epoch = epoch;
                res[r].batch = (uint32_t)batches;
                res[r].slot = k;
                sl.reqs.push_back(r);
                bytes += fp;
                fifo.pop_front();
            }
            if (sl.reqs.empty()) break;   // admission cap reached
            const uint32_t cnt = (uint32_t)sl.reqs.size();
            for (uint32_t q = cnt; q < sl.filled; ++q) sl.h_recs[q] = cg_transfer{0, 0, 0, 0xFFFFFFFFu, 0};
            sl.filled = cnt;
            const double ta = now();
            for (uint64_t r : sl.reqs) res[r].t_admit = ta;
            // graph shape: a fixed count, padded; micro-batches that run in one
            // launch take their own count
            const bool one_launch = !cfg->plain && B <= c->small_max;
            const uint32_t count = cfg->plain || one_launch ? cnt : B;
            hipError_t e1 = hipSuccess;
            if (one_launch) {
                // the launch reads the records from, and writes the verdicts
                // to, the slot's coherent host memory, with as many blocks per
                // record as the largest of them uses
                uint32_t bpr = 1;
                for (uint32_t q = 0; q < cnt; ++q) {
                    const cg_transfer &r = sl.h_recs[q];
                    const uint64_t most = r.kind <= CG_D2D && r.n ? r.n / 16 + 2 : 1;
                    const uint64_t nb = (most + kSmallUnits - 1) / kSmallUnits;
                    bpr = nb > bpr ? (uint32_t)std::min<uint64_t>(nb, 1u << 20) : bpr;
                }
                // its completion event right behind the launch
                rc = run_check(c, sl.m_recs, count, sl.m_out, CG_CHECK | CG_KEEP_ORDER, sl.s, tun, bpr, sl.done);
                if (rc) break;
            } else {
                e1 = hipMemcpyAsync(sl.d_recs, sl.h_recs, count * sizeof(cg_transfer), hipMemcpyHostToDevice, sl.s);
                if (e1 != hipSuccess) { rc = hip_fail(c, "serve: records upload", e1); break; }
                // micro-batches keep their order (their graphs are captured before the clock starts)
                rc = run_check(c, sl.d_recs, count, sl.d_out, CG_CHECK | CG_KEEP_ORDER | (cfg->plain ? CG_PLAIN : 0u),
                               sl.s, tun);
                if (rc) break;
                e1 = hipMemcpyAsync(sl.h_out, sl.d_out, cnt * sizeof(cg_verdict), hipMemcpyDeviceToHost, sl.s);
                if (e1 == hipSuccess) e1 = hipEventRecord(sl.done, sl.s);
            }
            if (e1 != hipSuccess) { rc = hip_fail(c, "serve: verdict download", e1); break; }
            sl.busy = true;
            sl.bytes = bytes;
            inflight += bytes;
            max_inflight = std::max(max_inflight, inflight);
            admitted += cnt;
            ++batches;
            progress = true;
        }
        if (rc) break;
        bool any_busy = false;
        for (auto &sl : slots) any_busy |= sl.busy;
        if (next == n && fifo.empty() && !any_busy) break;
        if (progress) {
            last_progress = t;
        } else {
            // requests wait only for the next arrival or for a batch on the GPU
            const bool waiting_arrival = fifo.empty() && next < n;
            if (!waiting_arrival && t - last_progress > 120.0) {
                rc = fail(c, CG_EHIP, "serve: no micro-batch finished for 120 s");
                break;
            }
            std::this_thread::yield();
        }
    }
    const double wall = now();
    if (rc) {
        for (auto &sl : slots) (void)hipStreamSynchronize(sl.s);
    }
    (void)hipEventDestroy(ev0);
    free_slots(slots);
    if (stats) {
        stats->wall_s = wall;
        stats->requests = admitted;
        stats->batches = batches;
        stats->events = nevents;
        stats->max_inflight_bytes = max_inflight;
        stats->table_versions = c->versions_made - versions0;
        stats->mean_batch = batches ? (double)admitted / batches : 0;
    }
    return rc;
}
