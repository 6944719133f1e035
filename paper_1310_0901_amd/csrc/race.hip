// Concurrent-access detection over a batch of transfer records (gfx950).
//
// Sec. 2 counts some concurrent accesses, in programs that use several
// threads, among the errors a checker reports; the paper gives no mechanism.
// Here each record reads [src, src + n) and writes [dst, dst + n) of the
// process's one address space, and carries the stream it was issued on and an
// epoch (the synchronising calls made before it).  Two records conflict when
// they share the epoch, run on different streams, and a written range of one
// meets a read or written range of the other.  Any 64-bit address, any length
// and any 32-bit epoch is decided; ranges are integer ranges that do not wrap.
//
// The join is an interval sweep.  Every record gives two intervals, ordered
// by (epoch, first byte).  The order comes from two stable passes of the
// 8-bit LSD radix sort of sort.hip, which skips a pass whose digit is the same
// in every key: the first sorts on the 64-bit first byte, the second on the
// 32-bit epoch.  When the epochs never decrease in record order, no epoch
// spans more than 4,096 records and they average at least 256 (a program's
// synchronisation windows), each epoch's intervals are instead sorted in LDS
// by one block, in place, and the global passes all skip.  An interval then
// meets an interval of another stream that starts no later exactly when the
// furthest last byte among earlier intervals of other streams of its epoch
// reaches its first byte, and one that starts later exactly when the smallest
// first byte among later intervals of other streams of its epoch reaches no
// further than its last.  Comparing (epoch, byte) pairs keeps the epochs
// apart without a segmented scan.  "Best among other streams" is kept as the
// best two entries of distinct streams; that combine is associative and
// commutative, so both directions are one reduce-then-scan over tiles.
#include <hip/hip_runtime.h>

#include "race.h"
#include "sort.h"

namespace xc {
namespace {

constexpr uint32_t kNoRec = 0xFFFFFFFFu;
constexpr uint32_t kNoStream = 0xFFFFFFFFu;
constexpr uint32_t kDead = 0x80000000u;         // interval-id bit: the interval touches no byte
constexpr uint64_t kHere = 1ull << 32;          // high word of every real sweep value (none is 0)

constexpr int kT = 256;                          // threads per block
constexpr int kWaves = kT / 64;
constexpr int kSweepItems = 8;                   // consecutive elements per thread
constexpr uint32_t kRunMax = 4096;               // records of one epoch sorted in LDS, at most
constexpr int kLocalN = 2 * kRunMax;             // their intervals
constexpr int kLT = 1024;                        // threads of the per-epoch sort
constexpr int kLWaves = kLT / 64;
constexpr int kLRounds = kLocalN / kLT;          // elements per thread
constexpr uint64_t kRunMean = 256;               // records per epoch, on average at least
constexpr int kSweepTile = kT * kSweepItems;
static_assert(kT == kSortKeyBlock, "one part of the key mask per block of k_race_keys");

// ---- records -------------------------------------------------------------

__device__ __forceinline__ bool rec_checked(const cg_transfer &t) { return t.kind <= CG_D2D; }

// Interval i of record i / 2: the source range for even i, the destination
// range for odd i, as its first and last byte.  A range that runs past 2^64
// is cut at 2^64 - 1: two ranges that meet above it both hold that byte, so
// no meeting is lost or added.  `live` is false when it touches no byte.
struct Iv {
    uint64_t first, last;
    bool live;
};

__device__ __forceinline__ Iv interval_of(const cg_transfer &t, uint64_t i)
{
    Iv v;
    v.first = (i & 1) ? t.dst : t.src;
    v.live = rec_checked(t) && t.n > 0;
    v.last = v.live && t.n - 1 <= ~v.first ? v.first + (t.n - 1) : ~0ull;
    return v;
}

// first pass keys: every interval's first byte (dead ones too, where they
// land does not matter), its id with kDead when it touches nothing
__global__ __launch_bounds__(kT) void k_race_keys(const cg_transfer *recs, uint64_t m, uint64_t *keys, uint32_t *vals,
                                                  uint64_t *parts, uint32_t *flag)
{
    __shared__ uint64_t part[kWaves];
    const uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (i == 0) {
        flag[0] = 0;
        flag[1] = 0;
    }
    const uint64_t k0 = recs[0].src;
    uint64_t x = 0;
    if (i < m) {
        const Iv v = interval_of(recs[i >> 1], i);
        keys[i] = v.first;
        vals[i] = (uint32_t)i | (v.live ? 0u : kDead);
        x = v.first ^ k0;
    }
    for (int d = 32; d >= 1; d >>= 1) x |= __shfl_xor(x, d);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t y = 0;
        for (int w = 0; w < kWaves; ++w) y |= part[w];
        parts[blockIdx.x] = y;
    }
}

// ---- per-epoch sort --------------------------------------------------------

// flag[0] becomes non-zero unless the epochs never decrease and no epoch
// spans more than kRunMax records (equal epochs kRunMax records apart mean a
// longer one, since they never decrease); flag[1] counts the epochs.  Without
// epochs all records are one epoch.
__global__ __launch_bounds__(kT) void k_race_local_check(const uint32_t *epochs, uint64_t count, uint32_t *flag)
{
    const uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x;
    bool bad = false, start = false;
    if (i < count) {
        start = i == 0 || (epochs && epochs[i] != epochs[i - 1]);
        if (!epochs) bad = i == 0 && count > kRunMax;
        else bad = (i > 0 && epochs[i] < epochs[i - 1]) || (i >= kRunMax && epochs[i] == epochs[i - kRunMax]);
    }
    const uint64_t b = __ballot(bad), st = __ballot(start);
    if ((threadIdx.x & 63) == 0) {
        if (b) atomicOr(&flag[0], 1u);
        if (st) atomicAdd(&flag[1], (uint32_t)__popcll(st));
    }
}

// the per-epoch path applies: see k_race_local_check
__device__ __forceinline__ bool local_path(const uint32_t *flag, uint64_t count)
{
    return flag[0] == 0 && (uint64_t)flag[1] * kRunMean <= count;
}

// One block per chunk of kRunMax records sorts, in place, the intervals of
// every epoch that starts in the chunk (at most kRunMax records, so at most
// kLocalN intervals) by first byte, with a stable LSD radix sort in LDS and
// 8-bit digits: each key travels with its index in the epoch's run, element
// e of the run sits in wave e / 512, round (e / 64) % 8, lane e % 64, ranks
// come from ballots as in the global sort, and a pass whose digit is the same
// in every key is skipped.  Dead intervals sort by their address like the
// others; the sweep skips them wherever they are.  The chunk's parts of the
// key mask are cleared, so every pass of both global sorts skips.  The
// write-back leaves what the sweep reads: the epoch as the key, the interval
// id, and in the spare buffers and `first` each interval's last byte, stream
// and first byte (k_race_gather fills them on the global path).
__global__ __launch_bounds__(kLT) void k_race_local_sort(uint64_t *keys, uint32_t *vals, uint64_t *ends,
                                                         uint32_t *strm, uint64_t *first, uint64_t *parts,
                                                         uint64_t nparts, const cg_transfer *recs,
                                                         const uint32_t *streams, const uint32_t *epochs,
                                                         uint64_t count, const uint32_t *flag)
{
    __shared__ uint64_t buf[kLocalN];
    __shared__ uint16_t bix[kLocalN];
    __shared__ uint32_t wrun[kLWaves][256];   // per wave and digit: running count, then prefix over waves
    __shared__ uint32_t dstart[256];
    __shared__ uint32_t wtot[kLWaves];
    __shared__ uint64_t wor[kLWaves];
    __shared__ uint32_t starts[kRunMax];
    __shared__ uint32_t nstarts, run_len;
    if (!local_path(flag, count)) return;   // the whole grid leaves: the global sort runs
    const uint32_t w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const uint64_t c0 = (uint64_t)blockIdx.x * kRunMax;
    const uint64_t c1 = c0 + kRunMax < count ? c0 + kRunMax : count;
    // parts cover 128 records each; the chunks tile the records, so every part is cleared once
    const uint64_t p1 = (c1 + 127) / 128 < nparts ? (c1 + 127) / 128 : nparts;
    for (uint64_t b = c0 / 128 + threadIdx.x; b < p1; b += kLT) parts[b] = 0;
    if (threadIdx.x == 0) nstarts = 0;
    __syncthreads();
    for (uint64_t i = c0 + threadIdx.x; i < c1; i += kLT) {
        const bool st = i == 0 || (epochs && epochs[i] != epochs[i - 1]);
        if (st) starts[atomicAdd(&nstarts, 1u)] = (uint32_t)(i - c0);
    }
    __syncthreads();
    const uint32_t ns = nstarts;
    for (uint32_t r = 0; r < ns; ++r) {
        const uint64_t s = c0 + starts[r];
        const uint32_t most = (uint32_t)(count - s < kRunMax ? count - s : kRunMax);
        const uint32_t ep = epochs ? epochs[s] : 0u;
        if (threadIdx.x == 0) run_len = most;
        __syncthreads();
        if (epochs)
            for (uint32_t j = 1 + threadIdx.x; j < most; j += kLT)
                if (epochs[s + j] != ep) atomicMin(&run_len, j);
        __syncthreads();
        const uint32_t n = 2 * run_len;   // intervals of this epoch
        const uint64_t i0 = 2 * s;
        const uint64_t k0 = keys[i0];
        uint64_t k[kLRounds];
        uint32_t ix[kLRounds];
        uint64_t x = 0;
#pragma unroll
        for (int i = 0; i < kLRounds; ++i) {
            const uint32_t e = w * 512 + i * 64 + l;
            k[i] = e < n ? keys[i0 + e] : ~0ull;
            ix[i] = e;
            if (e < n) x |= k[i] ^ k0;
        }
        for (int d = 32; d >= 1; d >>= 1) x |= __shfl_xor(x, d);
        if (l == 0) wor[w] = x;
        __syncthreads();
        uint64_t live = 0;
        for (int j = 0; j < kLWaves; ++j) live |= wor[j];
        for (int sh = 0; sh < 64; sh += 8) {
            if (((live >> sh) & 0xFFu) == 0) continue;   // the same digit everywhere: skip the pass
            for (int j = threadIdx.x; j < kLWaves * 256; j += kLT) (&wrun[0][0])[j] = 0;
            __syncthreads();
            uint32_t pk[kLRounds];
#pragma unroll
            for (int i = 0; i < kLRounds; ++i) {
                const bool valid = w * 512 + i * 64 + l < n;
                const uint32_t d = (uint32_t)(k[i] >> sh) & 0xFFu;
                const uint64_t peers = match8(d, valid);
                const uint32_t rank = (uint32_t)__popcll(peers & lanes_below());
                uint32_t run = 0;
                if (valid) run = wrun[w][d];
                if (valid && rank == 0) wrun[w][d] = run + (uint32_t)__popcll(peers);
                pk[i] = valid ? (d << 16) | (run + rank) : 0xFFFFFFFFu;
            }
            __syncthreads();
            uint32_t tot = 0;
            if (threadIdx.x < 256)
                for (int j = 0; j < kLWaves; ++j) {
                    const uint32_t c = wrun[j][threadIdx.x];
                    wrun[j][threadIdx.x] = tot;
                    tot += c;
                }
            uint32_t inc = tot;
            for (uint32_t d = 1; d < 64u; d <<= 1) {
                const uint32_t y = __shfl_up(inc, d);
                if (l >= d) inc += y;
            }
            if (threadIdx.x < 256 && l == 63) wtot[w] = inc;
            __syncthreads();
            if (threadIdx.x < 256) {
                uint32_t off = 0;
                for (uint32_t j = 0; j < w; ++j) off += wtot[j];
                dstart[threadIdx.x] = off + inc - tot;
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < kLRounds; ++i)
                if (pk[i] != 0xFFFFFFFFu) {
                    const uint32_t d = pk[i] >> 16;
                    const uint32_t pos = dstart[d] + wrun[w][d] + (pk[i] & 0xFFFFu);
                    buf[pos] = k[i];
                    bix[pos] = (uint16_t)ix[i];
                }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < kLRounds; ++i) {
                const uint32_t e = w * 512 + i * 64 + l;
                if (e < n) {
                    k[i] = buf[e];
                    ix[i] = bix[e];
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < kLRounds; ++i) {
            const uint32_t e = w * 512 + i * 64 + l;
            if (e < n) {
                const uint64_t iv = i0 + ix[i];
                const Iv v = interval_of(recs[iv >> 1], iv);
                keys[i0 + e] = ep;
                vals[i0 + e] = (uint32_t)iv | (v.live ? 0u : kDead);
                first[i0 + e] = v.first;
                ends[i0 + e] = v.last;
                strm[i0 + e] = streams[iv >> 1];
            }
        }
        __syncthreads();
    }
}

// Second pass keys (global path): the epoch of each interval, in the order of
// the first pass, moved into keys[0] / vals[0] with the key-bit parts of the
// second sort.  On the per-epoch path the keys already hold the epochs and the
// parts stay cleared.
__global__ __launch_bounds__(kT) void k_race_rekey(uint64_t *ka, uint32_t *va, const uint32_t *vb,
                                                   const uint64_t *maskp, const uint32_t *epochs, uint64_t m,
                                                   uint64_t *parts, const uint32_t *flag, uint64_t count)
{
    __shared__ uint64_t part[kWaves];
    if (local_path(flag, count)) return;
    const uint32_t *vin = sort_parity(*maskp) ? vb : va;   // va[i] is rewritten with its own value only
    const uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x;
    const uint64_t k0 = epochs ? epochs[(vin[0] & ~kDead) >> 1] : 0u;
    uint64_t x = 0;
    if (i < m) {
        const uint32_t v = vin[i];
        const uint64_t k = epochs ? epochs[(v & ~kDead) >> 1] : 0u;
        ka[i] = k;
        va[i] = v;
        x = k ^ k0;
    }
    for (int d = 32; d >= 1; d >>= 1) x |= __shfl_xor(x, d);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t y = 0;
        for (int w = 0; w < kWaves; ++w) y |= part[w];
        parts[blockIdx.x] = y;
    }
}

// ---- sweep ---------------------------------------------------------------

// A sweep value: (epoch tag, byte) compared as one 128-bit number.  Real
// values have kHere in the high word, so the empty value 0 is below all of
// them.  Forward values are (kHere | epoch, last byte): the largest among
// earlier intervals belongs to the latest epoch, and within it to the
// furthest-reaching interval.  Backward values are (kHere | ~epoch, ~first
// byte), so that the largest is the smallest (epoch, first byte).
struct Val {
    uint64_t h, l;
};

__device__ __forceinline__ bool v_ge(const Val &a, const Val &b) { return a.h > b.h || (a.h == b.h && a.l >= b.l); }
__device__ __forceinline__ bool v_gt(const Val &a, const Val &b) { return a.h > b.h || (a.h == b.h && a.l > b.l); }

// The best two entries (value, record) of distinct streams: (v1, s1, r1) has
// the largest value, (v2, r2) the largest value of any stream other than s1.
// Between equal values either entry may be kept: the values, which decide
// every conflict, come out the same, and any entry kept names a valid
// partner; the combining order is fixed, so results repeat.
struct Top2 {
    Val v1, v2;
    uint32_t s1, r1, r2;
};

__device__ __forceinline__ Top2 t2_none() { return Top2{{0, 0}, {0, 0}, kNoStream, kNoRec, kNoRec}; }

__device__ __forceinline__ Top2 t2_combine(const Top2 &x, const Top2 &y)
{
    const bool xw = v_ge(x.v1, y.v1);
    const Top2 a = xw ? x : y, b = xw ? y : x;
    Top2 o;
    o.v1 = a.v1;
    o.s1 = a.s1;
    o.r1 = a.r1;
    const bool other = b.s1 != a.s1;
    const Val cv = other ? b.v1 : b.v2;
    const uint32_t cr = other ? b.r1 : b.r2;
    const bool keep = v_ge(a.v2, cv);
    o.v2 = keep ? a.v2 : cv;
    o.r2 = keep ? a.r2 : cr;
    return o;
}

// insert one entry
__device__ __forceinline__ Top2 t2_add(const Top2 &x, const Val &v, uint32_t s, uint32_t r)
{
    Top2 o = x;
    if (v_gt(v, x.v1)) {
        // the old best stays as the second unless it has this stream
        const bool other = x.s1 != s;
        o.v2 = other ? x.v1 : x.v2;
        o.r2 = other ? x.r1 : x.r2;
        o.v1 = v;
        o.s1 = s;
        o.r1 = r;
    } else if (s != x.s1 && v_gt(v, x.v2)) {
        o.v2 = v;
        o.r2 = r;
    }
    return o;
}

// the best entry of a stream other than s
__device__ __forceinline__ void t2_other(const Top2 &x, uint32_t s, Val *v, uint32_t *r)
{
    const bool first = x.s1 != s;
    *v = first ? x.v1 : x.v2;
    *r = first ? x.r1 : x.r2;
}

template <int MODE>   // 0: up, 1: down, 2: xor
__device__ __forceinline__ uint64_t shfl64(uint64_t x, int d)
{
    return MODE == 0 ? __shfl_up(x, d) : MODE == 1 ? __shfl_down(x, d) : __shfl_xor(x, d);
}

template <int MODE>
__device__ __forceinline__ uint32_t shfl32(uint32_t x, int d)
{
    return MODE == 0 ? __shfl_up(x, d) : MODE == 1 ? __shfl_down(x, d) : __shfl_xor(x, d);
}

template <int MODE>
__device__ __forceinline__ Top2 t2_shfl(const Top2 &x, int d)
{
    Top2 y;
    y.v1.h = shfl64<MODE>(x.v1.h, d);
    y.v1.l = shfl64<MODE>(x.v1.l, d);
    y.v2.h = shfl64<MODE>(x.v2.h, d);
    y.v2.l = shfl64<MODE>(x.v2.l, d);
    y.s1 = shfl32<MODE>(x.s1, d);
    y.r1 = shfl32<MODE>(x.r1, d);
    y.r2 = shfl32<MODE>(x.r2, d);
    return y;
}

// combine of x over the block's threads before this one (FWD) or after it
template <bool FWD>
__device__ Top2 block_excl(const Top2 &x)
{
    __shared__ Top2 wtot[kWaves];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    Top2 inc = x;
    for (int d = 1; d < 64; d <<= 1) {
        const Top2 y = t2_shfl<FWD ? 0 : 1>(inc, d);
        if (FWD ? l >= d : l + d < 64) inc = t2_combine(inc, y);
    }
    Top2 ex = t2_shfl<FWD ? 0 : 1>(inc, 1);
    if (FWD ? l == 0 : l == 63) ex = t2_none();
    if (FWD ? l == 63 : l == 0) wtot[w] = inc;
    __syncthreads();
    for (int j = 0; j < kWaves; ++j)
        if (FWD ? j < w : j > w) ex = t2_combine(ex, wtot[j]);
    __syncthreads();
    return ex;
}

__device__ Top2 block_all(const Top2 &x)
{
    __shared__ Top2 wtot[kWaves];
    Top2 a = x;
    for (int d = 32; d >= 1; d >>= 1) a = t2_combine(a, t2_shfl<2>(a, d));
    if ((threadIdx.x & 63) == 0) wtot[threadIdx.x >> 6] = a;
    __syncthreads();
    Top2 o = wtot[0];
    for (int j = 1; j < kWaves; ++j) o = t2_combine(o, wtot[j]);
    __syncthreads();
    return o;
}

// one interval of the sorted order
struct Elem {
    uint64_t first, last;
    uint32_t ep, s, r, iv;
    bool valid, w, present;
};

// an interval id slot as read from the sorted order (kNoRec: a padding slot)
__device__ __forceinline__ Elem make_elem(uint32_t raw, uint32_t ep, uint64_t first, uint64_t last, uint32_t s)
{
    Elem e{0, 0, 0, kNoStream, kNoRec, raw & ~kDead, false, false, raw != kNoRec};
    if (e.present && !(raw & kDead)) {
        e.valid = true;
        e.r = e.iv >> 1;
        e.w = (e.iv & 1u) != 0;
        e.ep = ep;
        e.first = first;
        e.last = last;
        e.s = s;
    }
    return e;
}

// The sorted order: epochs K and interval ids V, with the last bytes E and
// streams S in the spare buffers and the first bytes F.
struct Sorted {
    const uint64_t *K, *E, *F;
    const uint32_t *V, *S;
};

__device__ __forceinline__ Sorted sorted_view(const uint64_t *ka, const uint64_t *kb, const uint32_t *va,
                                              const uint32_t *vb, const uint64_t *first, uint64_t mask)
{
    const bool b = sort_parity(mask) != 0;
    return Sorted{b ? kb : ka, b ? ka : kb, first, b ? vb : va, b ? va : vb};
}

__device__ __forceinline__ Elem load_elem(const Sorted &o, uint64_t p, uint64_t m)
{
    if (p >= m) return make_elem(kNoRec, 0, 0, 0, kNoStream);
    const uint32_t raw = o.V[p];
    if (raw & kDead) return make_elem(raw, 0, 0, 0, kNoStream);
    return make_elem(raw, (uint32_t)o.K[p], o.F[p], o.E[p], o.S[p]);
}

// first byte, last byte and stream of every sorted interval, written into
// `first` and the ping-pong buffers that do not hold the sorted order
__global__ __launch_bounds__(kT) void k_race_gather(uint64_t *ka, uint64_t *kb, uint32_t *va, uint32_t *vb,
                                                    uint64_t *first, const uint64_t *maskp, const cg_transfer *recs,
                                                    const uint32_t *streams, uint64_t m, const uint32_t *flag,
                                                    uint64_t count)
{
    const uint64_t p = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (p >= m || local_path(flag, count)) return;   // the per-epoch sort wrote them
    const bool b = sort_parity(*maskp) != 0;
    const uint32_t iv = (b ? vb : va)[p] & ~kDead;
    const Iv v = interval_of(recs[iv >> 1], iv);
    first[p] = v.first;
    (b ? ka : kb)[p] = v.last;
    (b ? va : vb)[p] = streams[iv >> 1];
}

// the four running combines: forward (last bytes) and backward (first
// bytes), of all intervals and of writes
struct Sweep {
    Top2 fa, fw, ba, bw;
};

__device__ __forceinline__ Val fwd_val(const Elem &e) { return Val{kHere | e.ep, e.last}; }
__device__ __forceinline__ Val bwd_val(const Elem &e) { return Val{kHere | (uint32_t)~e.ep, ~e.first}; }

__device__ __forceinline__ void sweep_add_fwd(Sweep &x, const Elem &e)
{
    if (!e.valid) return;
    const Val v = fwd_val(e);
    x.fa = t2_add(x.fa, v, e.s, e.r);
    if (e.w) x.fw = t2_add(x.fw, v, e.s, e.r);
}

__device__ __forceinline__ void sweep_add_bwd(Sweep &x, const Elem &e)
{
    if (!e.valid) return;
    const Val v = bwd_val(e);
    x.ba = t2_add(x.ba, v, e.s, e.r);
    if (e.w) x.bw = t2_add(x.bw, v, e.s, e.r);
}

__global__ __launch_bounds__(kT) void k_race_sweep_reduce(const uint64_t *ka, const uint64_t *kb, const uint32_t *va,
                                                          const uint32_t *vb, const uint64_t *first,
                                                          const uint64_t *maskp, uint64_t m, Top2 *agg)
{
    const Sorted o = sorted_view(ka, kb, va, vb, first, *maskp);
    // the combines do not depend on order: read the tile lane-contiguously
    const uint64_t base = (uint64_t)blockIdx.x * kSweepTile + threadIdx.x;
    Sweep x{t2_none(), t2_none(), t2_none(), t2_none()};
    for (int j = 0; j < kSweepItems; ++j) {
        const Elem e = load_elem(o, base + (uint64_t)j * kT, m);
        sweep_add_fwd(x, e);
        sweep_add_bwd(x, e);
    }
    const Top2 fa = block_all(x.fa), fw = block_all(x.fw), ba = block_all(x.ba), bw = block_all(x.bw);
    if (threadIdx.x == 0) {
        Top2 *o = agg + (uint64_t)blockIdx.x * 4;
        o[0] = fa;
        o[1] = fw;
        o[2] = ba;
        o[3] = bw;
    }
}

// per sweep tile: combine of the tiles before it (forward) and after it (backward)
__global__ __launch_bounds__(kT) void k_race_sweep_scan(const Top2 *agg, uint32_t tiles, Top2 *pre)
{
    const uint32_t per = (tiles + kT - 1) / kT;
    const uint32_t lo = min(tiles, threadIdx.x * per), hi = min(tiles, lo + per);
    Sweep c{t2_none(), t2_none(), t2_none(), t2_none()};
    for (uint32_t b = lo; b < hi; ++b) {
        c.fa = t2_combine(c.fa, agg[(uint64_t)b * 4 + 0]);
        c.fw = t2_combine(c.fw, agg[(uint64_t)b * 4 + 1]);
        c.ba = t2_combine(c.ba, agg[(uint64_t)b * 4 + 2]);
        c.bw = t2_combine(c.bw, agg[(uint64_t)b * 4 + 3]);
    }
    Top2 fa = block_excl<true>(c.fa), fw = block_excl<true>(c.fw);
    Top2 ba = block_excl<false>(c.ba), bw = block_excl<false>(c.bw);
    for (uint32_t b = lo; b < hi; ++b) {
        pre[(uint64_t)b * 4 + 0] = fa;
        pre[(uint64_t)b * 4 + 1] = fw;
        fa = t2_combine(fa, agg[(uint64_t)b * 4 + 0]);
        fw = t2_combine(fw, agg[(uint64_t)b * 4 + 1]);
    }
    for (uint32_t b = hi; b > lo; --b) {
        pre[(uint64_t)(b - 1) * 4 + 2] = ba;
        pre[(uint64_t)(b - 1) * 4 + 3] = bw;
        ba = t2_combine(ba, agg[(uint64_t)(b - 1) * 4 + 2]);
        bw = t2_combine(bw, agg[(uint64_t)(b - 1) * 4 + 3]);
    }
}

// per interval: a record of another stream it meets (writes: any access;
// reads: writes), or kNoRec
// LDS slot of tile element i: one pad slot per kSweepItems elements, so that
// threads reading their own consecutive runs spread over the banks
__device__ __forceinline__ int pad_slot(int i) { return i + i / kSweepItems; }
constexpr int kSweepSlots = kSweepTile + kSweepTile / kSweepItems;

__global__ __launch_bounds__(kT) void k_race_sweep_apply(const uint64_t *ka, const uint64_t *kb, const uint32_t *va,
                                                         const uint32_t *vb, const uint64_t *first,
                                                         const uint64_t *maskp, uint64_t m, const Top2 *pre,
                                                         uint32_t *res)
{
    __shared__ uint64_t sf[kSweepSlots], se[kSweepSlots];
    __shared__ uint32_t sk[kSweepSlots], sv[kSweepSlots], ss[kSweepSlots];
    const Sorted o = sorted_view(ka, kb, va, vb, first, *maskp);
    const uint64_t tile = (uint64_t)blockIdx.x * kSweepTile;
    // stage the tile through LDS: read lane-contiguously, walk per thread
    for (int j = 0; j < kSweepItems; ++j) {
        const int i = j * kT + threadIdx.x;
        const uint64_t p = tile + i;
        const int q = pad_slot(i);
        sv[q] = kNoRec;
        if (p < m) {
            const uint32_t raw = o.V[p];
            sv[q] = raw;
            if (!(raw & kDead)) {
                sk[q] = (uint32_t)o.K[p];
                sf[q] = o.F[p];
                se[q] = o.E[p];
                ss[q] = o.S[p];
            }
        }
    }
    __syncthreads();
    const int base = threadIdx.x * kSweepItems;
    auto elem = [&](int j) {
        const int q = pad_slot(base + j);
        const uint32_t raw = sv[q];
        if (raw & kDead) return make_elem(raw, 0, 0, 0, kNoStream);
        return make_elem(raw, sk[q], sf[q], se[q], ss[q]);
    };
    Sweep own{t2_none(), t2_none(), t2_none(), t2_none()};
    for (int j = 0; j < kSweepItems; ++j) {
        const Elem e = elem(j);
        sweep_add_fwd(own, e);
        sweep_add_bwd(own, e);
    }
    const Top2 *P = pre + (uint64_t)blockIdx.x * 4;
    Sweep x;
    x.fa = t2_combine(P[0], block_excl<true>(own.fa));
    x.fw = t2_combine(P[1], block_excl<true>(own.fw));
    x.ba = t2_combine(P[2], block_excl<false>(own.ba));
    x.bw = t2_combine(P[3], block_excl<false>(own.bw));
    uint32_t hit[kSweepItems];
#pragma unroll
    for (int j = 0; j < kSweepItems; ++j) {
        const Elem e = elem(j);
        hit[j] = kNoRec;
        if (e.valid) {
            // an earlier interval of another stream, in this epoch, reaching this one's first byte
            Val va, vw;
            uint32_t ra, rw;
            t2_other(x.fa, e.s, &va, &ra);
            t2_other(x.fw, e.s, &vw, &rw);
            const Val v = e.w ? va : vw;
            if (v.h == (kHere | e.ep) && v.l >= e.first) hit[j] = e.w ? ra : rw;
        }
        sweep_add_fwd(x, e);
    }
#pragma unroll
    for (int j = kSweepItems - 1; j >= 0; --j) {
        const Elem e = elem(j);
        if (e.valid && hit[j] == kNoRec) {
            // a later interval of another stream, in this epoch, starting at or before this one's last byte
            Val va, vw;
            uint32_t ra, rw;
            t2_other(x.ba, e.s, &va, &ra);
            t2_other(x.bw, e.s, &vw, &rw);
            const Val v = e.w ? va : vw;
            if (v.h == (kHere | (uint32_t)~e.ep) && ~v.l <= e.last) hit[j] = e.w ? ra : rw;
        }
        sweep_add_bwd(x, e);
        if (e.present) res[e.iv] = hit[j];
    }
}

__global__ __launch_bounds__(kT) void k_race_finalize(const cg_transfer *recs, uint64_t count, const uint32_t *res,
                                                      cg_race *out)
{
    const uint64_t r = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= count) return;
    const cg_transfer t = recs[r];
    cg_race o;
    o.reserved = 0;
    if (!rec_checked(t)) {
        o.flags = CG_RACE_UNCHECKED;
        o.partner = CG_NONE;
    } else {
        const uint32_t ps = res[2 * r], pd = res[2 * r + 1];
        o.flags = (ps != kNoRec ? CG_RACE_SRC : 0u) | (pd != kNoRec ? CG_RACE_DST : 0u);
        const uint32_t p = pd != kNoRec ? pd : ps;
        o.partner = p == kNoRec ? CG_NONE : (uint64_t)p;
    }
    out[r] = o;
}

uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

}  // namespace

hipError_t race_reserve(RaceWs &w, uint64_t intervals)
{
    if (intervals <= w.cap) return hipSuccess;
    race_release(w);
    hipError_t e = sort_reserve(w.sort, intervals);
    const uint64_t sweeps = ceil_div(intervals, kSweepTile);
    auto get = [&](void **p, uint64_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, bytes ? bytes : 8);
    };
    get((void **)&w.res, intervals * sizeof(uint32_t));
    get((void **)&w.first, intervals * sizeof(uint64_t));
    get((void **)&w.flag, 64);
    get(&w.agg, sweeps * 4 * sizeof(Top2));
    get(&w.pre, sweeps * 4 * sizeof(Top2));
    if (e != hipSuccess) {
        race_release(w);
        return e;
    }
    w.cap = intervals;
    return hipSuccess;
}

void race_release(RaceWs &w)
{
    sort_release(w.sort);
    void *ps[] = {w.res, w.first, w.agg, w.pre, w.flag};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    w = RaceWs{};
}

hipError_t race_launch(RaceWs &w, const cg_transfer *recs, const uint32_t *streams, const uint32_t *epochs,
                       uint64_t count, cg_race *out, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    const uint64_t m = 2 * count;
    const uint32_t sweeps = (uint32_t)ceil_div(m, kSweepTile);
    const uint32_t blocks = (uint32_t)ceil_div(m, kT);
    SortWs &q = w.sort;
    hipLaunchKernelGGL(k_race_keys, dim3(blocks), dim3(kT), 0, s, recs, m, q.keys[0], q.vals[0], q.parts, w.flag);
    hipLaunchKernelGGL(k_race_local_check, dim3((uint32_t)ceil_div(count, kT)), dim3(kT), 0, s, epochs, count, w.flag);
    hipLaunchKernelGGL(k_race_local_sort, dim3((uint32_t)ceil_div(count, kRunMax)), dim3(kLT), 0, s, q.keys[0],
                       q.vals[0], q.keys[1], q.vals[1], w.first, q.parts, ceil_div(m, kT), recs, streams, epochs, count,
                       w.flag);
    // without epochs, a batch of kRunMean to kRunMax records is one epoch that
    // the per-epoch sort takes (as the device decides too): the global passes
    // would all return at once, so they are not launched
    const bool one_local_epoch = !epochs && count <= kRunMax && count >= kRunMean;
    // first sort: by first byte
    hipError_t e = one_local_epoch ? sort_mask_only(q, m, s) : sort_pairs(q, m, s);
    if (e != hipSuccess) return e;
    // second sort, stable: by epoch (all 0 without epochs: only the mask is taken,
    // which then names keys[0] / vals[0], where the rekey moved the order)
    if (!one_local_epoch)
        hipLaunchKernelGGL(k_race_rekey, dim3(blocks), dim3(kT), 0, s, q.keys[0], q.vals[0], q.vals[1], q.mask, epochs,
                           m, q.parts, w.flag, count);
    e = epochs ? sort_pairs(q, m, s, nullptr, 4) : sort_mask_only(q, m, s);
    if (e != hipSuccess) return e;
    Top2 *agg = (Top2 *)w.agg, *pre = (Top2 *)w.pre;
    hipLaunchKernelGGL(k_race_gather, dim3(blocks), dim3(kT), 0, s, q.keys[0], q.keys[1], q.vals[0], q.vals[1], w.first,
                       q.mask, recs, streams, m, w.flag, count);
    hipLaunchKernelGGL(k_race_sweep_reduce, dim3(sweeps), dim3(kT), 0, s, q.keys[0], q.keys[1], q.vals[0], q.vals[1],
                       w.first, q.mask, m, agg);
    hipLaunchKernelGGL(k_race_sweep_scan, dim3(1), dim3(kT), 0, s, agg, sweeps, pre);
    hipLaunchKernelGGL(k_race_sweep_apply, dim3(sweeps), dim3(kT), 0, s, q.keys[0], q.keys[1], q.vals[0], q.vals[1],
                       w.first, q.mask, m, pre, w.res);
    hipLaunchKernelGGL(k_race_finalize, dim3((uint32_t)ceil_div(count, kT)), dim3(kT), 0, s, recs, count, w.res, out);
    return hipGetLastError();
}

}  // namespace xc
