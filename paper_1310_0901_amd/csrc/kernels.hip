// HIP kernels of the transfer checker, written for gfx950 (CDNA4, wave64).
//
// The method (Cudagrind, arXiv 1310.0901): every copy is cross-checked
// against the context's list of live device allocations (Sec. 2, Fig. 2
// caption); host source bytes must be addressable and defined, tracked with
// bitwise shadow precision (Sec. 1.1); the report gives the bytes the copy
// needs against the bytes the allocation holds (Sec. 4.5); definedness is
// carried through host/device, device/host and device/device copies (Sec. 5).
//
// Pipeline of one batched check (all integer, bit-exact):
//   k_classify     one lane per record: decode, interval lookup in the
//                  sorted allocation table (top level staged in LDS),
//                  range-derived verdict fields, scan descriptor, work weight,
//                  block-local exclusive scan of the weights; for a check the
//                  shadow indexes may answer, the valid bytes per shadow space
//                  and the marks of the 64 KiB shadow steps they fall in;
//   (shadowindex.hip) large check-only batches: indexes of the faulty chunks
//                  of those steps, which answer the records whose spaces they
//                  cover (their units leave the scan);
//   (segment.hip)  large batches only: every record's units cut at blocks of
//                  source memory, the pieces sorted by block and laid out as
//                  the batch's positions (descriptors, weights, block-local
//                  scan), so that work reading the same bytes runs together;
//                  the kernels below work by position and send findings to
//                  each position's record;
//   k_scan_sums    one block: exclusive scan of the per-block sums, tile size;
//   k_prefix_tiles global prefix; k_tile_starts first record of every tile;
//   k_batched      persistent kernel: tiles of the flattened 16-byte unit space,
//                  one contiguous chunk per XCD for a segmented batch, taken
//                  from per-chunk device counters; 16-byte V loads and aligned
//                  16-bit A loads, SWAR non-zero masks, popcount / ctz for the
//                  undefined count and first fault, DPP wave reductions, rare
//                  global atomics; optional realigned V store to the
//                  destination shadow.
// The plain path runs k_classify once, then k_plain once per record.
#include <hip/hip_runtime.h>

#include "xc_internal.h"

namespace xc {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr uint64_t NONE = CG_NONE;

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Bits j of a 16-byte chunk with lo <= j < hi (offsets relative to the chunk).
__device__ __forceinline__ uint32_t rmask(int64_t lo, int64_t hi)
{
    int64_t l = lo < 0 ? 0 : (lo > 16 ? 16 : lo);
    int64_t h = hi < 0 ? 0 : (hi > 16 ? 16 : hi);
    return h > l ? ((1u << (uint32_t)h) - (1u << (uint32_t)l)) : 0u;
}

// One bit per byte of w: set where the byte is non-zero (SWAR, no carries
// cross byte lanes because every byte sum stays below 0x100).
__device__ __forceinline__ uint32_t nz4(uint32_t w)
{
    uint32_t t = (((w & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | w) & 0x80808080u;
    return ((t >> 7) | (t >> 14) | (t >> 21) | (t >> 28)) & 0xFu;
}

__device__ __forceinline__ uint32_t nz16(u32x4 v)
{
    return nz4(v.x) | (nz4(v.y) << 4) | (nz4(v.z) << 8) | (nz4(v.w) << 12);
}

// 4-bit mask -> byte mask (0x00 / 0xFF per byte); the shifted copies of m do
// not overlap, so the multiply has no carries.
__device__ __forceinline__ uint32_t expand4(uint32_t m)
{
    return ((m * 0x00204081u) & 0x01010101u) * 0xFFu;
}

// Value a source chunk contributes to propagation: its V byte where the
// source byte is valid, 0xFF where it is not.
__device__ __forceinline__ u32x4 prop_val(u32x4 v, uint32_t ok)
{
    if (ok == 0xFFFFu) return v;
    u32x4 r;
    r.x = v.x | ~expand4(ok & 0xFu);
    r.y = v.y | ~expand4((ok >> 4) & 0xFu);
    r.z = v.z | ~expand4((ok >> 8) & 0xFu);
    r.w = v.w | ~expand4((ok >> 12) & 0xFu);
    return r;
}

// Bytes [s, s + 16) of the 32-byte concatenation a || b.
__device__ __forceinline__ u32x4 window(u32x4 a, u32x4 b, uint32_t s)
{
    const uint32_t q = s >> 2, r = s & 3u;
    uint32_t w0, w1, w2, w3, w4;
    switch (q) {
    case 0: w0 = a.x; w1 = a.y; w2 = a.z; w3 = a.w; w4 = b.x; break;
    case 1: w0 = a.y; w1 = a.z; w2 = a.w; w3 = b.x; w4 = b.y; break;
    case 2: w0 = a.z; w1 = a.w; w2 = b.x; w3 = b.y; w4 = b.z; break;
    default: w0 = a.w; w1 = b.x; w2 = b.y; w3 = b.z; w4 = b.w; break;
    }
    u32x4 o;
    o.x = __builtin_amdgcn_alignbyte(w1, w0, r);
    o.y = __builtin_amdgcn_alignbyte(w2, w1, r);
    o.z = __builtin_amdgcn_alignbyte(w3, w2, r);
    o.w = __builtin_amdgcn_alignbyte(w4, w3, r);
    return o;
}

// Global (address space 1) views of device addresses, so that the compiler
// emits global_load / global_store rather than flat accesses.
template <typename T> using gptr = __attribute__((address_space(1))) T *;
template <typename T> using gcptr = const __attribute__((address_space(1))) T *;

__device__ __forceinline__ void store_word_masked(uint64_t p, uint32_t w, uint32_t m)
{
    if (m == 0xFu) { *reinterpret_cast<gptr<uint32_t>>(p) = w; return; }
    gptr<uint8_t> b = reinterpret_cast<gptr<uint8_t>>(p);
    if (m & 1u) b[0] = (uint8_t)w;
    if (m & 2u) b[1] = (uint8_t)(w >> 8);
    if (m & 4u) b[2] = (uint8_t)(w >> 16);
    if (m & 8u) b[3] = (uint8_t)(w >> 24);
}

// Store the bytes of v selected by m at the 16-byte aligned address p.
__device__ __forceinline__ void store_masked(uint64_t p, u32x4 v, uint32_t m)
{
    if (m == 0xFFFFu) { *reinterpret_cast<gptr<u32x4>>(p) = v; return; }
    if (m & 0x000Fu) store_word_masked(p, v.x, m & 0xFu);
    if (m & 0x00F0u) store_word_masked(p + 4, v.y, (m >> 4) & 0xFu);
    if (m & 0x0F00u) store_word_masked(p + 8, v.z, (m >> 8) & 0xFu);
    if (m & 0xF000u) store_word_masked(p + 12, v.w, (m >> 12) & 0xFu);
}

template <bool NT>
__device__ __forceinline__ u32x4 ld16(uint64_t addr)
{
    gcptr<u32x4> p = reinterpret_cast<gcptr<u32x4>>(addr);
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

__device__ __forceinline__ uint32_t ld_u16(uint64_t addr)
{
    return *reinterpret_cast<gcptr<uint16_t>>(addr);
}

__device__ __forceinline__ int32_t clamp32(int64_t x)
{
    return x < -(1ll << 30) ? -(1 << 30) : (x > (1ll << 30) ? (1 << 30) : (int32_t)x);
}

// rmask for offsets already clamped to 32 bits
__device__ __forceinline__ uint32_t rmask32(int32_t lo, int32_t hi)
{
    const int32_t l = lo < 0 ? 0 : (lo > 16 ? 16 : lo);
    const int32_t h = hi < 0 ? 0 : (hi > 16 ? 16 : hi);
    return h > l ? ((1u << h) - (1u << l)) : 0u;
}

__device__ __forceinline__ uint32_t ufl32(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ uint64_t ufl64(uint64_t x)
{
    return ((uint64_t)ufl32((uint32_t)(x >> 32)) << 32) | ufl32((uint32_t)x);
}

// ---- DPP wave reductions (every lane of the wave must be active) --------
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ uint64_t dpp64(uint64_t x)
{
    uint32_t lo = dpp32<CTRL>((uint32_t)x), hi = dpp32<CTRL>((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t readlane64(uint64_t x, int l)
{
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}
// quad_perm [1,0,3,2] = 0xB1, quad_perm [2,3,0,1] = 0x4E, row_half_mirror =
// 0x141, row_mirror = 0x140: after the four steps every lane holds its
// 16-lane row's total; the four rows are combined from lanes 0/16/32/48.
__device__ __forceinline__ uint64_t wave_min64(uint64_t x)
{
    uint64_t y;
    y = dpp64<0xB1>(x); x = y < x ? y : x;
    y = dpp64<0x4E>(x); x = y < x ? y : x;
    y = dpp64<0x141>(x); x = y < x ? y : x;
    y = dpp64<0x140>(x); x = y < x ? y : x;
    uint64_t a = readlane64(x, 0), b = readlane64(x, 16), c = readlane64(x, 32), d = readlane64(x, 48);
    a = b < a ? b : a;
    c = d < c ? d : c;
    return c < a ? c : a;
}
__device__ __forceinline__ uint64_t wave_sum64(uint64_t x)
{
    x += dpp64<0xB1>(x);
    x += dpp64<0x4E>(x);
    x += dpp64<0x141>(x);
    x += dpp64<0x140>(x);
    return readlane64(x, 0) + readlane64(x, 16) + readlane64(x, 32) + readlane64(x, 48);
}
__device__ __forceinline__ uint32_t wave_or32(uint32_t x)
{
    x |= dpp32<0xB1>(x);
    x |= dpp32<0x4E>(x);
    x |= dpp32<0x141>(x);
    x |= dpp32<0x140>(x);
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 0) | (uint32_t)__builtin_amdgcn_readlane((int)x, 16) |
           (uint32_t)__builtin_amdgcn_readlane((int)x, 32) | (uint32_t)__builtin_amdgcn_readlane((int)x, 48);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// ---------------------------------------------------------------------------
// descriptor in registers
// ---------------------------------------------------------------------------
struct DV {
    uint64_t src_sh, dst_sh;
    int64_t v_lo, v_hi, d_lo, d_hi, a_src, a_dst;
    uint64_t e0, units;
    uint32_t ctl, phi, psi, delta, s;
};

__device__ __forceinline__ DV make_dv(const Desc &x)
{
    DV d;
    d.src_sh = x.src_sh; d.dst_sh = x.dst_sh;
    d.v_lo = x.v_lo; d.v_hi = x.v_hi; d.d_lo = x.d_lo; d.d_hi = x.d_hi;
    d.a_src = x.a_src; d.a_dst = x.a_dst; d.e0 = x.e0; d.units = x.units;
    d.ctl = x.ctl;
    d.phi = (d.ctl >> CTL_PHI_SHIFT) & 15u;
    d.psi = (d.ctl >> CTL_PSI_SHIFT) & 15u;
    d.delta = (d.ctl & CTL_DELTA) ? 1u : 0u;
    d.s = (d.phi - d.psi) & 15u;
    return d;
}

// Per-lane descriptor (lanes may work on different records).
__device__ __forceinline__ DV load_desc(const Desc *D, uint64_t t) { return make_dv(D[t]); }

// Wave-uniform descriptor: every field forced into scalar registers.
__device__ __forceinline__ DV load_desc_uniform(const Desc *D, uint64_t t)
{
    const Desc &x = D[t];
    Desc u;
    u.src_sh = ufl64(x.src_sh); u.dst_sh = ufl64(x.dst_sh);
    u.v_lo = (int64_t)ufl64((uint64_t)x.v_lo); u.v_hi = (int64_t)ufl64((uint64_t)x.v_hi);
    u.d_lo = (int64_t)ufl64((uint64_t)x.d_lo); u.d_hi = (int64_t)ufl64((uint64_t)x.d_hi);
    u.a_src = (int64_t)ufl64((uint64_t)x.a_src); u.a_dst = (int64_t)ufl64((uint64_t)x.a_dst);
    u.e0 = ufl64(x.e0); u.units = ufl64(x.units); u.ctl = ufl32(x.ctl);
    return make_dv(u);
}

// Source chunk c: V bytes, valid-byte mask, and (host source) the in-range
// bytes whose A bit is 0.  Nothing is read outside the valid byte range.
template <bool NT>
__device__ __forceinline__ void src_chunk(const DV &d, const Region &R, int64_t c, u32x4 &v,
                                          uint32_t &ok, uint32_t &unaddr)
{
    const int64_t i0 = 16 * c - (int64_t)d.phi;
    const uint32_t m = rmask(d.v_lo - i0, d.v_hi - i0);
    v = u32x4{0u, 0u, 0u, 0u};
    ok = 0u;
    unaddr = 0u;
    if (m) {
        v = ld16<NT>(d.src_sh + (uint64_t)(16 * c));
        if (d.ctl & CTL_SRC_HOST) {
            const uint32_t a = ld_u16((uint64_t)R.a16 + (uint64_t)((d.a_src + 16 * c) >> 3));
            ok = m & a;
            unaddr = m & ~a;
        } else {
            ok = m;
        }
    }
}

struct Acc {
    uint64_t first, undef;
    uint32_t flags;
};

__device__ __forceinline__ void acc_reset(Acc &a) { a.first = NONE; a.undef = 0; a.flags = 0; }

__device__ __forceinline__ void acc_min(Acc &a, int64_t i) { a.first = (uint64_t)i < a.first ? (uint64_t)i : a.first; }

// Findings of source chunk c (checking only).
__device__ __forceinline__ void src_findings(Acc &a, int64_t i0, u32x4 v, uint32_t ok, uint32_t unaddr)
{
    const uint32_t any = v.x | v.y | v.z | v.w;
    if (unaddr) {
        a.flags |= CG_SRC_UNADDR;
        acc_min(a, i0 + __builtin_ctz(unaddr));
    }
    if (any) {
        const uint32_t und = nz16(v) & ok;
        if (und) {
            a.flags |= CG_SRC_UNDEF;
            a.undef += (uint64_t)__builtin_popcount(und);
            acc_min(a, i0 + __builtin_ctz(und));
        }
    }
}

// Wave-wide flush of uniform-mode accumulators for record t (all lanes active).
__device__ __forceinline__ void flush_wave(Acc &a, cg_verdict *out, uint64_t t)
{
    if (__ballot(a.flags != 0u)) {
        const uint64_t first = wave_min64(a.first);
        const uint64_t und = wave_sum64(a.undef);
        const uint32_t fl = wave_or32(a.flags);
        if (lane_id() == 0) {
            atomicOr(&out[t].flags, fl);
            if (first != NONE) atomicMin((unsigned long long *)&out[t].first_bad, (unsigned long long)first);
            if (und) atomicAdd((unsigned long long *)&out[t].undef_bytes, (unsigned long long)und);
        }
    }
    acc_reset(a);
}

// ---------------------------------------------------------------------------
// uniform mode: the whole wave works on units [k_begin, k_end) of one record
// ---------------------------------------------------------------------------

// Chunks 64 j + lane (j < U) of an interior iteration: V from vbase, source A
// words from abase (SA), destination A words from dbase (DA); true when every
// V byte of the wave's chunks is 0 and every A bit 1.
template <int U, bool NT, bool SA, bool DA>
__device__ __forceinline__ bool clean_interior(uint64_t vbase, uint64_t abase, uint64_t dbase)
{
    const gcptr<u32x4> vp = reinterpret_cast<gcptr<u32x4>>(vbase);
    const gcptr<uint16_t> ap = reinterpret_cast<gcptr<uint16_t>>(abase);
    const gcptr<uint16_t> dp = reinterpret_cast<gcptr<uint16_t>>(dbase);
    const uint32_t lane = lane_id();
    u32x4 w[U];
    uint32_t sa[U], da[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const uint32_t cr = 64u * j + lane;
        if constexpr (NT) w[j] = __builtin_nontemporal_load(vp + cr);
        else w[j] = vp[cr];
        if constexpr (SA) sa[j] = ap[cr];
        if constexpr (DA) da[j] = dp[cr];
    }
    uint32_t bad = 0;
#pragma unroll
    for (int j = 0; j < U; ++j) {
        bad |= w[j].x | w[j].y | w[j].z | w[j].w;
        if constexpr (SA) bad |= sa[j] ^ 0xFFFFu;
        if constexpr (DA) bad |= da[j] ^ 0xFFFFu;
    }
    return __ballot(bad != 0u) == 0;
}
template <int U, bool NT, bool PROP>
__device__ __forceinline__ void run_uniform(const DV &d, const Region &R, uint64_t k_begin, uint64_t k_end,
                                            Acc &acc)
{
    // Lane l of sub-iteration j handles unit kb + 64 j + l: destination chunk
    // e = e0 + kb + 64 j + l and source chunk c = e - delta.  Per iteration all
    // offsets are taken relative to the first unit, in 32 bits.  Loads are
    // issued for every lane with the chunk index clamped into the range of
    // chunks that hold valid bytes, so that all U loads go out back to back
    // without branches; lanes whose own chunk has no valid byte ignore the data.
    const int32_t lane = (int32_t)lane_id();
    const bool check = (d.ctl & CTL_CHECK) != 0;
    const bool prop = PROP && (d.ctl & CTL_PROP) != 0;
    const bool dsta = (d.ctl & CTL_DST_A) != 0;
    const bool src_host = (d.ctl & CTL_SRC_HOST) != 0;
    const bool dst_host = (d.ctl & CTL_DST_HOST) != 0;
    const uint64_t a16b = (uint64_t)R.a16;

    for (uint64_t kb = k_begin; kb < k_end; kb += 64u * U) {
        const int64_t cb = (int64_t)(d.e0 + kb) - (int64_t)d.delta;
        const int64_t i0b = 16 * cb - (int64_t)d.phi;
        const int32_t vlo = clamp32(d.v_lo - i0b), vhi = clamp32(d.v_hi - i0b);
        const int32_t kend = clamp32((int64_t)(k_end - kb));
        const int32_t clo = (vlo >> 4) > 0 ? (vlo >> 4) : 0;
        const int32_t chi = ((vhi + 15) >> 4) < 64 * U ? ((vhi + 15) >> 4) : 64 * U;
        const uint64_t vbase = d.src_sh + (uint64_t)(16 * cb);
        const uint64_t abase = a16b + (uint64_t)((d.a_src + 16 * cb) >> 3);

        // Interior iteration of a check (kernels built without propagation,
        // whose register budget allows three waves per SIMD): every lane's U
        // source chunks lie wholly inside the valid source range (and, for a
        // host destination, its chunks inside the valid destination range), so
        // no byte mask or index clamp is needed.  When every V byte is 0 and
        // every A bit 1, the code below would find nothing and the iteration
        // ends here; otherwise (rare) that code runs the iteration again and
        // reports exactly.
        if (!PROP && check && vlo <= 0 && vhi >= 16 * 64 * U && kend >= 64 * U) {
            bool dfull = true;
            uint64_t dbase = 0;
            if (dsta) {
                const int64_t eb = (int64_t)(d.e0 + kb);
                const int64_t i0db = 16 * eb - (int64_t)d.psi;
                dfull = clamp32(d.d_lo - i0db) <= 0 && clamp32(d.d_hi - i0db) >= 16 * 64 * U;
                dbase = a16b + (uint64_t)((d.a_dst + 16 * eb) >> 3);
            }
            if (dfull) {
                // a host destination (D2H) has a device source; a host source
                // (H2D) has a device destination
                const bool clean = dsta ? clean_interior<U, NT, false, true>(vbase, abase, dbase)
                                 : src_host ? clean_interior<U, NT, true, false>(vbase, abase, dbase)
                                            : clean_interior<U, NT, false, false>(vbase, abase, dbase);
                if (clean) continue;
            }
        }

        u32x4 v[U];
        uint32_t ok[U], un[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            v[j] = u32x4{0u, 0u, 0u, 0u};
            ok[j] = 0u;
            un[j] = 0u;
        }
        if (chi > clo) {
            uint32_t av[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int32_t cr = 64 * j + lane;
                const int32_t cc = cr < clo ? clo : (cr >= chi ? chi - 1 : cr);
                v[j] = ld16<NT>(vbase + (uint32_t)(16 * cc));
                if (src_host) av[j] = ld_u16(abase + (uint32_t)(2 * cc));
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int32_t cr = 64 * j + lane;
                const uint32_t m = cr < kend ? rmask32(vlo - 16 * cr, vhi - 16 * cr) : 0u;
                if (src_host) {
                    ok[j] = m & av[j];
                    un[j] = m & ~av[j];
                } else {
                    ok[j] = m;
                }
            }
        }
        if (check) {
#pragma unroll
            for (int j = 0; j < U; ++j) src_findings(acc, i0b + 16 * (64 * j + lane), v[j], ok[j], un[j]);
        }
        if (dsta || prop) {
            const int64_t eb = (int64_t)(d.e0 + kb);
            const int64_t i0db = 16 * eb - (int64_t)d.psi;
            const int32_t dlo = clamp32(d.d_lo - i0db), dhi = clamp32(d.d_hi - i0db);
            const int32_t dclo = (dlo >> 4) > 0 ? (dlo >> 4) : 0;
            const int32_t dchi = ((dhi + 15) >> 4) < 64 * U ? ((dhi + 15) >> 4) : 64 * U;
            uint32_t ad[U];
            if (dst_host && dchi > dclo) {
                const uint64_t dbase = a16b + (uint64_t)((d.a_dst + 16 * eb) >> 3);
#pragma unroll
                for (int j = 0; j < U; ++j) {
                    const int32_t cr = 64 * j + lane;
                    const int32_t cc = cr < dclo ? dclo : (cr >= dchi ? dchi - 1 : cr);
                    ad[j] = ld_u16(dbase + (uint32_t)(2 * cc));
                }
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int32_t cr = 64 * j + lane;
                const uint32_t md = (cr < kend && dchi > dclo) ? rmask32(dlo - 16 * cr, dhi - 16 * cr) : 0u;
                uint32_t wm = md;
                if (dst_host) {
                    wm = md & ad[j];
                    const uint32_t ud = md & ~ad[j];
                    if (check && ud) {
                        acc.flags |= CG_DST_UNADDR;
                        acc_min(acc, i0db + 16 * cr + __builtin_ctz(ud));
                    }
                }
                if (prop && d.s == 0) {
                    // source and destination chunks coincide (equal phases)
                    if (wm) store_masked(d.dst_sh + (uint64_t)(16 * eb) + (uint32_t)(16 * cr), prop_val(v[j], ok[j]), wm);
                } else if (prop) {
                    const u32x4 own = prop_val(v[j], ok[j]);
                    u32x4 nxt;
                    nxt.x = __shfl_down(own.x, 1);
                    nxt.y = __shfl_down(own.y, 1);
                    nxt.z = __shfl_down(own.z, 1);
                    nxt.w = __shfl_down(own.w, 1);
                    if (j + 1 < U) {
                        const int jn = j + 1 < U ? j + 1 : j;
                        const u32x4 g = prop_val(v[jn], ok[jn]);
                        const uint32_t gx = __shfl(g.x, 0), gy = __shfl(g.y, 0), gz = __shfl(g.z, 0),
                                       gw = __shfl(g.w, 0);
                        if (lane == 63) nxt = u32x4{gx, gy, gz, gw};
                    }
                    const bool self = cr < kend && ((lane == 63 && j == U - 1) || cr + 1 >= kend);
                    if (self) {
                        u32x4 vn;
                        uint32_t okn, unn;
                        src_chunk<NT>(d, R, cb + cr + 1, vn, okn, unn);
                        nxt = prop_val(vn, okn);
                    }
                    if (wm) store_masked(d.dst_sh + (uint64_t)(16 * eb) + (uint32_t)(16 * cr), window(own, nxt, d.s), wm);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// one unit handled by one lane (small records, tile boundaries)
// ---------------------------------------------------------------------------
template <bool NT, bool PROP>
__device__ __forceinline__ void run_unit(const DV &d, const Region &R, uint64_t k, Acc &acc)
{
    const bool check = (d.ctl & CTL_CHECK) != 0;
    const int64_t e = (int64_t)(d.e0 + k);
    const int64_t c = e - (int64_t)d.delta;
    u32x4 v;
    uint32_t ok, un;
    src_chunk<NT>(d, R, c, v, ok, un);
    if (check) src_findings(acc, 16 * c - (int64_t)d.phi, v, ok, un);
    if (d.ctl & (CTL_DST_A | CTL_PROP)) {
        const int64_t i0d = 16 * e - (int64_t)d.psi;
        const uint32_t md = rmask(d.d_lo - i0d, d.d_hi - i0d);
        uint32_t wm = md;
        if ((d.ctl & CTL_DST_HOST) && md) {
            const uint32_t a = ld_u16((uint64_t)R.a16 + (uint64_t)((d.a_dst + 16 * e) >> 3));
            wm = md & a;
            const uint32_t ud = md & ~a;
            if (check && ud) {
                acc.flags |= CG_DST_UNADDR;
                acc_min(acc, i0d + __builtin_ctz(ud));
            }
        }
        if (PROP && (d.ctl & CTL_PROP) && wm) {
            u32x4 vn;
            uint32_t okn, unn;
            src_chunk<NT>(d, R, c + 1, vn, okn, unn);
            store_masked(d.dst_sh + (uint64_t)(16 * e), window(prop_val(v, ok), prop_val(vn, okn), d.s), wm);
        }
    }
}

// Segmented flush: lanes hold findings for records `rec` (contiguous runs of
// equal values; inactive lanes carry rec = ~0).  Only called when some lane
// found something.
__device__ __forceinline__ void flush_segmented(Acc &a, uint64_t rec, cg_verdict *out)
{
    const uint32_t lane = lane_id();
    const uint64_t prev = __shfl_up(rec, 1);
    const bool head = lane == 0u || prev != rec;
    const uint64_t heads = __ballot(head);
    const uint64_t below = heads & (lane == 63u ? ~0ull : ((2ull << lane) - 1ull));
    const uint32_t start = 63u - (uint32_t)__builtin_clzll(below);
    for (uint32_t dd = 1; dd < 64u; dd <<= 1) {
        const uint64_t of = __shfl_up(a.first, dd);
        const uint64_t ou = __shfl_up(a.undef, dd);
        const uint32_t ofl = __shfl_up(a.flags, dd);
        if (lane >= dd && lane - dd >= start) {
            a.first = of < a.first ? of : a.first;
            a.undef += ou;
            a.flags |= ofl;
        }
    }
    const uint64_t next = __shfl_down(rec, 1);
    const bool tail = lane == 63u || next != rec;
    if (tail && rec != ~0ull && a.flags) {
        atomicOr(&out[rec].flags, a.flags);
        if (a.first != NONE) atomicMin((unsigned long long *)&out[rec].first_bad, (unsigned long long)a.first);
        if (a.undef) atomicAdd((unsigned long long *)&out[rec].undef_bytes, (unsigned long long)a.undef);
    }
    acc_reset(a);
}

// ---------------------------------------------------------------------------
// k_classify
// ---------------------------------------------------------------------------

// Largest index j with base[j] <= p among live allocations, if p < end[j].
__device__ __forceinline__ int64_t table_lookup(const TableView &tb, const uint64_t *top, uint64_t p)
{
    if (tb.n == 0 || top[0] > p) return -1;
    uint32_t lo = 0, hi = tb.ntop - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (top[mid] <= p) lo = mid; else hi = mid - 1;
    }
    uint64_t a = (uint64_t)lo << tb.top_shift;
    uint64_t b = a + (1ull << tb.top_shift);
    b = (b < tb.n ? b : tb.n) - 1;
    while (a < b) {
        const uint64_t mid = (a + b + 1) >> 1;
        if (tb.base[mid] <= p) a = mid; else b = mid - 1;
    }
    return p < tb.end[a] ? (int64_t)a : -1;
}

// wave-wide sum of a 32-bit value (every lane active)
__device__ __forceinline__ uint32_t wave_add32(uint32_t x)
{
    for (int d = 32; d >= 1; d >>= 1) x += (uint32_t)__shfl_xor((int)x, d);
    return x;
}

// The table search of table_lookup done by one wave (every lane active): the
// top level, then the segment of 2^top_shift entries it picks, are each
// compared 64 entries at a time, so two rounds of independent loads take the
// place of a chain of dependent ones.  Entries are sorted by base, so the
// number of them at or below p is one past the last of them.
__device__ int64_t table_lookup_wave(const TableView &tb, uint64_t p)
{
    if (tb.n == 0) return -1;
    const uint32_t lane = lane_id();
    uint32_t c = 0;
    for (uint32_t k = lane; k < tb.ntop; k += 64) c += tb.top[k] <= p ? 1u : 0u;
    c = wave_add32(c);
    if (c == 0) return -1;
    const uint64_t a0 = (uint64_t)(c - 1) << tb.top_shift;
    const uint64_t a1 = a0 + (1ull << tb.top_shift) < tb.n ? a0 + (1ull << tb.top_shift) : tb.n;
    uint32_t c2 = 0;
    for (uint64_t k = a0 + lane; k < a1; k += 64) c2 += tb.base[k] <= p ? 1u : 0u;
    c2 = wave_add32(c2);
    const uint64_t j = a0 + c2 - 1;   // base[a0] is top[c - 1] <= p, so c2 >= 1
    return p < tb.end[j] ? (int64_t)j : -1;
}

// Byte indices i in [0, n) with hb <= p + i < hb + hl, as [lo, hi) (empty: 0, 0).
__device__ __forceinline__ void region_clip(uint64_t p, uint64_t n, uint64_t hb, uint64_t hl,
                                            uint64_t &lo, uint64_t &hi)
{
    lo = hi = 0;
    if (hl == 0) return;
    if (p >= hb) {
        const uint64_t off = p - hb;
        if (off >= hl) return;
        lo = 0;
        hi = (n < hl - off) ? n : hl - off;
    } else {
        const uint64_t gap = hb - p;
        if (gap >= n) return;
        lo = gap;
        hi = (n - gap > hl) ? gap + hl : n;
    }
}

__device__ __forceinline__ uint64_t clamp_scan(uint64_t x) { return x < kScanLimit ? x : kScanLimit; }

// does the record have a device source / destination to look up?
__device__ __forceinline__ bool dev_src(const cg_transfer &r) { return r.kind <= CG_D2D && r.n && r.kind != CG_H2D; }
__device__ __forceinline__ bool dev_dst(const cg_transfer &r) { return r.kind <= CG_D2D && r.n && r.kind != CG_D2H; }

// Decode record r, given the table entries holding its device source and
// destination pointers (js, jd: -1 when none, or when the side is on the
// host): its descriptor, its verdict's range-derived fields, and its number
// of units (returned).
__device__ uint64_t classify_rec(const cg_transfer &r, uint32_t mode, const DevState &st, int64_t js, int64_t jd,
                                 Desc &ds, cg_verdict &v)
{
    const uint64_t n = r.n;
    ds = Desc{};
    uint32_t flags = 0;
    uint64_t first = NONE, avail = 0;
    const bool check = (mode & CG_CHECK) != 0;
    uint64_t units = 0;

    if (r.kind > CG_D2D) {
        flags = CG_BAD_KIND;
    } else if (n != 0) {
        const bool src_host = r.kind == CG_H2D;
        const bool dst_host = r.kind == CG_D2H;
        const Region &R = st.region;
        uint64_t vlo = 0, vhi = 0, dlo = 0, dhi = 0, avail_s = 0, avail_d = 0;
        uint32_t phi = 0, psi = 0;
        uint64_t src0 = 0, dst0 = 0;   // shadow address of byte 0 (when valid)
        bool src_ok = false, dst_ok = false;
        if (src_host) {
            region_clip(r.src, n, R.hb, R.hl, vlo, vhi);
            if (vhi <= vlo || vlo > 0) { flags |= CG_SRC_UNADDR; first = 0; }
            else if (vhi < n) { flags |= CG_SRC_UNADDR; first = first < vhi ? first : vhi; }
            src_ok = vhi > vlo;
            src0 = (uint64_t)R.v + (r.src - R.hb);
            phi = (uint32_t)((r.src - R.hb) & 15u);
            ds.a_src = (int64_t)((r.src - R.hb) - phi);
        } else {
            const int64_t j = js;
            if (j < 0) { flags |= CG_SRC_UNALLOC; first = 0; }
            else {
                avail_s = st.table.end[j] - r.src;
                if (n > avail_s) { flags |= CG_SRC_OVERRUN; first = first < avail_s ? first : avail_s; }
                vlo = 0;
                vhi = n < avail_s ? n : avail_s;
                src0 = st.pool + st.table.off[j] + (r.src - st.table.base[j]);
                phi = (uint32_t)(src0 & 15u);
                src_ok = true;
            }
        }
        if (dst_host) {
            region_clip(r.dst, n, R.hb, R.hl, dlo, dhi);
            if (dhi <= dlo || dlo > 0) { flags |= CG_DST_UNADDR; first = 0; }
            else if (dhi < n) { flags |= CG_DST_UNADDR; first = first < dhi ? first : dhi; }
            dst_ok = dhi > dlo;
            dst0 = (uint64_t)R.v + (r.dst - R.hb);
            psi = (uint32_t)((r.dst - R.hb) & 15u);
            ds.a_dst = (int64_t)((r.dst - R.hb) - psi);
        } else {
            const int64_t j = jd;
            if (j < 0) { flags |= CG_DST_UNALLOC; first = 0; }
            else {
                avail_d = st.table.end[j] - r.dst;
                if (n > avail_d) { flags |= CG_DST_OVERRUN; first = first < avail_d ? first : avail_d; }
                dlo = 0;
                dhi = n < avail_d ? n : avail_d;
                dst0 = st.pool + st.table.off[j] + (r.dst - st.table.base[j]);
                psi = (uint32_t)(dst0 & 15u);
                dst_ok = true;
            }
        }
        bool overlap = false;
        if (r.kind == CG_D2D) {
            overlap = (r.src < r.dst) ? (r.dst - r.src < n) : (r.src - r.dst < n);
            if (overlap) flags |= CG_OVERLAP;
        }
        avail = src_host ? avail_d : (dst_host ? avail_s : (avail_s < avail_d ? avail_s : avail_d));

        const bool prop = (mode & CG_PROPAGATE) && !overlap;
        const bool dsta = check && dst_host;
        const bool dstwork = (prop || dsta) && dst_ok;
        vlo = clamp_scan(vlo); vhi = clamp_scan(vhi);
        dlo = clamp_scan(dlo); dhi = clamp_scan(dhi);
        const uint32_t delta = (dstwork && phi < psi) ? 1u : 0u;
        // unit ranges of the source and destination sides
        uint64_t e_lo = ~0ull, e_hi = 0;
        if (src_ok && vhi > vlo) {
            const uint64_t c_lo = (vlo + phi) >> 4, c_hi = ((vhi - 1 + phi) >> 4) + 1;
            e_lo = c_lo + delta;
            e_hi = c_hi + delta;
            // propagation needs every destination chunk, including those whose
            // bytes come only from invalid source bytes (written as 0xFF)
        }
        if (dstwork && dhi > dlo) {
            const uint64_t f_lo = (dlo + psi) >> 4, f_hi = ((dhi - 1 + psi) >> 4) + 1;
            e_lo = f_lo < e_lo ? f_lo : e_lo;
            e_hi = f_hi > e_hi ? f_hi : e_hi;
        }
        if (e_hi > e_lo) units = e_hi - e_lo; else e_lo = 0;
        ds.src_sh = src0 - phi;
        ds.dst_sh = dst0 - psi;
        ds.v_lo = (int64_t)vlo; ds.v_hi = (int64_t)vhi;
        ds.d_lo = (int64_t)dlo; ds.d_hi = (int64_t)dhi;
        ds.e0 = e_lo;
        ds.units = units;
        ds.ctl = (src_host ? CTL_SRC_HOST : 0u) | (dst_host ? CTL_DST_HOST : 0u) | (check ? CTL_CHECK : 0u) |
                 (prop && dst_ok ? CTL_PROP : 0u) | (dsta && dst_ok ? CTL_DST_A : 0u) |
                 (phi << CTL_PHI_SHIFT) | (psi << CTL_PSI_SHIFT) | (delta ? CTL_DELTA : 0u);
        if (!src_ok) { ds.v_lo = 0; ds.v_hi = 0; }
    }
    v.flags = flags;
    v.reserved = 0;
    v.first_bad = first;
    v.undef_bytes = 0;
    v.avail = avail;
    return units;
}

// Marks the steps (2^16 bytes of V) of shadow space k that hold its bytes
// [lo, hi), for that index's counting pass: bytes before the first 16-aligned
// step, then 16 marks per store.
__device__ __forceinline__ void mark_steps(const BatchArgs &a, int k, uint64_t lo, uint64_t hi)
{
    uint8_t *m = a.index_mark[k];
    if (!m || hi <= lo) return;
    uint64_t s = lo >> kIdxStepShift, e = ((hi - 1) >> kIdxStepShift) + 1;
    if (e > a.mark_cap[k]) e = a.mark_cap[k];
    for (; s < e && (s & 15u); ++s) m[s] = 1;
    for (; s + 16 <= e; s += 16) *reinterpret_cast<uint4 *>(m + s) = make_uint4(0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u);
    for (; s < e; ++s) m[s] = 1;
}

// space offsets of a descriptor's byte 0: of its source (host region or pool)
// and of a host destination
__device__ __forceinline__ uint64_t src_space_off(const Desc &ds, const DevState &st)
{
    const uint32_t phi = (ds.ctl >> CTL_PHI_SHIFT) & 15u;
    return (ds.ctl & CTL_SRC_HOST) ? (uint64_t)(ds.a_src + (int64_t)phi) : ds.src_sh + phi - st.pool;
}

__device__ __forceinline__ uint64_t dst_space_off(const Desc &ds)
{
    return (uint64_t)(ds.a_dst + (int64_t)((ds.ctl >> CTL_PSI_SHIFT) & 15u));
}

// the steps a transfer's index answer reads: its valid source bytes, and a
// host destination's valid bytes
__device__ __forceinline__ void mark_desc(const BatchArgs &a, const DevState &st, const Desc &ds)
{
    if (ds.v_hi > ds.v_lo) {
        const uint64_t o = src_space_off(ds, st);
        mark_steps(a, (ds.ctl & CTL_SRC_HOST) ? 0 : 1, o + (uint64_t)ds.v_lo, o + (uint64_t)ds.v_hi);
    }
    if ((ds.ctl & CTL_DST_A) && ds.d_hi > ds.d_lo) {
        const uint64_t o = dst_space_off(ds);
        mark_steps(a, 0, o + (uint64_t)ds.d_lo, o + (uint64_t)ds.d_hi);
    }
}

// Record t of a batch: its descriptor and work weight, and its verdict's
// range-derived fields; returns its number of units (and in sp[0], sp[1] its
// valid bytes in the host region and in the shadow pool, when sp is given).
__device__ uint64_t classify_one(const BatchArgs &a, const DevState &st, uint64_t t, const uint64_t *top,
                                 uint64_t *sp = nullptr)
{
    const cg_transfer r = a.recs[t];
    const int64_t js = dev_src(r) ? table_lookup(st.table, top, r.src) : -1;
    const int64_t jd = dev_dst(r) ? table_lookup(st.table, top, r.dst) : -1;
    Desc ds;
    cg_verdict v;
    const uint64_t units = classify_rec(r, a.mode, st, js, jd, ds, v);
    if (sp) {
        const uint64_t src = ds.v_hi > ds.v_lo ? (uint64_t)(ds.v_hi - ds.v_lo) : 0;
        const uint64_t dst = (ds.ctl & CTL_DST_A) && ds.d_hi > ds.d_lo ? (uint64_t)(ds.d_hi - ds.d_lo) : 0;
        sp[0] = ((ds.ctl & CTL_SRC_HOST) ? src : 0) + dst;
        sp[1] = (ds.ctl & CTL_SRC_HOST) ? 0 : src;
        mark_desc(a, st, ds);
    }
    a.desc[t] = ds;
    a.weight[t] = units;
    if (a.out && (a.mode & CG_CHECK)) a.out[t] = v;
    return units;
}

__global__ void __launch_bounds__(kClassifyBlock) k_classify(BatchArgs a)
{
    __shared__ uint64_t top[kMaxTop];
    __shared__ uint64_t wsum[kClassifyBlock / 64];
    __shared__ uint64_t isum[2][kClassifyBlock / 64];
    const uint32_t tid = threadIdx.x;
    const DevState st = *a.st;
    for (uint32_t k = tid; k < st.table.ntop; k += kClassifyBlock) top[k] = st.table.top[k];
    __syncthreads();
    const uint64_t t = (uint64_t)blockIdx.x * kClassifyBlock + tid;
    uint64_t w = 0, sp[2] = {0, 0};
    if (t < a.count) {
        const uint64_t u = classify_one(a, st, t, top, sp);
        w = u ? u : 1;
    }
    const uint32_t lane = lane_id(), wid = tid >> 6;
    if (a.index_bytes[0]) {
        // the batch's valid bytes per shadow space (the shadow indexes' cost
        // test): wave sums here, one atomic per block below
        for (int k = 0; k < 2; ++k) {
            uint64_t x = sp[k];
            for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d);
            if (lane == 0) isum[k][wid] = x;
        }
    }
    // block exclusive scan of w
    uint64_t x = w;
    for (uint32_t d = 1; d < 64u; d <<= 1) {
        const uint64_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63u) wsum[wid] = x;
    __syncthreads();
    uint64_t off = 0;
    for (uint32_t k = 0; k < wid; ++k) off += wsum[k];
    if (t < a.count) a.local[t] = off + x - w;
    if (tid == kClassifyBlock - 1) a.bsum[blockIdx.x] = off + x;
    if (a.index_bytes[0] && tid == 0)
        for (int k = 0; k < 2; ++k) {
            uint64_t b = 0;
            for (uint32_t q = 0; q < kClassifyBlock / 64; ++q) b += isum[k][q];
            if (b) atomicAdd((unsigned long long *)a.index_bytes[k], (unsigned long long)b);
        }
}

// After the shadow indexes have answered positions (their weight set to 0)
// of a batch in its given order: each position's weight max(units, 1) again,
// with the block-local prefix and block sums that k_classify leaves.
__global__ void __launch_bounds__(kClassifyBlock) k_reweigh(BatchArgs a)
{
    __shared__ uint64_t wsum[kClassifyBlock / 64];
    const uint32_t tid = threadIdx.x;
    const uint64_t t = (uint64_t)blockIdx.x * kClassifyBlock + tid;
    uint64_t w = 0;
    if (t < a.count) {
        const uint64_t u = a.weight[t];
        w = u ? u : 1;
    }
    const uint32_t lane = lane_id(), wid = tid >> 6;
    uint64_t x = w;
    for (uint32_t d = 1; d < 64u; d <<= 1) {
        const uint64_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63u) wsum[wid] = x;
    __syncthreads();
    uint64_t off = 0;
    for (uint32_t k = 0; k < wid; ++k) off += wsum[k];
    if (t < a.count) a.local[t] = off + x - w;
    if (tid == kClassifyBlock - 1) a.bsum[blockIdx.x] = off + x;
}

// ---------------------------------------------------------------------------
// pitched 2D records (check_transfers_2d) as positions of their own
// ---------------------------------------------------------------------------


// rows of a 2D record that are worked: every row below index 2^32 that
// starts below byte 2^62 of the record (its bytes are numbered row by row)
__device__ __forceinline__ uint64_t rows_worked(const cg_transfer2d &r)
{
    if (r.width == 0 || r.rows == 0) return 0;
    const uint64_t lim = r.width >= kScanLimit ? 1 : (kScanLimit + r.width - 1) / r.width;
    uint64_t n = r.rows < lim ? r.rows : lim;
    return n < (1ull << 32) ? n : (1ull << 32);
}

// A bound of the bytes from any row's start to the end of that row's valid
// source and destination parts, for a record whose rows do not follow row 0:
// a device side ends within its allocation (none is larger than
// st.size_bound); a host side ends within the region, at most `gap + hl`
// bytes from a row that starts `gap` bytes below it.  The host side's rows
// start no lower than row 0 unless their addresses wrap past 2^64.
__device__ __forceinline__ uint64_t row_extent_bound(const Pitch &P, uint64_t rows, const DevState &st)
{
    uint64_t e = st.size_bound;
    if (P.kind == CG_H2D || P.kind == CG_D2H) {
        const Region &R = st.region;
        const uint64_t p = P.kind == CG_H2D ? P.src : P.dst, q = P.kind == CG_H2D ? P.spitch : P.dpitch;
        const bool wraps = q != 0 && rows > 1 && rows - 1 > (~0ull - p) / q;
        const uint64_t gap = wraps ? R.hb : (p < R.hb ? R.hb - p : 0);
        const uint64_t h = gap + R.hl;
        e = e > h ? e : h;
    }
    return e;
}

// do rows 0 .. n-1 of one side, starting at p with pitch q and `w` bytes
// long, all lie in [lo, hi)?  (p >= lo is known)
__device__ __forceinline__ bool rows_inside(uint64_t p, uint64_t q, uint64_t w, uint64_t n, uint64_t lo, uint64_t hi)
{
    (void)lo;
    if (p >= hi || w > hi - p) return false;
    if (n <= 1 || q == 0) return true;
    return n - 1 <= (hi - p - w) / q;   // p + (n-1) q + w <= hi
}

// the transfer record of row r
__device__ __forceinline__ cg_transfer row_record(const Pitch &P, uint64_t r)
{
    return cg_transfer{P.src + r * P.spitch, P.dst + r * P.dpitch, P.width, P.kind, 0u};
}

// The steps the index answer of a record whose rows follow row 0 reads: on
// each side, the span from the first row's start to the last row's end when
// it is at most 4 times the rows' bytes (plus 4 steps); a sparser side asks
// for every step of its space instead, so that marking stays within a
// fraction of the bytes the rows hold.
__device__ __forceinline__ void mark_rows(const BatchArgs &a, const DevState &st, const Desc &ds, const Pitch &P)
{
    auto side = [&](int k, uint64_t o, uint64_t q) {
        const uint64_t span = (P.rows - 1) * q + P.width;
        if (span / 4 <= P.rows * P.width + (4ull << kIdxStepShift)) mark_steps(a, k, o, o + span);
        else a.index_bytes[k][kIdxAll] = 1;
    };
    if (ds.v_hi > ds.v_lo) side((ds.ctl & CTL_SRC_HOST) ? 0 : 1, src_space_off(ds, st), P.spitch);
    if ((ds.ctl & CTL_DST_A) && ds.d_hi > ds.d_lo) side(0, dst_space_off(ds), P.dpitch);
}

// One lane per pitched 2D record: row 0 looked up and classified (its
// descriptor is the position's), whether every row follows from it, the
// units (rows * upr) and the verdict before any row is worked: row 0's when
// the rows are uniform, else {0, NONE, 0, row 0's avail} (the rows bring
// their own flags), with ROWS_LIMIT when not every row is worked.  A record
// with no rows or width 0 gives {0, NONE, 0, 0}, one with rows and a bad
// kind {BAD_KIND, NONE, 0, 0}; both weigh 1 and have no units.  upr bounds
// the units of every row: a uniform row's follow from the width, any other
// row's from the extent of its valid parts (so a bogus width costs no more
// than the memory its rows can reach).
__global__ void __launch_bounds__(kClassifyBlock) k_classify_2d(BatchArgs a, const cg_transfer2d *recs2d, Pitch *pitch)
{
    __shared__ uint64_t top[kMaxTop];
    __shared__ uint64_t wsum[kClassifyBlock / 64];
    __shared__ uint64_t isum[2][kClassifyBlock / 64];
    uint64_t ib[2] = {0, 0};   // this record's valid bytes per shadow space (the indexes' cost test)
    const uint32_t tid = threadIdx.x;
    const DevState st = *a.st;
    for (uint32_t k = tid; k < st.table.ntop; k += kClassifyBlock) top[k] = st.table.top[k];
    __syncthreads();
    const uint64_t t = (uint64_t)blockIdx.x * kClassifyBlock + tid;
    uint64_t w = 0;
    if (t < a.count) {
        const cg_transfer2d R2 = recs2d[t];
        Pitch P{R2.src, R2.dst, R2.width, R2.rows, R2.spitch, R2.dpitch, 0, R2.kind, 0};
        Desc ds = {};
        cg_verdict v{0u, 0u, NONE, 0, 0};
        uint64_t units = 0;
        const uint64_t rows = rows_worked(R2);
        if (rows == 0) {
            // nothing to check
        } else if (R2.kind > CG_D2D) {
            v.flags = CG_BAD_KIND;
        } else {
            const cg_transfer r0 = row_record(P, 0);
            const int64_t js = dev_src(r0) ? table_lookup(st.table, top, r0.src) : -1;
            const int64_t jd = dev_dst(r0) ? table_lookup(st.table, top, r0.dst) : -1;
            cg_verdict v0;
            const uint64_t u0 = classify_rec(r0, a.mode, st, js, jd, ds, v0);
            const Region &R = st.region;
            auto side_ok = [&](bool host, int64_t j, uint64_t p, uint64_t q) {
                if (host) return R.hl > 0 && p >= R.hb && rows_inside(p, q, P.width, rows, R.hb, R.hb + R.hl);
                return j >= 0 && rows_inside(p, q, P.width, rows, st.table.base[j], st.table.end[j]);
            };
            const bool uniform = (v0.flags & ~CG_OVERLAP) == 0 && (R2.kind != CG_D2D || R2.spitch == R2.dpitch) &&
                                 side_ok(R2.kind == CG_H2D, js, P.src, P.spitch) &&
                                 side_ok(R2.kind == CG_D2H, jd, P.dst, P.dpitch);
            P.rows = rows;
            uint64_t ext = P.width < kScanLimit ? P.width : kScanLimit;
            if (!uniform) {
                const uint64_t b = row_extent_bound(P, rows, st);
                ext = b < ext ? b : ext;
            }
            // rows that follow row 0 at pitches that keep the 16-byte phases
            // all have row 0's units: no padding between rows
            const bool step = uniform && ((P.spitch | P.dpitch) & 15u) == 0 && u0 > 0;
            P.upr = step ? u0 : (ext + 14) / 16 + 2;
            P.uniform = uniform ? (step ? kRowsStep : kRowsUniform) : 0u;
            // rows back to back on every side the check reads: one transfer
            // (in the rows' allocations, so its lookups are row 0's)
            if (step && !(a.mode & CG_PROPAGATE) && R2.spitch == R2.width &&
                (R2.kind != CG_D2H || R2.dpitch == R2.width)) {
                const cg_transfer rc{P.src, P.dst, rows * P.width, P.kind, 0u};
                cg_verdict vc;
                P.upr = classify_rec(rc, a.mode, st, js, jd, ds, vc);
                P.uniform = kRowsContig;
            }
            units = P.uniform == kRowsContig ? P.upr : rows * P.upr;
            if (P.uniform && a.index_bytes[0]) {
                // the valid bytes read per shadow space, for the indexes' cost
                // test: one transfer's, or row 0's times the rows
                const uint64_t nr = P.uniform == kRowsContig ? 1 : rows;
                const uint64_t src = ds.v_hi > ds.v_lo ? nr * (uint64_t)(ds.v_hi - ds.v_lo) : 0;
                const uint64_t dst = (ds.ctl & CTL_DST_A) && ds.d_hi > ds.d_lo ? nr * (uint64_t)(ds.d_hi - ds.d_lo) : 0;
                ib[0] = ((ds.ctl & CTL_SRC_HOST) ? src : 0) + dst;
                ib[1] = (ds.ctl & CTL_SRC_HOST) ? 0 : src;
                if (P.uniform == kRowsContig) mark_desc(a, st, ds);
                else mark_rows(a, st, ds, P);
            }
            v = uniform ? v0 : cg_verdict{0u, 0u, NONE, 0, v0.avail};
            if (rows < R2.rows) v.flags |= CG_ROWS_LIMIT;
        }
        pitch[t] = P;
        a.desc[t] = ds;
        a.weight[t] = units;
        if (a.out && (a.mode & CG_CHECK)) a.out[t] = v;
        w = units ? units : 1;
    }
    const uint32_t lane = lane_id(), wid = tid >> 6;
    if (a.index_bytes[0])
        for (int k = 0; k < 2; ++k) {
            uint64_t y = ib[k];
            for (int d = 32; d >= 1; d >>= 1) y += __shfl_xor(y, d);
            if (lane == 0) isum[k][wid] = y;
        }
    uint64_t x = w;
    for (uint32_t d = 1; d < 64u; d <<= 1) {
        const uint64_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63u) wsum[wid] = x;
    __syncthreads();
    uint64_t off = 0;
    for (uint32_t k = 0; k < wid; ++k) off += wsum[k];
    if (t < a.count) a.local[t] = off + x - w;
    if (tid == kClassifyBlock - 1) a.bsum[blockIdx.x] = off + x;
    // one atomic per block and space for the cost test
    if (a.index_bytes[0] && tid == 0)
        for (int k = 0; k < 2; ++k) {
            uint64_t b = 0;
            for (uint32_t q = 0; q < kClassifyBlock / 64; ++q) b += isum[k][q];
            if (b) atomicAdd((unsigned long long *)a.index_bytes[k], (unsigned long long)b);
        }
}

// Row r's descriptor when the rows are uniform: row 0's shifted by the
// pitches; the phases, and so the realignment and the unit range, are row r's.
__device__ Desc row_desc(const Desc &d0, const Pitch &P, uint64_t r)
{
    const uint32_t phi0 = (d0.ctl >> CTL_PHI_SHIFT) & 15u, psi0 = (d0.ctl >> CTL_PSI_SHIFT) & 15u;
    const uint64_t src0 = d0.src_sh + phi0 + r * P.spitch, dst0 = d0.dst_sh + psi0 + r * P.dpitch;
    const uint32_t phi = (uint32_t)(src0 & 15u), psi = (uint32_t)(dst0 & 15u);
    const bool dstwork = (d0.ctl & (CTL_PROP | CTL_DST_A)) != 0;
    const uint32_t delta = (dstwork && phi < psi) ? 1u : 0u;
    const uint64_t w = P.width;
    uint64_t e_lo = delta, e_hi = ((w - 1 + phi) >> 4) + 1 + delta;
    if (dstwork) {
        const uint64_t f_hi = ((w - 1 + psi) >> 4) + 1;
        e_lo = 0;
        e_hi = f_hi > e_hi ? f_hi : e_hi;
    }
    Desc x = d0;
    x.src_sh = src0 - phi;
    x.dst_sh = dst0 - psi;
    x.v_lo = 0;
    x.v_hi = (int64_t)w;
    x.d_lo = 0;
    x.d_hi = (int64_t)w;
    x.a_src = d0.a_src + (int64_t)phi0 + (int64_t)(r * P.spitch) - (int64_t)phi;
    x.a_dst = d0.a_dst + (int64_t)psi0 + (int64_t)(r * P.dpitch) - (int64_t)psi;
    x.e0 = e_lo;
    x.units = e_hi - e_lo;
    x.ctl = (d0.ctl & ~((15u << CTL_PHI_SHIFT) | (15u << CTL_PSI_SHIFT) | CTL_DELTA)) | (phi << CTL_PHI_SHIFT) |
            (psi << CTL_PSI_SHIFT) | (delta ? CTL_DELTA : 0u);
    return x;
}

// every field of a wave-uniform descriptor in scalar registers
__device__ __forceinline__ DV dv_uniform(const Desc &x)
{
    Desc u;
    u.src_sh = ufl64(x.src_sh); u.dst_sh = ufl64(x.dst_sh);
    u.v_lo = (int64_t)ufl64((uint64_t)x.v_lo); u.v_hi = (int64_t)ufl64((uint64_t)x.v_hi);
    u.d_lo = (int64_t)ufl64((uint64_t)x.d_lo); u.d_hi = (int64_t)ufl64((uint64_t)x.d_hi);
    u.a_src = (int64_t)ufl64((uint64_t)x.a_src); u.a_dst = (int64_t)ufl64((uint64_t)x.a_dst);
    u.e0 = ufl64(x.e0); u.units = ufl64(x.units); u.ctl = ufl32(x.ctl);
    return make_dv(u);
}

// findings of one row (row-relative byte indices) into a record's
// accumulator: byte c of row r is byte r * width + c of the record
__device__ __forceinline__ void acc_add_row(Acc &acc, const Acc &ra, uint32_t rflags, uint64_t rfirst, uint64_t base)
{
    acc.flags |= ra.flags | rflags;
    acc.undef += ra.undef;
    if (ra.first != NONE) acc_min(acc, (int64_t)(base + ra.first));
    if (rfirst != NONE) acc_min(acc, (int64_t)(base + rfirst));
}

// ---------------------------------------------------------------------------
// k_pointers: pointer queries (kernel arguments) against the live allocations,
// through the same table lookup as the transfers
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kClassifyBlock) k_pointers(const DevState *stp, const uint64_t *ptrs, uint64_t count,
                                                             cg_ptr_check *out)
{
    __shared__ uint64_t top[kMaxTop];
    const DevState st = *stp;
    for (uint32_t k = threadIdx.x; k < st.table.ntop; k += kClassifyBlock) top[k] = st.table.top[k];
    __syncthreads();
    const uint64_t t = (uint64_t)blockIdx.x * kClassifyBlock + threadIdx.x;
    if (t >= count) return;
    const uint64_t p = ptrs[t];
    int64_t j = table_lookup(st.table, top, p);
    if (j < 0 && p > 0) {
        // one past the end of an allocation
        const int64_t k = table_lookup(st.table, top, p - 1);
        if (k >= 0 && st.table.end[k] == p) j = k;
    }
    cg_ptr_check o;
    o.reserved = 0;
    if (j < 0) {
        o.flags = CG_PTR_UNALLOC;
        o.base = 0;
        o.avail = 0;
    } else {
        o.flags = 0;
        o.base = st.table.base[j];
        o.avail = st.table.end[j] - p;
    }
    out[t] = o;
}

// MI355X has 8 XCDs, each with its own L2; the blocks of a launch are placed
// on them round robin (block b on XCD b mod 8).
constexpr uint32_t kXcds = 8;
constexpr uint64_t kNoTile = ~0ull;

// ---------------------------------------------------------------------------
// k_scan_sums: one block, exclusive scan of the classify-block sums
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_scan_sums(BatchArgs a, uint32_t tile_units, uint32_t waves)
{
    __shared__ uint64_t wsum[16];
    const uint32_t tid = threadIdx.x, lane = lane_id(), wid = tid >> 6;
    const uint64_t nb = (a.count + kClassifyBlock - 1) / kClassifyBlock;
    const uint64_t per = (nb + 1023) / 1024;
    const uint64_t b0 = tid * per, b1 = (b0 + per < nb) ? b0 + per : nb;
    uint64_t s = 0;
    for (uint64_t b = b0; b < b1; ++b) s += a.bsum[b];
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
        a.boff[b] = run;
        run += a.bsum[b];
    }
    if (tid == 1023) {
        const uint64_t total = off + x;
        // tiles of at most tile_units, small enough that every wave of the
        // persistent grid gets a few of them, and few enough to fit tile_start
        uint64_t tu = tile_units;
        while (tu > kMinTile && (total + tu - 1) / tu < 4ull * waves) tu >>= 1;
        while ((total + tu - 1) / tu > a.tiles_cap) tu <<= 1;
        a.ctl->total_units = total;
        a.ctl->tile_units = tu;
        a.ctl->ntiles = (total + tu - 1) / tu;
        for (int x = 0; x < kXcds; ++x) {
            a.ctl->counter[x] = 0;
            a.ctl->lds_counter[x] = 0;
        }
        a.prefix[a.count] = total;
    }
}

// ---------------------------------------------------------------------------
// k_prefix_tiles: global prefix; k_tile_starts: first record of every tile
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_prefix_tiles(BatchArgs a)
{
    const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= a.count) return;
    a.prefix[t] = a.local[t] + a.boff[t / kClassifyBlock];
}

// One lane per tile (grid-stride): the last record whose prefix is at or
// below the tile's first unit.  Prefixes strictly increase (weights >= 1)
// except over a tail of empty positions of weight 0 (a segmented batch),
// where they equal the total, above every unit.
__global__ void __launch_bounds__(256) k_tile_starts(BatchArgs a)
{
    const uint64_t ntiles = a.ctl->ntiles, tu = a.ctl->tile_units;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < ntiles; j += stride) {
        const uint64_t u = j * tu;
        uint64_t lo = 0, hi = a.count - 1;
        while (lo < hi) {
            const uint64_t mid = (lo + hi + 1) >> 1;
            if (a.prefix[mid] <= u) lo = mid; else hi = mid - 1;
        }
        a.tile_start[j] = (uint32_t)lo;
    }
}

// ---------------------------------------------------------------------------
// k_batched: persistent kernel over the tiles of the flattened unit space
// ---------------------------------------------------------------------------

// Units [k0, k1) of a pitched record whose rows step by the pitches with row
// 0's phases (kRowsStep), checked without propagation, by the whole wave:
// the rows' units follow each other with no gap (upr is a row's units), and
// each lane works its own unit of an iteration in whichever row it falls, so
// that short rows and row ends share iterations.  d is row 0's descriptor;
// row r's source and destination lie r * spitch and r * dpitch further on.
template <int U, bool NT>
__device__ void run_rows_flat(const DV &d, const Pitch &P, const Region &R, uint64_t k0, uint64_t k1, Acc &acc)
{
    const uint32_t lane = lane_id();
    const uint64_t ur = P.upr;
    const bool src_host = (d.ctl & CTL_SRC_HOST) != 0;
    const bool dsta = (d.ctl & CTL_DST_A) != 0;
    const uint64_t a16b = (uint64_t)R.a16;
    uint64_t rb = k0 / ur, jb = k0 - rb * ur;   // row and unit of the iteration's first unit
    for (uint64_t kb = k0; kb < k1; kb += 64u * U) {
        u32x4 v[U];
        uint32_t ms[U], as[U], md[U], ad[U];
        int64_t fs[U], fd[U] = {};   // record byte index of byte 0 of the source / destination chunk
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint32_t c = 64u * j + lane;
            uint64_t r = rb, q = jb + c;
            if (q >= ur) {
                // ur >= 64 U: q < 2 ur; else q < ur + 64 U, small
                const uint64_t x = ur >= 64u * U ? 1u : (uint64_t)((uint32_t)q / (uint32_t)ur);
                r += x;
                q -= x * ur;
            }
            const bool live = kb + c < k1;
            const int64_t cs = (int64_t)(d.e0 + q) - (int64_t)d.delta;
            const int64_t i0 = 16 * cs - (int64_t)d.phi;
            const int64_t base = (int64_t)(r * P.width);
            fs[j] = base + i0;
            ms[j] = live ? rmask(d.v_lo - i0, d.v_hi - i0) : 0u;
            v[j] = u32x4{0u, 0u, 0u, 0u};
            as[j] = 0xFFFFu;
            if (ms[j]) {
                v[j] = ld16<NT>(d.src_sh + r * P.spitch + (uint64_t)(16 * cs));
                if (src_host) as[j] = ld_u16(a16b + (((uint64_t)(d.a_src + 16 * cs) + r * P.spitch) >> 3));
            }
            md[j] = 0u;
            ad[j] = 0xFFFFu;
            if (dsta) {
                const int64_t e = (int64_t)(d.e0 + q);
                const int64_t i0d = 16 * e - (int64_t)d.psi;
                fd[j] = base + i0d;
                md[j] = live ? rmask(d.d_lo - i0d, d.d_hi - i0d) : 0u;
                if (md[j]) ad[j] = ld_u16(a16b + (((uint64_t)(d.a_dst + 16 * e) + r * P.dpitch) >> 3));
            }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            src_findings(acc, fs[j], v[j], ms[j] & as[j], ms[j] & ~as[j]);
            const uint32_t ud = md[j] & ~ad[j];
            if (dsta && ud) {
                acc.flags |= CG_DST_UNADDR;
                acc_min(acc, fd[j] + __builtin_ctz(ud));
            }
        }
        jb += 64u * U;
        if (jb >= ur) {
            const uint64_t x = ur >= 64u * U ? 1u : (uint64_t)((uint32_t)jb / (uint32_t)ur);
            rb += x;
            jb -= x * ur;
        }
    }
}

// Units [k0, k1) of pitched position t, by the whole wave: row by row, each
// row's own units through the wave-uniform loop; rows that do not follow row
// 0 are looked up (64 table entries per step) and classified here, and their
// range-derived flags join the record's (OR and min: a row worked in parts by
// several waves adds them more than once to the same effect).
template <int U, bool NT, bool PROP>
__device__ void run_pitched(const BatchArgs &a, const DevState *st, uint64_t t, uint64_t k0, uint64_t k1, Acc &acc)
{
    const Pitch &Pg = a.pitch[t];
    Pitch P;
    P.src = ufl64(Pg.src); P.dst = ufl64(Pg.dst); P.width = ufl64(Pg.width); P.rows = ufl64(Pg.rows);
    P.spitch = ufl64(Pg.spitch); P.dpitch = ufl64(Pg.dpitch); P.upr = ufl64(Pg.upr);
    P.kind = ufl32(Pg.kind); P.uniform = ufl32(Pg.uniform);
    const Desc d0 = a.desc[t];
    if (!PROP && P.uniform == kRowsContig) {   // (made only for checks without propagation)
        run_uniform<U, NT, false>(dv_uniform(d0), st->region, k0, k1, acc);
        return;
    }
    // rows shorter than 64 units share iterations (at most 4 chunks per
    // lane: every lane keeps a row's worth of indices for each); longer rows
    // go row by row, their interiors through the unmasked loads
    constexpr int UF = U > 4 ? 4 : U;
    if (!PROP && P.uniform == kRowsStep && P.upr < 64u) {
        run_rows_flat<UF, NT>(dv_uniform(d0), P, st->region, k0, k1, acc);
        return;
    }
    const uint64_t r0 = k0 / P.upr;
    // kRowsStep: each next row's descriptor is the last one's moved by the pitches
    DV ds = dv_uniform(row_desc(d0, P, r0));
    for (uint64_t r = r0; r * P.upr < k1; ++r) {
        const uint64_t j0 = (k0 > r * P.upr ? k0 : r * P.upr) - r * P.upr;
        const uint64_t j1 = (k1 < (r + 1) * P.upr ? k1 : (r + 1) * P.upr) - r * P.upr;
        uint32_t rflags = 0;
        uint64_t rfirst = NONE;
        DV d;
        if (P.uniform == kRowsStep) {
            d = ds;
            ds.src_sh += P.spitch;
            ds.dst_sh += P.dpitch;
            ds.a_src += (int64_t)P.spitch;
            ds.a_dst += (int64_t)P.dpitch;
        } else if (P.uniform) {
            d = dv_uniform(row_desc(d0, P, r));
        } else {
            const cg_transfer row = row_record(P, r);
            const int64_t js = dev_src(row) ? table_lookup_wave(st->table, row.src) : -1;
            const int64_t jd = dev_dst(row) ? table_lookup_wave(st->table, row.dst) : -1;
            Desc x;
            cg_verdict v;
            classify_rec(row, a.mode, *st, js, jd, x, v);
            rflags = ufl32(v.flags);
            rfirst = ufl64(v.first_bad);
            d = dv_uniform(x);
        }
        Acc ra;
        acc_reset(ra);
        const uint64_t e = j1 < d.units ? j1 : d.units;
        if (e > j0) run_uniform<U, NT, PROP>(d, st->region, j0, e, ra);
        acc_add_row(acc, ra, rflags, rfirst, r * P.width);
    }
}

// Unit k of pitched position t, by one lane (short rows, tile ends).
template <bool NT, bool PROP>
__device__ void run_unit_pitched(const BatchArgs &a, const DevState *st, uint64_t t, uint64_t k, Acc &acc)
{
    const Pitch P = a.pitch[t];
    if (P.upr == 0) return;   // no rows, or a bad kind: nothing to work
    if (!PROP && P.uniform == kRowsContig) {
        const DV d = load_desc(a.desc, t);
        if (k < d.units) run_unit<NT, false>(d, st->region, k, acc);
        return;
    }
    const uint64_t r = k / P.upr, j = k - r * P.upr;
    uint32_t rflags = 0;
    uint64_t rfirst = NONE;
    Desc x;
    if (P.uniform) {
        x = row_desc(a.desc[t], P, r);
    } else {
        const cg_transfer row = row_record(P, r);
        const int64_t js = dev_src(row) ? table_lookup(st->table, st->table.top, row.src) : -1;
        const int64_t jd = dev_dst(row) ? table_lookup(st->table, st->table.top, row.dst) : -1;
        cg_verdict v;
        classify_rec(row, a.mode, *st, js, jd, x, v);
        rflags = v.flags;
        rfirst = v.first_bad;
    }
    const DV d = make_dv(x);
    Acc ra;
    acc_reset(ra);
    if (j < d.units) run_unit<NT, PROP>(d, st->region, j, ra);
    acc_add_row(acc, ra, rflags, rfirst, r * P.width);
}

// Blocks b = x, x + nch, x + 2 nch, ... of the grid run on XCD x; b / nch is
// their rank there.  A work queue split into nch chunks gives each claiming
// block of XCD x a first item of chunk x by rank, without an atomic.  claim
// 0: every block claims; 1: the blocks of even rank; 2: those of odd rank.
__device__ __forceinline__ uint32_t claimers_on(uint32_t x, uint32_t nch, int claim)
{
    const uint32_t n = (gridDim.x + nch - 1 - x) / nch;
    return claim == 0 ? n : (claim == 1 ? (n + 1) / 2 : n / 2);
}

__device__ __forceinline__ int64_t claim_rank(uint32_t nch, int claim)
{
    const uint32_t r = blockIdx.x / nch;
    if (claim == 0) return r;
    return (int)(r & 1u) == claim - 1 ? (int64_t)(r >> 1) : -1;
}

// The waves' loop of the scan kernel (claim: which blocks take first tiles;
// PITCH: the positions are pitched 2D records, a.pitch).
template <int U, bool NT, bool PROP, bool PITCH, int CLAIM>
__device__ void batched_loop(const BatchArgs &a)
{
    const uint32_t lane = lane_id();
    const uint64_t ntiles = ufl64(a.ctl->ntiles);
    const uint64_t tu = ufl64(a.ctl->tile_units);
    const uint64_t total = ufl64(a.ctl->total_units);
    const uint64_t T = a.count;
    const Region R = a.st->region;
    Acc acc;
    acc_reset(acc);
    // Tiles are split into kXcds contiguous chunks, chunk x worked by the
    // waves of the blocks that run on XCD x, in ascending order, so that the
    // neighbouring segments of a batch sorted by source block share that
    // XCD's L2.
    // First tile: the wave's own index in its chunk (no atomic, so that the
    // waves of a small batch leave at once); later tiles from the chunk's
    // counter; a wave whose chunk is used up takes tiles from the others'.
    // Only a batch worked as segments has that locality to keep; any
    // other batch is one chunk for all waves (tiles interleaved over XCDs).
    const uint32_t nch = a.perm ? kXcds : 1u;
    const uint32_t wpb = blockDim.x >> 6;
    const uint32_t xcd = blockIdx.x % nch;
    auto chunk_lo = [&](uint32_t x) { return ntiles * x / nch; };
    auto waves_on = [&](uint32_t x) { return (uint64_t)claimers_on(x, nch, CLAIM) * wpb; };
    const int64_t rank = claim_rank(nch, CLAIM);
    uint64_t jn = kNoTile;
    if (rank >= 0) {
        jn = chunk_lo(xcd) + (uint64_t)rank * wpb + (threadIdx.x >> 6);
        if (jn >= chunk_lo(xcd + 1)) jn = kNoTile;
    }
    uint32_t y = xcd, left = nch;
    for (;;) {
        while (jn == kNoTile && left > 0) {
            // a chunk no larger than its number of waves is all first tiles:
            // nothing to take there, and no atomic (small batches leave at once)
            const uint64_t lo = chunk_lo(y), hi = chunk_lo(y + 1);
            uint64_t c = hi;
            if (hi - lo > waves_on(y)) {
                uint32_t nx = 0;
                if (lane == 0) nx = atomicAdd(&a.ctl->counter[y], 1u);
                c = lo + waves_on(y) + ufl32(__shfl(nx, 0));
            }
            if (c < hi) {
                jn = c;
            } else {
                y = (y + 1) % nch;
                --left;
            }
        }
        if (jn == kNoTile) break;
        const uint64_t j = ufl64(jn);
        jn = kNoTile;
        uint64_t u = (uint64_t)j * tu;
        const uint64_t u_end = (u + tu < total) ? u + tu : total;
        uint64_t t = ufl32(a.tile_start[j]);
        // record t's units [pt, pt1) and, once loaded, its descriptor d; when a
        // record is finished by the wave-uniform loop, the next record's
        // metadata is loaded together with this record's data, so that
        // mid-size records do not pay two round trips each
        uint64_t pt = ufl64(a.prefix[t]), pt1 = ufl64(a.prefix[t + 1]);
        bool have_d = false;
        DV d = make_dv(Desc{});
        while (u < u_end) {
            // a run of 64 units or more goes through the wave-uniform loop whole
            // (its last iteration may be partial); shorter runs, which may hold
            // several records, go one unit per lane
            const uint64_t seg_end = pt1 < u_end ? pt1 : u_end;
            uint64_t nfull = seg_end - u >= 64 ? seg_end - u : 0;
            // pitched positions of short rows go one unit per lane (many rows
            // per wave), unless their rows share the wave's iterations
            if constexpr (PITCH) {
                const uint32_t un = ufl32(a.pitch[t].uniform);
                if (nfull && ufl64(a.pitch[t].upr) < 64 && un != kRowsContig && (PROP || un != kRowsStep))
                    nfull = 0;
            }
            if (nfull) {
                if (!have_d) d = load_desc_uniform(a.desc, t);
                const bool ahead = u + nfull == pt1 && u + nfull < u_end && t + 1 < T;
                uint64_t npt1 = pt1;
                DV nd = d;
                if (ahead) {
                    npt1 = ufl64(a.prefix[t + 2]);
                    nd = load_desc_uniform(a.desc, t + 1);
                }
                if constexpr (PITCH) run_pitched<U, NT, PROP>(a, a.st, t, u - pt, u - pt + nfull, acc);
                else run_uniform<U, NT, PROP>(d, R, u - pt, u - pt + nfull, acc);
                if (a.out) flush_wave(acc, a.out, a.perm ? ufl32(a.perm[t]) : t);
                u += nfull;
                if (u == pt1) {
                    ++t;
                    pt = pt1;
                    if (ahead) {
                        pt1 = npt1;
                        d = nd;
                        have_d = true;
                    } else {
                        if (u < u_end) pt1 = ufl64(a.prefix[t + 1]);
                        have_d = false;
                    }
                } else {
                    have_d = true;
                }
                continue;
            }
            // up to 64 units, one per lane, possibly of several records
            const uint64_t g_end = (u + 64 < u_end) ? u + 64 : u_end;
            const uint64_t ul = u + lane;
            const bool act = ul < g_end;
            uint64_t lo = t, hi = (t + 64 < T - 1) ? t + 64 : T - 1;
            while (lo < hi) {
                const uint64_t mid = (lo + hi + 1) >> 1;
                if (a.prefix[mid] <= ul) lo = mid; else hi = mid - 1;
            }
            const uint64_t tl = lo;
            if (PITCH && act) {
                run_unit_pitched<NT, PROP>(a, a.st, tl, ul - a.prefix[tl], acc);
            } else if (act) {
                const DV d = load_desc(a.desc, tl);
                const uint64_t k = ul - a.prefix[tl];
                if (k < d.units) run_unit<NT, PROP>(d, R, k, acc);
            }
            if (a.out && __ballot(acc.flags != 0u))
                flush_segmented(acc, act ? (a.perm ? (uint64_t)a.perm[tl] : tl) : ~0ull, a.out);
            else acc_reset(acc);
            if (g_end < u_end) {
                const uint64_t t63 = ufl64(__shfl(tl, 63));
                t = (ufl64(a.prefix[t63 + 1]) <= g_end) ? t63 + 1 : t63;
                pt = ufl64(a.prefix[t]);
                pt1 = ufl64(a.prefix[t + 1]);
                have_d = false;
            }
            u = g_end;
        }
    }
}

template <int U, bool NT, bool PROP>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(PROP ? 1 : 3))) k_batched(BatchArgs a)
{
    batched_loop<U, NT, PROP, false, 0>(a);
}

// the scan kernel over pitched 2D records (check_transfers_2d)
template <int U, bool NT, bool PROP>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(PROP ? 1 : 3))) k_batched_2d(BatchArgs a)
{
    batched_loop<U, NT, PROP, true, 0>(a);
}

// ---------------------------------------------------------------------------
// k_host_lds: host-source segments with their source bytes staged in LDS
// ---------------------------------------------------------------------------
// A batch worked as segments reads each host byte many times (about 160 on
// the 1M-record configuration), and through the vector memory path every
// re-read costs an address and an L2-to-L1 transfer.  Here the host-source
// positions (sorted last, by block of source memory) are taken in tasks of
// kTaskPos consecutive positions, each by one workgroup: for every window of
// kWinChunks chunks that the task's segments of one block touch, the window's
// V bytes and A bits are copied into LDS once, and every segment overlapping
// it is checked from there by one wave.  Only check-only host-to-device
// records have host sources worked here: their destination needs no check
// of its own.  Findings go to each position's record with the same atomics
// as in k_batched.  Tasks are split into one contiguous range per XCD, like
// k_batched's tiles, so that the tasks of one block stage it from one L2.
constexpr uint32_t kWinChunks = 2048;   // 32 KiB of V bytes per window
constexpr uint32_t kTaskPos = 256;      // positions per task, at most

// One position of a task, as the waves need it: absolute chunk indices (the
// shadow address over 16) of the segment's chunks [c_lo, c_hi), the record
// byte index i0 of chunk c_lo's first byte, the record's valid source bytes
// [v_lo, v_hi), and the verdict it reports to.
struct HostPos {
    int64_t c_lo, c_hi, i0, v_lo, v_hi;
    uint64_t blk;
    uint32_t rec, pad;
};

template <int U>
__device__ __forceinline__ void lds_segment(const HostPos &P, int64_t wc0, int64_t wc1, const u32x4 *sv,
                                            const uint16_t *sa, Acc &acc)
{
    const int64_t ca = P.c_lo > wc0 ? P.c_lo : wc0;
    const int64_t cb = P.c_hi < wc1 ? P.c_hi : wc1;
    const int32_t lane = (int32_t)lane_id();
    for (int64_t c = ca; c < cb; c += 64 * U) {
        const int64_t i0f = P.i0 + 16 * (c - P.c_lo);
        const int32_t base = (int32_t)(c - wc0);
        const int32_t n = (int32_t)(cb - c < 64 * U ? cb - c : 64 * U);
        // all U reads issued back to back: lanes past the segment's chunks in
        // this window read its last chunk again and ignore it
        u32x4 v[U];
        uint32_t av[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int32_t k = 64 * j + lane;
            const int32_t kk = k < n ? k : n - 1;
            v[j] = sv[base + kk];
            av[j] = sa[base + kk];
        }
        // every chunk of the iteration wholly valid: one test over them
        if (i0f >= P.v_lo && i0f + 16 * n <= P.v_hi) {
            uint32_t bad = 0;
#pragma unroll
            for (int j = 0; j < U; ++j) bad |= v[j].x | v[j].y | v[j].z | v[j].w | (av[j] ^ 0xFFFFu);
            if (__ballot(bad != 0u) == 0) continue;
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int32_t k = 64 * j + lane;
            const int64_t i0 = i0f + 16 * k;
            const uint32_t m = k < n ? rmask(P.v_lo - i0, P.v_hi - i0) : 0u;
            src_findings(acc, i0, v[j], m & av[j], m & ~av[j]);
        }
    }
}

// The workgroups' loop over the host-source tasks (claim: which blocks take
// first tasks, as in batched_loop); sv / sa / sp / s_task / s_next / s_list
// are the block's LDS.
template <int U>
__device__ void host_loop(const BatchArgs &a, const uint64_t *meta, int claim, u32x4 *sv, uint16_t *sa, HostPos *sp,
                          uint64_t *s_task, uint32_t *s_next, uint16_t *s_list)
{
    const uint64_t p_begin = meta[2], p_end = meta[0];
    if (p_begin >= p_end) return;
    const uint32_t lb = (uint32_t)meta[1];
    const uint32_t tp = a.task_pos ? a.task_pos : kTaskPos;   // positions per task, at most kTaskPos
    const uint64_t ntasks = (p_end - p_begin + tp - 1) / tp;
    const Region R = a.st->region;
    const int64_t vbase = (int64_t)((uint64_t)R.v >> 4);     // V is 16-byte aligned
    const int64_t nvch = (int64_t)((R.hl + 15) >> 4);         // chunks of V
    const int64_t nach = (int64_t)(((R.hl + 63) >> 6) * 4);   // 16-bit A words
    const gcptr<u32x4> gv = reinterpret_cast<gcptr<u32x4>>((uint64_t)R.v);
    const gcptr<uint16_t> ga = reinterpret_cast<gcptr<uint16_t>>((uint64_t)R.a16);
    // tasks in kXcds contiguous chunks, chunk x taken by the workgroups on XCD x
    auto chunk_lo = [&](uint32_t x) { return ntasks * x / kXcds; };
    auto groups_on = [&](uint32_t x) { return (uint64_t)claimers_on(x, kXcds, claim); };
    const uint32_t xcd = blockIdx.x % kXcds;
    const int64_t rank = claim_rank(kXcds, claim);
    uint64_t jn = kNoTile;
    if (rank >= 0) {
        jn = chunk_lo(xcd) + (uint64_t)rank;
        if (jn >= chunk_lo(xcd + 1)) jn = kNoTile;
    }
    uint32_t y = xcd, left = kXcds;
    Acc acc;
    acc_reset(acc);
    for (;;) {
        if (threadIdx.x == 0) {
            while (jn == kNoTile && left > 0) {
                const uint64_t lo = chunk_lo(y), hi = chunk_lo(y + 1);
                uint64_t c = hi;
                if (hi - lo > groups_on(y)) c = lo + groups_on(y) + atomicAdd(&a.ctl->lds_counter[y], 1u);
                if (c < hi) jn = c;
                else {
                    y = (y + 1) % kXcds;
                    --left;
                }
            }
            *s_task = jn;
        }
        __syncthreads();
        const uint64_t j = *s_task;
        jn = kNoTile;
        __syncthreads();
        if (j == kNoTile) break;
        const uint64_t q0 = p_begin + j * tp;
        const uint32_t np = (uint32_t)(p_end - q0 < tp ? p_end - q0 : tp);
        for (uint32_t t = threadIdx.x; t < np; t += blockDim.x) {
            const Desc d = a.desc[q0 + t];
            const uint32_t phi = (d.ctl >> CTL_PHI_SHIFT) & 15u;
            const int64_t e = (int64_t)d.e0 - ((d.ctl & CTL_DELTA) ? 1 : 0);
            HostPos h;
            h.c_lo = (int64_t)(d.src_sh >> 4) + e;
            h.c_hi = h.c_lo + (int64_t)d.units;
            h.i0 = 16 * e - (int64_t)phi;
            h.v_lo = d.v_lo;
            h.v_hi = d.v_hi;
            h.blk = (uint64_t)h.c_lo >> (lb - 4);
            h.rec = a.perm[q0 + t];
            h.pad = 0;
            sp[t] = h;
        }
        __syncthreads();
        // the task's positions by block (they are sorted by block)
        for (uint32_t g0 = 0; g0 < np;) {
            const uint64_t blk = sp[g0].blk;
            uint32_t g1 = g0 + 1;
            int64_t cmin = sp[g0].c_lo, cmax = sp[g0].c_hi;
            while (g1 < np && sp[g1].blk == blk) {
                cmin = sp[g1].c_lo < cmin ? sp[g1].c_lo : cmin;
                cmax = sp[g1].c_hi > cmax ? sp[g1].c_hi : cmax;
                ++g1;
            }
            for (int64_t wc0 = (cmin / kWinChunks) * kWinChunks; wc0 < cmax; wc0 += kWinChunks) {
                const int64_t wc1 = wc0 + kWinChunks;
                // stage the window: V chunks and A words inside the buffers,
                // zeros elsewhere; every load is issued (at a clamped index,
                // inside the buffer) before the first is used
                // (passes of 4 chunks per thread: 2 for 256 threads, 1 for 512)
                for (uint32_t k0 = 0; k0 < kWinChunks; k0 += 4 * blockDim.x) {
                    u32x4 gvv[4];
                    uint32_t gav[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int64_t c = wc0 + k0 + threadIdx.x + i * blockDim.x - vbase;
                        gvv[i] = gv[c < 0 ? 0 : (c < nvch ? c : nvch - 1)];
                        gav[i] = ga[c < 0 ? 0 : (c < nach ? c : nach - 1)];
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const uint32_t k = k0 + threadIdx.x + i * blockDim.x;
                        const int64_t c = wc0 + k - vbase;
                        sv[k] = (c >= 0 && c < nvch) ? gvv[i] : u32x4{0u, 0u, 0u, 0u};
                        sa[k] = (uint16_t)((c >= 0 && c < nach) ? gav[i] : 0u);
                    }
                }
                // the group's positions that overlap the window, listed once
                if (threadIdx.x == 0) {
                    s_next[0] = 0;
                    s_next[1] = 0;
                }
                __syncthreads();
                for (uint32_t t = threadIdx.x; t < g1 - g0; t += blockDim.x) {
                    const HostPos &P = sp[g0 + t];
                    if (P.c_hi > wc0 && P.c_lo < wc1) s_list[atomicAdd(&s_next[1], 1u)] = (uint16_t)(g0 + t);
                }
                __syncthreads();
                const uint32_t nlist = s_next[1];
                // listed positions taken one at a time by whichever wave is
                // free, so that a few long segments do not hold up the others
                for (;;) {
                    uint32_t q = 0;
                    if (lane_id() == 0) q = atomicAdd(&s_next[0], 1u);
                    q = ufl32(__shfl(q, 0));
                    if (q >= nlist) break;
                    const HostPos P = sp[s_list[q]];
                    lds_segment<U>(P, wc0, wc1, sv, sa, acc);
                    if (a.out) flush_wave(acc, a.out, P.rec);
                }
                __syncthreads();
            }
            g0 = g1;
        }
    }
}

// A check-only batch worked as segments with its host-source positions left
// to LDS: blocks of even rank on their XCD start with the scan kernel's tiles,
// blocks of odd rank with the host-source tasks, and each turns to the other
// queue when its own is used up, so that the HBM-bound device-source work and
// the LDS-bound host-source work run side by side to the end.
template <int U, bool NT>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(3))) k_batched_lds(BatchArgs a)
{
    __shared__ u32x4 sv[kWinChunks];
    __shared__ uint16_t sa[kWinChunks];
    __shared__ HostPos sp[kTaskPos];
    __shared__ uint64_t s_task;
    __shared__ uint32_t s_next[2];
    __shared__ uint16_t s_list[kTaskPos];
    if (((blockIdx.x / kXcds) & 1u) != 0) {
        host_loop<4>(a, a.lds_meta, 2, sv, sa, sp, &s_task, s_next, s_list);
        __syncthreads();
        batched_loop<U, NT, false, false, 1>(a);
    } else {
        batched_loop<U, NT, false, false, 1>(a);
        __syncthreads();
        host_loop<4>(a, a.lds_meta, 2, sv, sa, sp, &s_task, s_next, s_list);
    }
}

// ---------------------------------------------------------------------------
// k_plain: one record per launch, waves split its units evenly
// ---------------------------------------------------------------------------
template <int U, bool NT, bool PROP>
__global__ void __launch_bounds__(512) k_plain(BatchArgs a, uint64_t t, uint64_t units)
{
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t w = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    uint64_t span = (units + waves - 1) / waves;
    span = (span + 63) & ~63ull;
    const uint64_t k0 = w * span;
    if (k0 >= units) return;
    const uint64_t k1 = (k0 + span < units) ? k0 + span : units;
    const DV d = load_desc_uniform(a.desc, t);
    Acc acc;
    acc_reset(acc);
    run_uniform<U, NT, PROP>(d, a.st->region, k0, k1, acc);
    if (a.out) flush_wave(acc, a.out, t);
}

// ---------------------------------------------------------------------------
// k_small: a small batch in one launch
// ---------------------------------------------------------------------------

// A batch of few records in one launch, up to `bpr` blocks per record.  The
// blocks a record uses follow from its byte count alone (at most one per
// kSmallUnits units), so that every block of the record agrees on them and
// the unused ones leave after one load.  Block b of record t: waves 0 and 1
// look up the record's source and destination pointers side by side, one
// lane classifies it; the record's units are
// split evenly over its blocks, and a block's share over its waves (the
// wave-uniform loop).  A record of one block gets its whole verdict from that
// block.  Otherwise a block that finds something merges it into the record's
// accumulator with atomics; the last of the record's blocks to finish (the
// accumulator's counter) writes the whole verdict -- the range-derived fields
// of its own classification and the findings of all blocks -- and puts the
// accumulator back to its starting state {NONE, 0, 0, 0}, so that the next
// call needs no clearing.

template <int U, bool NT, bool PROP>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(PROP ? 1 : 3)))
k_small(BatchArgs a, SmallAcc *acc, uint32_t bpr)
{
    __shared__ Desc sd;
    __shared__ cg_verdict sv;
    __shared__ uint64_t su;
    __shared__ uint64_t wfirst[8], wund[8];
    __shared__ uint32_t wfl[8];
    __shared__ int64_t sj[2];   // the source's and the destination's allocation (-1: none)
    const uint32_t lane = lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint64_t t = blockIdx.x / bpr;
    const uint32_t b = blockIdx.x % bpr;
    const cg_transfer r = a.recs[t];
    // units never exceed n / 16 + 2 (one per 16-byte chunk the bytes touch)
    const uint64_t most = r.kind <= CG_D2D && r.n ? r.n / 16 + 2 : 1;
    const uint64_t want = (most + kSmallUnits - 1) / kSmallUnits;
    const uint32_t nb = want < bpr ? (uint32_t)want : bpr;   // blocks of this record, at least 1
    if (b >= nb) return;
    const DevState *st = a.st;
    if (wid < 2) {
        // the source's lookup on wave 0, the destination's on wave 1, side by side
        const bool src = wid == 0;
        int64_t j = -1;
        if (src ? dev_src(r) : dev_dst(r)) j = table_lookup_wave(st->table, src ? r.src : r.dst);
        if (lane == 0) sj[wid] = j;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Desc ds;
        cg_verdict v;
        su = classify_rec(r, a.mode, *st, sj[0], sj[1], ds, v);
        sd = ds;
        sv = v;
    }
    __syncthreads();
    const uint64_t units = su;
    // this block's units, then this wave's, in whole iterations of 64 units
    const uint64_t per_b = ((units + nb - 1) / nb + 63) & ~63ull;
    const uint64_t b0 = (uint64_t)b * per_b < units ? (uint64_t)b * per_b : units;
    const uint64_t b1 = b0 + per_b < units ? b0 + per_b : units;
    const uint64_t per_w = ((b1 - b0 + nw - 1) / nw + 63) & ~63ull;
    const uint64_t k0 = b0 + wid * per_w < b1 ? b0 + wid * per_w : b1;
    const uint64_t k1 = k0 + per_w < b1 ? k0 + per_w : b1;
    Acc ac;
    acc_reset(ac);
    if (k1 > k0) {
        const DV d = load_desc_uniform(&sd, 0);
        run_uniform<U, NT, PROP>(d, st->region, k0, k1, ac);
    }
    if (!a.out) return;   // propagation only: no verdict (uniform over the grid)
    uint64_t f = NONE, u = 0;
    uint32_t fl = 0;
    if (__ballot(ac.flags != 0u)) {
        f = wave_min64(ac.first);
        u = wave_sum64(ac.undef);
        fl = wave_or32(ac.flags);
    }
    if (lane == 0) {
        wfirst[wid] = f;
        wund[wid] = u;
        wfl[wid] = fl;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (uint32_t w = 1; w < nw; ++w) {
        f = wfirst[w] < f ? wfirst[w] : f;
        u += wund[w];
        fl |= wfl[w];
    }
    cg_verdict v = sv;
    if (nb > 1) {
        SmallAcc &x = acc[t];
        if (fl) {
            atomicOr(&x.flags, fl);
            if (f != NONE) atomicMin((unsigned long long *)&x.first, (unsigned long long)f);
            if (u) atomicAdd((unsigned long long *)&x.undef, (unsigned long long)u);
        }
        __threadfence();
        if (atomicAdd(&x.done, 1u) != nb - 1) return;
        __threadfence();
        // the last block of the record: every other block's findings are in
        fl |= __hip_atomic_load(&x.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t af = __hip_atomic_load(&x.first, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        u = __hip_atomic_load(&x.undef, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        f = af < f ? af : f;
        __hip_atomic_store(&x.flags, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&x.first, NONE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&x.undef, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&x.done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    v.flags |= fl;
    v.first_bad = f < v.first_bad ? f : v.first_bad;
    v.undef_bytes = u;
    a.out[t] = v;
}

// accumulators to their starting state
__global__ void __launch_bounds__(256) k_small_reset(SmallAcc *acc, uint64_t n)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) acc[i] = SmallAcc{NONE, 0, 0, 0};
}

// ---------------------------------------------------------------------------
// shadow fills and bandwidth probes
// ---------------------------------------------------------------------------
// A small upload from coherent host memory: one block copies n 8-byte words
// with system-scope loads (they observe the host's latest writes); for the
// few kilobytes of a table delta, a context state or fill ranges, a launch
// waits less than a DMA copy.
__global__ void __launch_bounds__(256) k_upload(const uint64_t *src, uint64_t *dst, uint64_t n)
{
    for (uint64_t i = threadIdx.x; i < n; i += 256)
        dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void __launch_bounds__(256) k_fill(const FillRange *ranges, uint64_t k)
{
    for (uint64_t i = blockIdx.x; i < k; i += gridDim.x) {
        const FillRange fr = ranges[i];
        uint8_t *p = reinterpret_cast<uint8_t *>(fr.ptr);
        const uint8_t v = (uint8_t)fr.val;
        const uint64_t len = fr.len;
        uint64_t head = (16u - (fr.ptr & 15u)) & 15u;
        head = head < len ? head : len;
        if (threadIdx.x < head) p[threadIdx.x] = v;
        const uint64_t body = (len - head) & ~15ull;
        const uint32_t w = 0x01010101u * v;
        const u32x4 vv{w, w, w, w};
        for (uint64_t o = head + 16ull * threadIdx.x; o < head + body; o += 16ull * blockDim.x)
            *reinterpret_cast<u32x4 *>(p + o) = vv;
        const uint64_t tail = len - head - body;
        if (threadIdx.x < tail) p[head + body + threadIdx.x] = v;
    }
}

__global__ void __launch_bounds__(256) k_probe_read(const u32x4 *p, uint64_t n16, uint64_t *sink)
{
    u32x4 acc{0u, 0u, 0u, 0u};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const u32x4 a = __builtin_nontemporal_load(p + i);
        const u32x4 b = __builtin_nontemporal_load(p + i + stride);
        const u32x4 c = __builtin_nontemporal_load(p + i + 2 * stride);
        const u32x4 d = __builtin_nontemporal_load(p + i + 3 * stride);
        acc ^= a ^ b ^ c ^ d;
    }
    for (; i < n16; i += stride) acc ^= __builtin_nontemporal_load(p + i);
    const uint32_t x = acc.x ^ acc.y ^ acc.z ^ acc.w;
    if (x == 0x9E3779B9u) atomicXor((unsigned long long *)sink, (unsigned long long)x);
}

// L2-resident read ceiling: block b reads slice b mod 8 (the XCD it runs on)
// `passes` times with the same cached 16-byte loads as the scan kernel, each
// block from its own starting offset, so that the blocks sharing a CU do not
// hit in its L1 on each other's lines; a slice that fits its XCD's L2 is then
// served from L2 to the L1s.
__global__ void __launch_bounds__(256) k_probe_l2(const u32x4 *p, uint64_t slice16, uint32_t passes, uint64_t *sink)
{
    const u32x4 *q = p + (uint64_t)(blockIdx.x % kXcds) * slice16;
    const uint64_t step = 4ull * blockDim.x;
    const uint64_t groups = slice16 / step;   // whole groups of 4 loads per thread
    uint64_t g = ((uint64_t)(blockIdx.x / kXcds) * 37u) % (groups ? groups : 1);
    u32x4 acc{0u, 0u, 0u, 0u};
    for (uint64_t k = 0; k < groups * passes; ++k) {
        const u32x4 *r = q + g * step + threadIdx.x;
        const u32x4 a = r[0], b = r[blockDim.x], c = r[2 * blockDim.x], d = r[3 * blockDim.x];
        acc ^= a ^ b ^ c ^ d;
        g = g + 1 == groups ? 0 : g + 1;
    }
    const uint32_t x = acc.x ^ acc.y ^ acc.z ^ acc.w;
    if (x == 0x9E3779B9u) atomicXor((unsigned long long *)sink, (unsigned long long)x);
}

__global__ void __launch_bounds__(256) k_probe_copy(u32x4 *d, const u32x4 *p, uint64_t n16)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        d[i] = __builtin_nontemporal_load(p + i);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_classify(const BatchArgs &a, hipStream_t s)
{
    const uint64_t blocks = (a.count + kClassifyBlock - 1) / kClassifyBlock;
    hipLaunchKernelGGL(k_classify, dim3((uint32_t)blocks), dim3(kClassifyBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_reweigh(const BatchArgs &a, hipStream_t s)
{
    const uint64_t blocks = (a.count + kClassifyBlock - 1) / kClassifyBlock;
    hipLaunchKernelGGL(k_reweigh, dim3((uint32_t)blocks), dim3(kClassifyBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_classify_2d(const BatchArgs &a, const cg_transfer2d *recs2d, Pitch *pitch, hipStream_t s)
{
    const uint64_t blocks = (a.count + kClassifyBlock - 1) / kClassifyBlock;
    hipLaunchKernelGGL(k_classify_2d, dim3((uint32_t)blocks), dim3(kClassifyBlock), 0, s, a, recs2d, pitch);
    return hipGetLastError();
}

hipError_t launch_scan_sums(const BatchArgs &a, uint32_t tile_units, uint32_t waves, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, a, tile_units, waves);
    return hipGetLastError();
}

hipError_t launch_prefix_tiles(const BatchArgs &a, hipStream_t s)
{
    const uint64_t blocks = (a.count + 255) / 256;
    hipLaunchKernelGGL(k_prefix_tiles, dim3((uint32_t)blocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_tile_starts, dim3(1024), dim3(256), 0, s, a);
    return hipGetLastError();
}

// the host-source tasks alone (the LDS path run after the scan kernel)
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_host_lds(BatchArgs a)
{
    __shared__ u32x4 sv[kWinChunks];
    __shared__ uint16_t sa[kWinChunks];
    __shared__ HostPos sp[kTaskPos];
    __shared__ uint64_t s_task;
    __shared__ uint32_t s_next[2];
    __shared__ uint16_t s_list[kTaskPos];
    host_loop<4>(a, a.lds_meta, 0, sv, sa, sp, &s_task, s_next, s_list);
}

template <int U, bool NT>
static void launch_batched_t(const BatchArgs &a, const LaunchShape &sh, hipStream_t s)
{
    if (a.pitch && (a.mode & CG_PROPAGATE)) {
        hipLaunchKernelGGL((k_batched_2d<U, NT, true>), dim3(sh.grid), dim3(sh.block), 0, s, a);
    } else if (a.pitch) {
        hipLaunchKernelGGL((k_batched_2d<U, NT, false>), dim3(sh.grid), dim3(sh.block), 0, s, a);
    } else if (a.lds_meta && sh.lds_after) {
        BatchArgs d = a;
        d.lds_meta = nullptr;
        hipLaunchKernelGGL((k_batched<U, NT, false>), dim3(sh.grid), dim3(sh.block), 0, s, d);
        hipLaunchKernelGGL(k_host_lds, dim3(sh.cus * 3), dim3(256), 0, s, a);
    } else if (a.lds_meta)
        hipLaunchKernelGGL((k_batched_lds<U, NT>), dim3(sh.grid), dim3(sh.block), 0, s, a);
    else if (a.mode & CG_PROPAGATE)
        hipLaunchKernelGGL((k_batched<U, NT, true>), dim3(sh.grid), dim3(sh.block), 0, s, a);
    else
        hipLaunchKernelGGL((k_batched<U, NT, false>), dim3(sh.grid), dim3(sh.block), 0, s, a);
}

template <int U, bool NT>
static void launch_plain_t(const BatchArgs &a, uint64_t t, uint64_t units, uint32_t grid, uint32_t block,
                           hipStream_t s)
{
    if (a.mode & CG_PROPAGATE)
        hipLaunchKernelGGL((k_plain<U, NT, true>), dim3(grid), dim3(block), 0, s, a, t, units);
    else
        hipLaunchKernelGGL((k_plain<U, NT, false>), dim3(grid), dim3(block), 0, s, a, t, units);
}

#define XC_DISPATCH(FN, ...)                                                   \
    do {                                                                       \
        const bool nt_ = sh.nontemporal != 0;                                  \
        switch (sh.unroll) {                                                   \
        case 1: nt_ ? FN<1, true>(__VA_ARGS__) : FN<1, false>(__VA_ARGS__); break; \
        case 2: nt_ ? FN<2, true>(__VA_ARGS__) : FN<2, false>(__VA_ARGS__); break; \
        case 8: nt_ ? FN<8, true>(__VA_ARGS__) : FN<8, false>(__VA_ARGS__); break; \
        default: nt_ ? FN<4, true>(__VA_ARGS__) : FN<4, false>(__VA_ARGS__); break; \
        }                                                                      \
    } while (0)

hipError_t launch_batched(const BatchArgs &a, const LaunchShape &sh, hipStream_t s)
{
    if (a.lds_meta && (a.mode & CG_PROPAGATE)) return hipErrorInvalidValue;   // check-only
    XC_DISPATCH(launch_batched_t, a, sh, s);
    return hipGetLastError();
}

template <int U, bool NT>
static void launch_small_t(const BatchArgs &a, SmallAcc *acc, uint32_t bpr, uint32_t block, hipStream_t s)
{
    const dim3 grid((uint32_t)(a.count * bpr));
    if (a.mode & CG_PROPAGATE)
        hipLaunchKernelGGL((k_small<U, NT, true>), grid, dim3(block), 0, s, a, acc, bpr);
    else
        hipLaunchKernelGGL((k_small<U, NT, false>), grid, dim3(block), 0, s, a, acc, bpr);
}

hipError_t launch_small(const BatchArgs &a, SmallAcc *acc, uint32_t bpr, const LaunchShape &sh, hipStream_t s)
{
    if (a.count == 0 || bpr == 0 || a.count * bpr > 0x7FFFFFFFull || sh.block > 512 || sh.block % 64)
        return hipErrorInvalidValue;
    XC_DISPATCH(launch_small_t, a, acc, bpr, sh.block, s);
    return hipGetLastError();
}

hipError_t launch_small_reset(SmallAcc *acc, uint64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_small_reset, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, acc, n);
    return hipGetLastError();
}

hipError_t launch_plain(const BatchArgs &a, uint64_t rec, uint64_t units, const LaunchShape &sh, hipStream_t s)
{
    const uint64_t per_block = (uint64_t)(sh.block / 64) * 64u * sh.unroll * 4u;
    uint64_t grid = (units + per_block - 1) / per_block;
    if (grid > sh.grid) grid = sh.grid;
    if (grid == 0) grid = 1;
    XC_DISPATCH(launch_plain_t, a, rec, units, (uint32_t)grid, sh.block, s);
    return hipGetLastError();
}

hipError_t launch_pointers(const DevState *st, const uint64_t *ptrs, uint64_t count, cg_ptr_check *out, hipStream_t s)
{
    const uint64_t blocks = (count + kClassifyBlock - 1) / kClassifyBlock;
    hipLaunchKernelGGL(k_pointers, dim3((uint32_t)blocks), dim3(kClassifyBlock), 0, s, st, ptrs, count, out);
    return hipGetLastError();
}

hipError_t launch_upload(const void *src, void *dst, uint64_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, s, static_cast<const uint64_t *>(src),
                       static_cast<uint64_t *>(dst), bytes / 8);
    return hipGetLastError();
}

hipError_t launch_fill(const FillRange *ranges_dev, uint64_t k, hipStream_t s)
{
    if (k == 0) return hipSuccess;
    const uint32_t grid = (uint32_t)(k < 65536 ? k : 65536);
    hipLaunchKernelGGL(k_fill, dim3(grid), dim3(256), 0, s, ranges_dev, k);
    return hipGetLastError();
}

hipError_t launch_probe_read(const void *p, uint64_t bytes, uint64_t *sink, hipStream_t s)
{
    hipLaunchKernelGGL(k_probe_read, dim3(8192), dim3(256), 0, s, reinterpret_cast<const u32x4 *>(p), bytes / 16,
                       sink);
    return hipGetLastError();
}

hipError_t launch_probe_l2(const void *p, uint64_t slice_bytes, uint32_t passes, uint32_t blocks, uint64_t *sink,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_probe_l2, dim3(blocks), dim3(256), 0, s, reinterpret_cast<const u32x4 *>(p), slice_bytes / 16,
                       passes, sink);
    return hipGetLastError();
}

hipError_t launch_probe_copy(void *d, const void *p, uint64_t bytes, hipStream_t s)
{
    hipLaunchKernelGGL(k_probe_copy, dim3(8192), dim3(256), 0, s, reinterpret_cast<u32x4 *>(d),
                       reinterpret_cast<const u32x4 *>(p), bytes / 16);
    return hipGetLastError();
}

}  // namespace xc
