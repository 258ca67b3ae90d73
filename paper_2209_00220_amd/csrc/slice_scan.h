// Scan of the slice layouts (PP-VBS, ByteSlice): one wave per 2048-row tile.
//
// Tile layout of a tile-interleaved slice (BS_1 of both layouts): lane L of the
// wave owns the 32 consecutive rows 32L .. 32L+31 of the tile, so its 32 result
// bits are exactly dword L of the tile's 64 result dwords.  Its bytes are eight
// dwords; dword i holds rows 8q + i (q = 0..3) in byte q, dwords 0-3 at tile
// offset 16L and dwords 4-7 at 1024 + 16L, so each 16-byte load instruction of
// the wave reads 1 KB contiguously.  ByteSlice's later slices hold the same
// eight dwords per lane contiguously at 32L: only lanes with pending rows read
// them, and a lane's 32 bytes then sit in one cache line.
//
// Byte compares are four at a time inside a dword (SIMD within a register):
// the high bit of every byte lane carries the outcome, and shifting dword i
// right by 7 - i drops byte q's outcome onto bit 8q + i, the row's bit.  Each
// lane thus builds its rows' outcome dword directly; no cross-lane transposes.
//
// The comparison of a row against a literal goes byte by byte (Sec. 3.3,
// Algorithm 3 generalised to every operator): a differing byte decides the row;
// a row still equal after byte j is pending, except that at j < l a row without
// a byte j+1 is a proper prefix of the literal and so below it (the literal's
// remaining bytes are not all zero), and at j = l a row with a byte l+1 is above
// the literal and one without it equal.  Later bytes are read only for pending
// rows: the early stop of Algorithm 3 (Lemma 1) at row granularity.
//
// PP-VBS later levels: a pending row's byte j sits in BS_j at the tile's
// directory entry plus the M_j bits before the row (a wave prefix of the lanes'
// M_j dword popcounts, then the lane's own).  While every lane has at most
// `gather` (<= 4) pending rows, each lane gathers its rows' bytes straight from
// HBM; otherwise the tile copies its run of BS_j into LDS with one coalesced read
// and each lane reads its rows' bytes from there.
//
// Level 2's gathers are issued right after the tile's byte-1 pass and used one
// tile later: the wave runs the next tile's byte-1 pass while they are in
// flight, so a gather's latency overlaps useful work instead of stalling the
// wave (vector memory counters retire in order, so waiting for a gather also
// waits for every load issued before it -- the next tiles' loads are issued
// after it).  Deeper levels are rare on skewed data and run at once.
#pragma once

#include "device_common.h"

namespace bst {
namespace dev {

constexpr int kGatherSlots = 4;                 // pending rows per lane gathered directly
constexpr uint32_t kOutOfRange = 0x40000000u;   // a buffer offset past any record: the load reads nothing

// ------------------------------------------------------------ four-byte compares
constexpr uint32_t kHigh = 0x80808080u, kLow7 = 0x7f7f7f7fu;

// One literal byte broadcast to the four byte lanes of a dword.
struct ByteLit {
    uint32_t c;    // c * 0x01010101
    uint32_t cl;   // its low seven bits per byte
};

__device__ __forceinline__ ByteLit byte_lit(uint32_t b) {
    const uint32_t c = (b & 0xffu) * 0x01010101u;
    return ByteLit{c, c & kLow7};
}

// High bit of each byte: that byte of x >= the literal byte (unsigned).  xh = x | kHigh.
// (x | 0x80) - (c & 0x7f) lies in [1, 255] per byte, so no borrow crosses bytes and its
// high bit compares the low seven bits; where the top bits differ, x's top bit decides.
__device__ __forceinline__ uint32_t swar_ge(uint32_t x, uint32_t xh, ByteLit L) {
    const uint32_t t = xh - L.cl;
    const uint32_t d = x ^ L.c;
    return (d & x) | (~d & t);
}

// High bit of each byte: that byte of x differs from the literal byte.
// (d & 0x7f) + 0x7f sets the high bit exactly when the low seven bits of d are not 0.
__device__ __forceinline__ uint32_t swar_ne(uint32_t x, ByteLit L) {
    const uint32_t d = x ^ L.c;
    return ((d & kLow7) + kLow7) | d;
}

// Rows 8q + I of a lane take the high bits of the four bytes of v (dword I).
template <int I>
__device__ __forceinline__ uint32_t collect(uint32_t acc, uint32_t v) {
    return acc | ((v >> (7 - I)) & (0x01010101u << I));
}

// Per-byte outcome masks of a lane's 32 rows (eight dwords of one slice):
// ge_* = byte >= literal byte, ne_* = byte != literal byte, each one bit per row.
template <bool GE_LO, bool NE_LO, bool GE_HI, bool NE_HI>
__device__ __forceinline__ void swar_lane(const uint32_t (&x)[8], ByteLit lo, ByteLit hi, uint32_t& ge_lo,
                                          uint32_t& ne_lo, uint32_t& ge_hi, uint32_t& ne_hi) {
    ge_lo = ne_lo = ge_hi = ne_hi = 0;
    Unroll<0, 8>::run([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const uint32_t v = x[i], vh = v | kHigh;
        if (GE_LO) ge_lo = collect<i>(ge_lo, swar_ge(v, vh, lo));
        if (NE_LO) ne_lo = collect<i>(ne_lo, swar_ne(v, lo));
        if (GE_HI) ge_hi = collect<i>(ge_hi, swar_ge(v, vh, hi));
        if (NE_HI) ne_hi = collect<i>(ne_hi, swar_ne(v, hi));
    });
}

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ uint32_t wave_total(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_sum(v), 63);
}

__device__ __forceinline__ bool wave_any(bool p) { return ballot(p) != 0; }

// Number of 64-row groups (lane pairs) in which v is non-zero in either lane.
__device__ __forceinline__ uint32_t groups_with(uint32_t v) {
    const uint64_t b = ballot(v != 0);
    return (uint32_t)__builtin_popcountll((b | (b >> 1)) & 0x5555555555555555ull);
}

// 128-byte lines holding the M_j words of the groups in which v is non-zero in
// either lane (a tile's 32 words fill two lines: lanes 0-31 and 32-63).
__device__ __forceinline__ uint32_t mask_lines(uint32_t v) {
    const uint64_t b = ballot(v != 0);
    return ((uint32_t)b != 0u ? 1u : 0u) + ((uint32_t)(b >> 32) != 0u ? 1u : 0u);
}

// 128-byte lines of a slice that the lanes' byte spans [first, first + len)
// touch, each line once: spans of increasing lanes are disjoint and increasing,
// so a line two spans share is the last of one and the first of the next
// non-empty one.  Uniform; for the instrumented build only.
__device__ inline uint32_t span_lines(uint64_t first, uint32_t len) {
    uint32_t lines = 0;
    uint64_t prev = ~0ull;
    for (int i = 0; i < 64; ++i) {
        const uint32_t l = (uint32_t)__builtin_amdgcn_readlane((int)len, i);
        if (!l) continue;
        const uint64_t f = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(first >> 32), i) << 32) |
                           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)first, i);
        const uint64_t a = f >> 7, b = (f + l - 1) >> 7;
        lines += (uint32_t)(b - a + 1) - (a == prev ? 1u : 0u);
        prev = b;
    }
    return lines;
}

// True in both lanes of a lane pair when v is non-zero in either.
__device__ __forceinline__ bool pair_any(uint32_t v, uint32_t lane) {
    const uint64_t b = ballot(v != 0);
    return ((b >> (lane & ~1u)) & 3u) != 0;
}

// ------------------------------------------------------------ level rules
// The length rule of a level on lane-held row masks: rows still equal to the
// literal (plo / phi) either have a next byte (m) or end.  Returns the rows
// newly found in the tracked relation; klo / khi are all ones while the level is
// shorter than the lower / upper literal.
template <int MODE>
__device__ __forceinline__ uint32_t length_rule(uint32_t& plo, uint32_t& phi, uint32_t m, uint32_t klo, uint32_t khi) {
    uint32_t hit;
    if (MODE == kModeLT || MODE == kModeBetween) hit = plo & ~m & klo;   // a proper prefix: below
    else if (MODE == kModeGT) hit = plo & m & ~klo;                     // equal, then more bytes: above
    else hit = plo & ~m & ~klo;                                         // equal over the whole literal
    plo &= m & klo;
    if (MODE == kModeBetween) {
        hit |= phi & m & ~khi;   // equal to the upper literal, then more bytes: above it
        phi &= m & khi;
    }
    return hit;
}

// Outcome of a level's byte for the pending rows: rlo = rows whose byte is on
// the tracked side of the lower literal's byte ('<' and BETWEEN: below; '>':
// above), elo = rows whose byte equals it; rhi / ehi the same against the
// upper literal (BETWEEN: above / equal).  Then the length rule with m = rows
// that have a next byte.  `out` holds rows in the relation ('<', '>', '='), or
// rows still in range (BETWEEN).
template <int MODE>
__device__ __forceinline__ void apply_level(uint32_t& out, uint32_t& plo, uint32_t& phi, uint32_t rlo, uint32_t elo,
                                            uint32_t rhi, uint32_t ehi, uint32_t m, uint32_t klo, uint32_t khi) {
    uint32_t hit = MODE == kModeEQ ? 0u : (plo & rlo);
    plo &= elo;
    if (MODE == kModeBetween) {
        hit |= phi & rhi;
        phi &= ehi;
    }
    hit |= length_rule<MODE>(plo, phi, m, klo, khi);
    out = MODE == kModeBetween ? (out & ~hit) : (out | hit);
}

// Outcome masks of one gathered row (bit `beta`, byte b) at a level.
template <int MODE>
__device__ __forceinline__ void row_masks(uint32_t b, uint32_t beta, uint32_t cl, uint32_t ch, uint32_t& rlo,
                                          uint32_t& elo, uint32_t& rhi, uint32_t& ehi) {
    if (MODE == kModeLT || MODE == kModeBetween) rlo |= b < cl ? beta : 0u;
    if (MODE == kModeGT) rlo |= b > cl ? beta : 0u;
    elo |= b == cl ? beta : 0u;
    if (MODE == kModeBetween) {
        rhi |= b > ch ? beta : 0u;
        ehi |= b == ch ? beta : 0u;
    }
}

// Outcome masks of a whole lane from its 32 bytes of a dense slice.
template <int MODE>
__device__ __forceinline__ void lane_masks(const uint32_t (&x)[8], uint32_t cl, uint32_t ch, uint32_t& rlo,
                                           uint32_t& elo, uint32_t& rhi, uint32_t& ehi) {
    uint32_t gel, nel, geh, neh;
    swar_lane<MODE != kModeEQ, true, MODE == kModeBetween, MODE == kModeBetween>(x, byte_lit(cl), byte_lit(ch), gel,
                                                                                    nel, geh, neh);
    rlo = MODE == kModeGT ? (gel & nel) : ~gel;
    elo = ~nel;
    rhi = geh & neh;
    ehi = ~neh;
}

// ------------------------------------------------------------ tiles
// Loads of one tile (zeros, and no memory read, when `valid` is false).
struct TileData {
    uint32_t x[8];   // the lane's 32 bytes of BS_1
    uint32_t m2;     // PP-VBS: the lane's dword of M_2 (when the literal needs it)
    uint32_t in;     // the lane's dword of the incoming mask (all ones without one)
    uint32_t dir2;   // PP-VBS: BS_2 position of the tile's first byte 2 (all lanes)
};

// The lane's 32 bytes of a tile-interleaved slice (two 16-byte chunks `gap`
// bytes apart: 1024 for BS_1, 16 for ByteSlice's later slices), or zeros when
// `off` is out of range.
template <uint32_t GAP = 1024>
__device__ __forceinline__ void load_lane_bytes(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t (&x)[8]) {
    const uint4 a = buffer_load16(r, off), b = buffer_load16(r, off + GAP);
    x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
    x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
}

// Lane's dword of the tile's M_j words (0 when the column has no byte j, when
// `valid` is false or when off_lane is kOutOfRange).
__device__ __forceinline__ uint32_t load_mask_dword(const DevCol& c, uint32_t j, uint64_t t, uint32_t off_lane,
                                                    bool valid = true) {
    const bool has = valid && j <= c.K;
    const void* base = has ? (const void*)(c.m[j] + t * 32) : (const void*)c.bs[1];
    return buffer_load4(buffer_rsrc(base, has ? 256u : 0u), off_lane);
}

template <bool NEED_M2, bool NEED_DIR, bool HAS_IN>
__device__ __forceinline__ TileData load_tile(const DevCol& c, const uint64_t* __restrict__ in_mask, uint64_t t,
                                              uint32_t lane, bool valid) {
    TileData d;
    const auto r1 = buffer_rsrc(c.bs[1] + (valid ? t * kTileRows : 0), valid ? kTileRows : 0u);
    load_lane_bytes(r1, lane * 16, d.x);
    d.m2 = NEED_M2 ? load_mask_dword(c, 2, t, lane * 4, valid) : 0u;
    d.dir2 = 0;
    if (NEED_DIR) {
        const bool has = valid && c.K >= 2;
        const void* base = has ? (const void*)(c.dir[2] + ((t * kTileRows) >> c.dir_shift)) : (const void*)c.bs[1];
        d.dir2 = buffer_load4(buffer_rsrc(base, has ? 4u : 0u), 0);
    }
    d.in = ~0u;
    if (HAS_IN) {
        // the mask has ceil(n/64) words; the last tile may hold fewer than 32
        const uint64_t nd = ((c.n + 63) >> 6) * 2, d0 = t * 64;
        const uint32_t avail = (valid && d0 < nd) ? (uint32_t)(nd - d0 < 64 ? nd - d0 : 64) * 4u : 0u;
        const void* base = avail ? (const void*)(reinterpret_cast<const uint32_t*>(in_mask) + d0) : (const void*)in_mask;
        d.in = buffer_load4(buffer_rsrc(base, avail), lane * 4);
    }
    return d;
}

// A tile between its byte-1 pass and the settling of its later bytes.
struct TileState {
    uint32_t out, plo, phi, act;
    uint32_t pend;                // PP-VBS: the rows whose bytes are in flight (the lowest
                                  // kGatherSlots set bits of the lane, in ascending order)
    uint32_t b[kGatherSlots];     // their bytes
    uint32_t d[8];                // ByteSlice: the lane's 32 bytes of BS_2 (lanes with pending rows)
    uint32_t inflight;            // uniform: level-2 bytes are in flight (PP-VBS: the gather slots used)
};

// Bytes an exhaustive (no early stop) scan of this tile would touch.
template <bool DENSE>
__device__ uint64_t full_read_bytes(const DevCol& c, const ScanLit& lit, uint64_t t, bool has_in) {
    const uint32_t l = lit.llo > lit.lhi ? lit.llo : lit.lhi;
    uint64_t bytes = kTileRows + 256 + (has_in ? 256 : 0);
    for (uint32_t j = 2; j <= c.K && j <= l + 1; ++j) {
        if (DENSE) {
            if (j <= l) bytes += kTileRows;
        } else {
            bytes += 256;
            if (j <= l)
                for (uint32_t k = 0; k < 32; ++k) bytes += __builtin_popcountll(c.m[j][t * 32 + k]);
        }
    }
    return bytes;
}

constexpr uint32_t kStageBytes = 2080;   // 130 chunks of 16 bytes: a 2048-byte run plus alignment
constexpr uint32_t kWaveLds = kStageBytes;

// Copy bytes [start, start+len) of a slice into this wave's LDS buffer with
// 16-byte loads from the aligned-down start; returns start's offset in the buffer.
__device__ __forceinline__ uint32_t stage_run(const uint8_t* __restrict__ src, uint64_t start, uint32_t len,
                                              uint8_t* buf, uint32_t lane) {
    const uint64_t a = start & ~15ull;
    // bytes from the aligned start, rounded up to whole 16-byte chunks: the range
    // check drops a partly covered chunk, and slices carry 64 bytes of slack past
    // their last byte, so the rounded range stays inside the allocation
    const uint32_t span = (uint32_t)(start + len - a + 15) & ~15u;
    const auto r = buffer_rsrc(src + a, span);
    // 130 chunks: lanes 0..63 and 64..127 always, 128..129 by two lanes
    const uint4 c0 = buffer_load16(r, 16 * lane);
    const uint4 c1 = buffer_load16(r, 16 * (lane + 64));
    uint4 c2 = make_uint4(0, 0, 0, 0);
    if (lane < kStageBytes / 16 - 128) c2 = buffer_load16(r, 16 * (lane + 128));
    *reinterpret_cast<uint4*>(buf + 16 * lane) = c0;
    *reinterpret_cast<uint4*>(buf + 16 * (lane + 64)) = c1;
    if (lane < kStageBytes / 16 - 128) *reinterpret_cast<uint4*>(buf + 16 * (lane + 128)) = c2;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return (uint32_t)(start - a);
}

template <int MODE, int SHORT, bool DENSE, bool HAS_IN, bool COUNT>
struct SliceScan {
    // SHORT bit 0 (bit 1): the lower (upper) literal is one byte long; SHORT < 0:
    // the lengths are read at run time
    static constexpr bool kLoShort = SHORT >= 0 && (SHORT & 1) != 0;
    static constexpr bool kHiShort = SHORT >= 0 && (SHORT & 2) != 0;
    // rows equal to a one-byte '<' or lower-BETWEEN literal on byte 1 are never
    // below it: their equal-so-far mask is not needed
    static constexpr bool kNeedLo = !((MODE == kModeLT || MODE == kModeBetween) && kLoShort);
    // one-byte literals are settled by byte 1 and M_2
    static constexpr bool kByte1Only = MODE == kModeBetween ? (kLoShort && kHiShort) : kLoShort;
    // M_2 settles rows equal on byte 1: unused only by a one-byte '<'
    static constexpr bool kNeedM2 = !DENSE && !(MODE == kModeLT && kLoShort);
    static constexpr bool kNeedDir = !DENSE && !kByte1Only;

    __device__ static TileData load(const DevCol& c, const uint64_t* in_mask, uint64_t t, uint32_t lane, bool valid) {
        return load_tile<kNeedM2, kNeedDir, HAS_IN>(c, in_mask, t, lane, valid);
    }

    // Rows equal to the literals over bytes 1..j whose M_{j+1} bit the
    // algorithm needs (instrumented build only): none of those equal to a whole
    // '<' or lower-BETWEEN literal, which are not below it whatever follows.
    __device__ static uint32_t tied_next(const ScanLit& lit, uint32_t j, uint32_t lo_eq, uint32_t hi_eq) {
        const bool lo_done = (MODE == kModeLT || MODE == kModeBetween) && j >= lit.llo;
        return (lo_done ? 0u : lo_eq) | (MODE == kModeBetween ? hi_eq : 0u);
    }

    // Lemma-1 counters of a level's pending rows (instrumented build only);
    // first: the offset in BS_j of the lane's first byte there.
    __device__ static void count_level(Stats& st, uint32_t j, uint32_t pend, uint32_t mj, uint32_t lane,
                                       uint64_t first) {
        const bool g = pair_any(pend, lane);
        if (j == 2) st.deep_groups += groups_with(pend);
        st.rowbytes += wave_total(__builtin_popcount(pend));
        // the group's bytes of BS_j: PP-VBS the M_j word's bits, ByteSlice all 64
        const uint32_t len = g ? (DENSE ? 32u : (uint32_t)__builtin_popcount(mj)) : 0u;
        st.alg += wave_total(len);
        st.lines += span_lines(first, len);
    }

    // Byte 1 and the presence of byte 2 for tile t; then, if rows are still
    // pending, issue level 2's reads (settled by finish()).  Returns false for
    // a slot past the wave's last tile.
    __device__ static void begin(const DevCol& c, const ScanLit& lit, uint64_t t, uint32_t lane, const TileData& td,
                                 TileState& s, uint8_t* lds, Stats& st, bool live) {
        s.inflight = 0;
        if (!live) return;
        const uint32_t K = c.K;
        // rows this lane's dword may report: selected by the incoming mask and inside the column
        // (32-bit compare of uniform values: a 64-bit one needs a vector register for one side)
        const bool full = (uint32_t)t < (uint32_t)(c.n / kTileRows);
        uint32_t act = HAS_IN ? td.in : ~0u;
        if (!full) {
            const uint64_t r0 = (t * 64 + lane) * 32;
            act &= r0 + 32 <= c.n ? ~0u : (r0 < c.n ? (1u << (c.n - r0)) - 1u : 0u);
        }
        s.act = act;
        const uint32_t c1lo = lit_byte(lit.lo, 1), c1hi = lit_byte(lit.hi, 1);
        uint32_t gel, nel, geh, neh;
        swar_lane<MODE != kModeEQ, MODE != kModeLT || kNeedLo, MODE == kModeBetween, MODE == kModeBetween>(
            td.x, byte_lit(c1lo), byte_lit(c1hi), gel, nel, geh, neh);
        uint32_t out, plo = 0, phi = 0;
        if (MODE == kModeLT) out = ~gel;
        else if (MODE == kModeGT) out = gel & nel;
        else if (MODE == kModeEQ) out = 0;
        else out = gel & ~(geh & neh) & act;   // BETWEEN: byte 1 in [lo_1, hi_1]
        if (kNeedLo) plo = ~nel & act;
        if (MODE == kModeBetween) phi = ~neh & act;
        if (COUNT) {
            st.alg += kTileRows + 256 + (HAS_IN ? 256 : 0);
            st.lines += (kTileRows + 256 + (HAS_IN ? 256 : 0)) / 128;
            st.full += full_read_bytes<DENSE>(c, lit, t, HAS_IN);
            st.rowbytes += wave_total(__builtin_popcount(act));
            // M_2 words read: the groups with rows equal on byte 1 that need them
            const uint32_t tied1 = tied_next(lit, 1, plo, phi);
            if (!DENSE && K >= 2) {
                st.alg += 8ull * groups_with(tied1);
                st.lines += mask_lines(tied1);
            }
        }
        // byte 2's presence settles the rows equal on byte 1 that end there
        const uint32_t klo = SHORT < 0 ? (1 < lit.llo ? ~0u : 0u) : (kLoShort ? 0u : ~0u);
        const uint32_t khi = SHORT < 0 ? (1 < lit.lhi ? ~0u : 0u) : (kHiShort ? 0u : ~0u);
        {
            const uint32_t m2v = DENSE ? (K >= 2 ? ~0u : 0u) : td.m2;
            const uint32_t hit = length_rule<MODE>(plo, phi, m2v, klo, khi);
            out = MODE == kModeBetween ? (out & ~hit) : (out | hit);
        }
        s.out = out;
        s.plo = plo;
        s.phi = phi;
        if constexpr (kByte1Only) return;
        const uint32_t pend = plo | phi;
        if (!wave_any(pend != 0)) return;
        if constexpr (DENSE) {
            if (COUNT) count_level(st, 2, pend, td.m2, lane, t * kTileRows + lane * 32);
            // the pending lanes' 32 bytes of BS_2 (contiguous per lane), held in the
            // same registers as BS_1's
            const auto r2 = buffer_rsrc(c.bs[2] + t * kTileRows, kTileRows);
            load_lane_bytes<16>(r2, pend ? lane * 32 : kOutOfRange, s.d);
            s.inflight = 1;
        } else {
            const uint32_t incl = wave_incl_sum((uint32_t)__builtin_popcount(td.m2));
            const uint32_t runlen = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
            const uint32_t run0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)td.dir2);
            if (COUNT) count_level(st, 2, pend, td.m2, lane, (uint64_t)run0 + incl - __builtin_popcount(td.m2));
            const uint32_t cnt = (uint32_t)__builtin_popcount(pend);
            if (wave_any(cnt > lit.gather)) {
                // a lane with more pending rows than it gathers: the whole tile's
                // run of BS_2 into LDS, read row by row (settles level 2 at once)
                settle_staged(c, lit, t, 2, run0, runlen, incl - __builtin_popcount(td.m2), td.m2, lane, s, lds, st);
                settle_deeper(c, lit, t, 3, lane, s, lds, st);
                return;
            }
            const auto r2 = buffer_rsrc(c.bs[2] + run0, runlen);
            const uint32_t excl = incl - (uint32_t)__builtin_popcount(td.m2);
            // as many gather slots as the lane with the most pending rows needs
            // (most tiles have a row or two pending in all)
            uint32_t used = 1;
            Unroll<1, kGatherSlots>::run([&](auto sc) { used += wave_any(cnt > (uint32_t)decltype(sc)::value) ? 1u : 0u; });
            uint32_t rem = pend;
            Unroll<0, kGatherSlots>::run([&](auto sc) {
                constexpr int k = decltype(sc)::value;
                if ((uint32_t)k < used) {
                    const uint32_t beta = rem & (0u - rem);
                    const uint32_t off = beta ? excl + (uint32_t)__builtin_popcount(td.m2 & (beta - 1u)) : kOutOfRange;
                    s.b[k] = __builtin_amdgcn_raw_buffer_load_b8(r2, (int)off, 0, 0);
                    rem ^= beta;
                }
            });
            s.pend = pend;
            s.inflight = used;
        }
    }

    // Settle level 2 from the bytes begin() requested, then any deeper levels,
    // and store the tile's result dwords.
    __device__ static void finish(const DevCol& c, const ScanLit& lit, uint64_t* __restrict__ out, uint64_t t,
                                  uint32_t lane, TileState& s, uint8_t* lds, Stats& st, bool live) {
        if (!live) return;
        if (!kByte1Only && s.inflight) {
            const uint32_t K = c.K;
            const uint32_t cl = lit_byte(lit.lo, 2), ch = lit_byte(lit.hi, 2);
            uint32_t rlo = 0, elo = 0, rhi = 0, ehi = 0, m;
            if constexpr (DENSE) {
                lane_masks<MODE>(s.d, cl, ch, rlo, elo, rhi, ehi);
                m = K > 2 ? ~0u : 0u;
            } else {
                uint32_t rem = s.pend;
                const uint32_t used = (uint32_t)__builtin_amdgcn_readfirstlane((int)s.inflight);
                Unroll<0, kGatherSlots>::run([&](auto sc) {
                    constexpr int k = decltype(sc)::value;
                    if ((uint32_t)k < used) {
                        const uint32_t beta = rem & (0u - rem);
                        row_masks<MODE>(s.b[k], beta, cl, ch, rlo, elo, rhi, ehi);
                        rem ^= beta;
                    }
                });
                // M_3 for the rows equal over two bytes, read once they are known
                // (by the lanes holding them; few tiles have any).  A '<' literal
                // of at most two bytes never consults it: a row equal to it over
                // two bytes is not below it, with or without a third.
                const bool need_m3 = K >= 3 && (MODE != kModeLT || lit.llo > 2);
                const uint32_t tied = (s.plo & elo) | (MODE == kModeBetween ? (s.phi & ehi) : 0u);
                m = need_m3 && wave_any(tied != 0) ? load_mask_dword(c, 3, t, tied ? lane * 4 : kOutOfRange) : 0u;
            }
            if (COUNT && !DENSE && K > 2) {
                const uint32_t tied = tied_next(lit, 2, s.plo & elo, s.phi & ehi);
                st.alg += 8ull * groups_with(tied);
                st.lines += mask_lines(tied);
            }
            apply_level<MODE>(s.out, s.plo, s.phi, rlo, elo, rhi, ehi, m, 2 < lit.llo ? ~0u : 0u,
                              2 < lit.lhi ? ~0u : 0u);
            settle_deeper(c, lit, t, 3, lane, s, lds, st);
        }
        store(c, lit, out, t, lane, s);
    }

    __device__ static void store(const DevCol& c, const ScanLit& lit, uint64_t* __restrict__ out, uint64_t t,
                                 uint32_t lane, const TileState& s) {
        // negation as a xor with a mask held in a scalar register
        const uint32_t neg =
            MODE != kModeBetween ? (uint32_t)__builtin_amdgcn_readfirstlane((int)(lit.negate ? ~0u : 0u)) : 0u;
        const uint32_t v = (s.out ^ neg) & s.act;
        const uint64_t d = t * 64 + lane;
        const bool full = (uint32_t)t < (uint32_t)(c.n / kTileRows);
        if (full || d < ((c.n + 63) >> 6) * 2) store_result_dword(out, d, v);
    }

    // Level j (PP-VBS) from the tile's run of BS_j staged in LDS: each lane reads
    // its pending rows' bytes one by one.  mj: the lane's M_j dword; excl: the
    // M_j bits of the lanes before it.
    __device__ static void settle_staged(const DevCol& c, const ScanLit& lit, uint64_t t, uint32_t j, uint32_t run0,
                                         uint32_t runlen, uint32_t excl, uint32_t mj, uint32_t lane, TileState& s,
                                         uint8_t* lds, Stats& st) {
        const uint32_t K = c.K;
        const uint32_t sh = stage_run(c.bs[j], run0, runlen, lds, lane);
        const uint32_t cl = lit_byte(lit.lo, j), ch = lit_byte(lit.hi, j);
        uint32_t rlo = 0, elo = 0, rhi = 0, ehi = 0;
        uint32_t rem = s.plo | s.phi;
        while (rem) {
            const uint32_t beta = rem & (0u - rem);
            const uint32_t b = lds[sh + excl + (uint32_t)__builtin_popcount(mj & (beta - 1u))];
            row_masks<MODE>(b, beta, cl, ch, rlo, elo, rhi, ehi);
            rem ^= beta;
        }
        const uint32_t pend = s.plo | s.phi;
        const uint32_t m = j < K ? load_mask_dword(c, j + 1, t, pend ? lane * 4 : kOutOfRange) : 0u;
        if (COUNT && j < K) {
            const uint32_t tied = tied_next(lit, j, s.plo & elo, s.phi & ehi);
            st.alg += 8ull * groups_with(tied);
            st.lines += mask_lines(tied);
        }
        apply_level<MODE>(s.out, s.plo, s.phi, rlo, elo, rhi, ehi, m, j < lit.llo ? ~0u : 0u,
                          j < lit.lhi ? ~0u : 0u);
    }

    // Levels j0 .. K for rows still pending, one level at a time (rare on
    // skewed columns): PP-VBS reads the tile's M_j dwords and directory entry,
    // then gathers or stages as at level 2; ByteSlice reads the pending lanes'
    // bytes of BS_j.
    __device__ static void settle_deeper(const DevCol& c, const ScanLit& lit, uint64_t t, uint32_t j0, uint32_t lane,
                                         TileState& s, uint8_t* lds, Stats& st) {
        const uint32_t K = c.K;
        for (uint32_t j = j0; j <= K; ++j) {
            const uint32_t pend = s.plo | s.phi;
            if (!wave_any(pend != 0)) return;
            const uint32_t cl = lit_byte(lit.lo, j), ch = lit_byte(lit.hi, j);
            uint32_t rlo = 0, elo = 0, rhi = 0, ehi = 0, m;
            if constexpr (DENSE) {
                if (COUNT) count_level(st, j, pend, 0u, lane, t * kTileRows + lane * 32);
                uint32_t x[8];
                load_lane_bytes<16>(buffer_rsrc(c.bs[j] + t * kTileRows, kTileRows), pend ? lane * 32 : kOutOfRange, x);
                lane_masks<MODE>(x, cl, ch, rlo, elo, rhi, ehi);
                m = j < K ? ~0u : 0u;
            } else {
                const uint32_t mj = load_mask_dword(c, j, t, lane * 4);
                const uint32_t run0 = c.dir[j][(t * kTileRows) >> c.dir_shift];
                const uint32_t pc = (uint32_t)__builtin_popcount(mj);
                const uint32_t incl = wave_incl_sum(pc);
                const uint32_t runlen = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
                const uint32_t excl = incl - pc;
                if (COUNT) count_level(st, j, pend, mj, lane, (uint64_t)run0 + excl);
                if (wave_any((uint32_t)__builtin_popcount(pend) > lit.gather)) {
                    settle_staged(c, lit, t, j, run0, runlen, excl, mj, lane, s, lds, st);
                    continue;
                }
                const auto rj = buffer_rsrc(c.bs[j] + run0, runlen);
                uint32_t rem = pend, bit[kGatherSlots], b[kGatherSlots];
                Unroll<0, kGatherSlots>::run([&](auto sc) {
                    constexpr int k = decltype(sc)::value;
                    const uint32_t beta = rem & (0u - rem);
                    const uint32_t off = beta ? excl + (uint32_t)__builtin_popcount(mj & (beta - 1u)) : kOutOfRange;
                    bit[k] = beta;
                    b[k] = __builtin_amdgcn_raw_buffer_load_b8(rj, (int)off, 0, 0);
                    rem ^= beta;
                });
                m = j < K ? load_mask_dword(c, j + 1, t, pend ? lane * 4 : kOutOfRange) : 0u;
                Unroll<0, kGatherSlots>::run([&](auto sc) {
                    constexpr int k = decltype(sc)::value;
                    row_masks<MODE>(b[k], bit[k], cl, ch, rlo, elo, rhi, ehi);
                });
            }
            if (COUNT && !DENSE && j < K) {
                const uint32_t tied = tied_next(lit, j, s.plo & elo, s.phi & ehi);
                st.alg += 8ull * groups_with(tied);
                st.lines += mask_lines(tied);
            }
            apply_level<MODE>(s.out, s.plo, s.phi, rlo, elo, rhi, ehi, m, j < lit.llo ? ~0u : 0u,
                              j < lit.lhi ? ~0u : 0u);
        }
    }

    // Tiles t_begin, t_begin + stride, ... below t_end.  The loads of the next
    // tiles are issued ahead (unconditionally: a slot past the end reads
    // nothing), and a tile's level-2 reads are used one tile later.  The loop
    // has one exit, and no register is copied between tiles (a copy would wait
    // for the load it copies).
    __device__ static void range(const DevCol& c, const ScanLit& lit, const uint64_t* __restrict__ in_mask,
                                 uint64_t* __restrict__ out, uint64_t t_begin, uint64_t t_end, uint64_t stride,
                                 uint32_t lane, uint8_t* lds, Stats& st) {
        if (t_begin >= t_end) return;
        uint64_t t = t_begin;
        // 32-bit uniform counters decide which slots hold a tile
        const uint32_t mine = (uint32_t)((t_end - t_begin + stride - 1) / stride);
        if constexpr (kByte1Only) {
            // settled by byte 1 (and M_2): the next tile's loads are issued once
            // this one is done (measured: deeper prefetch only adds concurrent
            // streams, which HBM serves less efficiently)
            TileData a = load(c, in_mask, t, lane, true);
            TileState s;
            for (uint32_t i = 0; i < mine; ++i) {
                begin(c, lit, t, lane, a, s, lds, st, true);
                finish(c, lit, out, t, lane, s, lds, st, true);
                a = load(c, in_mask, t + stride, lane, i + 1 < mine);
                t += stride;
            }
        } else {
            // tile i's level-2 reads are in flight while tile i+1's byte 1 is compared
            TileData a = load(c, in_mask, t, lane, true);
            TileData b = load(c, in_mask, t + stride, lane, 1 < mine);
            TileState sa, sb;
            begin(c, lit, t, lane, a, sa, lds, st, true);
            a = load(c, in_mask, t + 2 * stride, lane, 2 < mine);
            for (uint32_t i = 0; i < mine; i += 2) {
                begin(c, lit, t + stride, lane, b, sb, lds, st, i + 1 < mine);
                b = load(c, in_mask, t + 3 * stride, lane, i + 3 < mine);
                finish(c, lit, out, t, lane, sa, lds, st, true);
                t += stride;
                begin(c, lit, t + stride, lane, a, sa, lds, st, i + 2 < mine);
                a = load(c, in_mask, t + 3 * stride, lane, i + 4 < mine);
                finish(c, lit, out, t, lane, sb, lds, st, i + 1 < mine);
                t += stride;
            }
        }
    }
};

// Waves per SIMD the variant is built for: 8 (64 VGPRs) where a tile's work
// ends with its byte-1 pass; variants that keep a tile's later-byte reads in
// flight (two tiles' gathered bytes or dense slice bytes besides two tiles'
// loads), and BETWEEN with its two literals, are built for 7 (73 VGPRs);
// ByteSlice BETWEEN with a multi-byte literal, whose tile state holds a lane's
// 32 bytes of the second slice, for 6 (85 VGPRs).
template <int MODE, int SHORT, bool DENSE>
constexpr int scan_waves() {
    constexpr bool one = SliceScan<MODE, SHORT, DENSE, false, false>::kByte1Only;
    return (one && MODE != kModeBetween) ? 8 : (DENSE && MODE == kModeBetween && !one) ? 6 : 7;
}

template <int MODE, int SHORT, bool DENSE, bool HAS_IN, bool COUNT>
__device__ __forceinline__ void scan_slices_range(const DevCol& c, const ScanLit& lit,
                                                  const uint64_t* __restrict__ in_mask, uint64_t* __restrict__ out,
                                                  uint64_t t_begin, uint64_t t_end, uint64_t stride, uint32_t lane,
                                                  uint8_t* lds, Stats& st) {
    SliceScan<MODE, SHORT, DENSE, HAS_IN, COUNT>::range(c, lit, in_mask, out, t_begin, t_end, stride, lane, lds, st);
}

}  // namespace dev
}  // namespace bst
