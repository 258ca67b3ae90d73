#pragma once
// Device code shared by the gfx950 kernels of the ByteStore library.
//
// Device layouts (built by host_encode.cpp), all in tiles of 2048 rows:
//  * first byte slice BS_1 (PP-VBS, ByteSlice): in tile t, lane L of a wave owns
//    the 32 rows t*2048 + k*64 + L (k = 0..31), stored as 32 contiguous bytes at
//    t*2048 + L*32.  Two 16-byte loads per lane bring a whole tile in, and byte k
//    of every lane is exactly one 64-row group in row order, so a ballot over a
//    byte compare is one result word.
//  * later slices: ByteSlice BS_j tile-interleaved like BS_1; PP-VBS BS_j compacted in
//    row order (only rows with a j-th byte), bitmask M_j one uint64 per 64 rows,
//    directory DIR_j = running count of j-th bytes every 2^dir_shift rows.
//  * Bit-Packed: in tile t, lane L's 32 codes packed LSB first into w dwords;
//    dword i of lane L at t*64*w + i*64 + L.
//
// Result bitvectors: uint64 words, bit r % 64 of word r / 64.  Each tile's 32
// words are produced by one wave (no atomics) and written by one coalesced
// 256-byte store.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <type_traits>

#include "internal.h"

namespace bst {
namespace dev {

constexpr int kBlock = 256;           // threads per workgroup: 4 waves
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kMinWaves = 6;            // waves per SIMD the scan kernels are built for

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// number of set bits of m below this lane
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// v_writelane: lane `lane` of `old` takes the uniform value `src` (the compiler
// inserts the wait states that a preceding scalar write of `src` needs).
__device__ int bst_writelane_i32(int src, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

// Lanes 2k and 2k+1 of v take the low and high halves of the uniform word w.
__device__ __forceinline__ uint32_t put_word_at(uint32_t v, uint32_t k, uint64_t w) {
    v = (uint32_t)bst_writelane_i32((int)(uint32_t)w, (int)(2 * k), (int)v);
    return (uint32_t)bst_writelane_i32((int)(uint32_t)(w >> 32), (int)(2 * k + 1), (int)v);
}

// Calls f(std::integral_constant<int, I>) for I = 0..N-1, unrolled at compile time.
template <int I, int N>
struct Unroll {
    template <class F>
    __device__ __forceinline__ static void run(F&& f) {
        f(std::integral_constant<int, I>{});
        Unroll<I + 1, N>::run(f);
    }
};
template <int N>
struct Unroll<N, N> {
    template <class F>
    __device__ __forceinline__ static void run(F&&) {}
};

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// byte j (1-based) of a literal padded to BST_KMAX bytes
__device__ __forceinline__ uint32_t lit_byte(uint64_t lit6, uint32_t j) {
    return (uint32_t)(lit6 >> (8 * (BST_KMAX - j))) & 0xffu;
}

__device__ __forceinline__ uint64_t valid_mask(uint64_t word, uint64_t n) {
    uint64_t nwords = (n + 63) >> 6;
    if (word >= nwords) return 0;
    if (word == nwords - 1 && (n & 63)) return (1ull << (n & 63)) - 1;
    return ~0ull;
}

struct Stats {
    uint64_t alg = 0, rowbytes = 0, deep_groups = 0, full = 0;
};

// Position in BS_j of the first j-th byte of 64-row group g (PP-VBS): the
// directory entry at or before the group plus the mask popcounts in between.
__device__ __forceinline__ uint64_t vbs_group_base(const DevCol& c, uint32_t j, uint64_t g) {
    const uint64_t row = g << 6;
    const uint64_t q = row >> c.dir_shift;
    uint64_t base = c.dir[j][q];
    const uint64_t* m = c.m[j];
    for (uint64_t gg = (q << c.dir_shift) >> 6; gg < g; ++gg) base += __builtin_popcountll(m[gg]);
    return base;
}

// ------------------------------------------------------------ slice scan
// A tile of a slice-layout scan is one wave's work: 32 groups of 64 rows, each
// group's result one uint64 word.  The comparison of a row against a literal
// proceeds byte by byte (Sec. 3.3, Algorithm 3 generalised to every operator):
// a row whose byte differs from the literal's is decided; a row still equal
// after byte j stays pending, except that at j < l a row without a byte j+1 is
// a proper prefix of the literal and hence smaller (the literal's remaining
// bytes are not all zero), and at j = l a row with a byte l+1 is greater, one
// without it equal.  Bytes compare unsigned.
//
// Byte 1 is compared for all 32 groups from registers; the presence of byte 2
// (M_2, prefetched with the tile) settles what the lengths decide; later bytes
// are read only for rows still undecided -- the early stop of Algorithm 3,
// tested wave-uniformly per tile and level (see process_tile).

// Per-lane registers of one tile.
struct TileData {
    uint4 q0, q1;   // 32 first-slice bytes: byte k is row tile*2048 + 64k + lane
    uint32_t m2;    // PP-VBS: dword `lane` of the tile's 32 M_2 words (0 when unused)
    uint32_t m3;    // PP-VBS: the same of M_3 (0 when the column has no third byte)
    uint32_t in;    // dword `lane` of the tile's 32 incoming-mask words (all ones when none)
    uint32_t dir2;  // PP-VBS: the directory entry of BS_2 at the tile's first row, where the
                    // tile's run of BS_2 starts (the same in every lane)
};

// Raw buffer access (gfx9-family descriptor: no format, no swizzle).  A buffer
// load past num_records returns zeros without touching memory, so every load
// below is issued unconditionally: the hardware's in-order count of pending
// loads then matches the program order exactly, and the compiler can wait for
// one tile's data while the next tiles' loads stay in flight.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kRawBufferWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRawBufferWord3);
}

__device__ __forceinline__ uint4 buffer_load16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
    return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ uint32_t buffer_load4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
}

// Lane's dword of the 32 mask words of tile t for level j (0 when the column has
// no byte j, or when `valid` is false).
__device__ __forceinline__ uint32_t load_mask_dword(const DevCol& c, uint32_t j, uint64_t t, uint32_t lane,
                                                    bool valid = true) {
    const bool has = valid && j <= c.K;
    const void* base = has ? (const void*)(c.m[j] + t * 32) : (const void*)c.bs[1];
    return buffer_load4(buffer_rsrc(base, has ? 256u : 0u), lane * 4);
}

// Loads of tile t (all zeros when `valid` is false: no memory is read).
template <bool DENSE, bool HAS_IN>
__device__ __forceinline__ TileData load_tile(const DevCol& c, const uint64_t* __restrict__ in_mask, uint64_t t,
                                              uint32_t lane, bool valid = true) {
    TileData d;
    const auto r1 = buffer_rsrc(c.bs[1] + (valid ? t * kTileRows : 0), valid ? kTileRows : 0u);
    d.q0 = buffer_load16(r1, lane * 32);
    d.q1 = buffer_load16(r1, lane * 32 + 16);
    d.m2 = DENSE ? 0u : load_mask_dword(c, 2, t, lane, valid);
    d.m3 = DENSE ? 0u : load_mask_dword(c, 3, t, lane, valid);
    d.dir2 = 0;
    if (!DENSE) {
        // fetched with the tile, in the same in-order stream of vector loads: level
        // 2's gathers then wait for nothing issued after the tile's own loads
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

// 64-bit value held by lanes 2k (low half) and 2k+1 (high half) of v; k uniform.
__device__ __forceinline__ uint64_t lane_word(uint32_t v, uint32_t k) {
    return (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)v, (int)(2 * k)) |
           ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)v, (int)(2 * k + 1)) << 32);
}

// Rows equal to the literal on bytes 1..j meet m (rows that have a byte j+1):
// settle what the lengths decide.  plo: pending against the (lower) literal,
// phi: pending against the upper BETWEEN literal; hit: rows newly found in the
// tracked relation (LT / GT / EQ; BETWEEN: below lo or above hi).  klo / khi are
// all ones while j is shorter than the literal (j < l), else zero.
template <int MODE>
__device__ __forceinline__ void level_mask_step(uint64_t& plo, uint64_t& phi, uint64_t& hit, uint64_t m,
                                                uint64_t klo, uint64_t khi) {
    if (MODE == kModeLT || MODE == kModeBetween) {
        hit |= plo & ~m & klo;       // a proper prefix of the literal is below it
    } else if (MODE == kModeGT) {
        hit |= plo & m & ~klo;       // equal over the literal's length, then more bytes: above
    } else {
        hit |= plo & ~m & ~klo;      // equal over the literal's length and no more bytes: equal
    }
    plo &= m & klo;
    if (MODE == kModeBetween) {
        hit |= phi & m & ~khi;
        phi &= m & khi;
    }
}

template <int MODE>
__device__ __forceinline__ void level_step(uint64_t& plo, uint64_t& phi, uint64_t& hit, uint64_t m, uint32_t j,
                                           uint32_t llo, uint32_t lhi) {
    level_mask_step<MODE>(plo, phi, hit, m, j < llo ? ~0ull : 0ull, j < lhi ? ~0ull : 0ull);
}

// Compare byte j+1 (bb, valid in pending lanes) against the literal's byte.
template <int MODE>
__device__ __forceinline__ void byte_step(uint64_t& plo, uint64_t& phi, uint64_t& hit, uint32_t bb, uint32_t clo,
                                          uint32_t chi) {
    if (MODE == kModeLT || MODE == kModeBetween) hit |= ballot(bb < clo) & plo;
    if (MODE == kModeGT) hit |= ballot(bb > clo) & plo;
    if (MODE == kModeBetween) hit |= ballot(bb > chi) & phi;
    plo &= ballot(bb == clo);
    if (MODE == kModeBetween) phi &= ballot(bb == chi);
}

// Fold newly settled rows into a group's result word (kept un-negated until the
// tile is stored: rows in the relation for '<', '>', '='; rows in range for BETWEEN).
template <int MODE>
__device__ __forceinline__ uint64_t apply_hit(uint64_t res, uint64_t hit) {
    return MODE == kModeBetween ? (res & ~hit) : (res | hit);
}

// Bytes an exhaustive (no early stop) scan of this tile would touch.
template <bool DENSE>
__device__ uint64_t full_read_bytes(const DevCol& c, const ScanLit& lit, uint64_t t, bool has_in) {
    uint32_t l = lit.llo > lit.lhi ? lit.llo : lit.lhi;
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

// Inclusive prefix sum over the wave's lanes.
// DPP moves (row_shr within each 16-lane row, then row_bcast:15 / :31 across
// rows) instead of LDS permutes: six dependent VALU adds.  Lanes without a
// source lane, and rows masked off, add 0.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v, uint32_t lane) {
    (void)lane;
    constexpr int kRowShr = 0x110, kRowBcast15 = 0x142, kRowBcast31 = 0x143;
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowShr + 1, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowShr + 2, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowShr + 4, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowShr + 8, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowBcast15, 0xa, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowBcast31, 0xc, 0xf, false);
    return v;
}

// Sum over the wave's lanes (uniform).
__device__ __forceinline__ uint32_t wave_sum(uint32_t v, uint32_t lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_sum(v, lane), 63);
}

// Bit k set when the 64-bit word of group k (lanes 2k and 2k+1 of v) is non-zero.
__device__ __forceinline__ uint32_t group_mask(uint32_t v) {
    uint64_t b = ballot(v != 0);
    b = (b | (b >> 1)) & 0x5555555555555555ull;   // group k's flag at bit 2k
    b = (b | (b >> 1)) & 0x3333333333333333ull;   // then gather the even bits
    b = (b | (b >> 2)) & 0x0f0f0f0f0f0f0f0full;
    b = (b | (b >> 4)) & 0x00ff00ff00ff00ffull;
    b = (b | (b >> 8)) & 0x0000ffff0000ffffull;
    b = (b | (b >> 16)) & 0x00000000ffffffffull;
    return (uint32_t)b;
}

constexpr uint32_t kStageBytes = 2080;   // 130 chunks of 16 bytes: a 2048-byte run plus alignment

// Per-wave LDS scratch of the row-sparse level (after the staged run): the list
// of pending rows, then per lane dword of the tile the rows found in the
// relation, the rows still tied with the lower / upper literal, and (for the
// instrumented build) the rows equal on the level's byte.
constexpr uint32_t kSparseRows = 256;   // up to four rows per lane, in rounds of 64
struct SparseLds {
    uint16_t list[kSparseRows];
    uint32_t hit[64], lo[64], hi[64], eq[64];
};
constexpr uint32_t kWaveLds = kStageBytes + sizeof(SparseLds);

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

// One level for a tile with at most kSparseRows pending rows: one row per lane
// and round of 64.  The pending rows (bits of plov | phiv) are listed in LDS;
// each lane takes one per round and finds its byte j (PP-VBS: the directory
// entry plus the M_j popcounts before it; ByteSlice: its place in the
// tile-interleaved slice).  The gathers of all rounds are issued first; then,
// round by round, each lane applies the byte and length rules of the level to
// its row alone and sets the row's bits in the per-dword outcome arrays with
// LDS atomics; every lane then reads back its dword.  incl: inclusive lane prefix of the M_j dword popcounts
// (PP-VBS); row_excl / total: this lane's exclusive prefix and the tile's total
// of pending rows.
// The byte rules of one level for one row: b is the row's byte, cl / ch the
// literals' bytes at this level, plo / phi whether the row is still equal to the
// lower / upper literal, more whether the row has a next byte, lo_open / hi_open
// whether the literal goes on after this byte.  Returns flags: kRuleHit (found
// in the tracked relation; BETWEEN: out of range), kRuleKeepLo / kRuleKeepHi
// (still equal, and the row has a next byte) and kRuleEq (the byte equals a
// literal's).  Flags rather than reference outputs: a store to one of two
// locals chosen at run time would put them in scratch memory.
constexpr uint32_t kRuleHit = 1, kRuleKeepLo = 2, kRuleKeepHi = 4, kRuleEq = 8;

template <int MODE>
__device__ __forceinline__ uint32_t row_rule(uint32_t b, uint32_t cl, uint32_t ch, bool plo, bool phi, bool more,
                                             bool lo_open, bool hi_open) {
    uint32_t f = 0;
    if (plo) {
        if (b == cl) f |= kRuleEq;
        if (MODE == kModeLT || MODE == kModeBetween) {
            if (b < cl) f |= kRuleHit;                                           // below
            else if (b == cl && lo_open) f |= more ? kRuleKeepLo : kRuleHit;     // a prefix: below
        } else if (MODE == kModeGT) {
            if (b > cl) f |= kRuleHit;                                           // above
            else if (b == cl && more) f |= lo_open ? kRuleKeepLo : kRuleHit;     // equal, then more: above
        } else {
            if (b == cl) {                                                       // equal over the literal
                if (lo_open) f |= more ? kRuleKeepLo : 0u;
                else f |= more ? 0u : kRuleHit;
            }
        }
    }
    if (MODE == kModeBetween && phi) {
        if (b == ch) f |= kRuleEq;
        if (b > ch) f |= kRuleHit;                                               // above the upper literal
        else if (b == ch && more) f |= hi_open ? kRuleKeepHi : kRuleHit;
    }
    return f;
}

template <int MODE, bool DENSE, bool COUNT>
__device__ __forceinline__ void sparse_level(const DevCol& c, const ScanLit& lit, uint64_t t, uint32_t j,
                                             uint64_t run0, uint32_t cur_mv, uint32_t next_mv, uint32_t incl,
                                             uint32_t& outv, uint32_t& plov, uint32_t& phiv, uint32_t lane,
                                             SparseLds* sp, uint32_t row_excl, uint32_t total, uint32_t& eq_rows) {
    const uint32_t K = c.K;
    sp->hit[lane] = 0;
    sp->lo[lane] = 0;
    sp->hi[lane] = 0;
    if (COUNT) sp->eq[lane] = 0;
    uint32_t v = plov | phiv;
    uint32_t idx = row_excl;
    while (v) {
        const uint32_t b = __builtin_ctz(v);
        v &= v - 1;
        sp->list[idx++] = (uint16_t)((lane << 5) | b);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // All rounds' gathers are issued before any is used, so the tile waits for
    // one gather however many rounds it has; the rules then run round by round.
    constexpr int kRounds = kSparseRows / 64;
    uint32_t bb[kRounds];
    Unroll<0, kRounds>::run([&](auto rc) {
        constexpr uint32_t r = decltype(rc)::value;
        bb[r] = 0;
        if (r * 64 < total) {
            // every lane runs the cross-lane reads (lanes past `total` on entry 0)
            const uint32_t ent = r * 64 + lane;
            const uint32_t e = ent < total ? (uint32_t)sp->list[ent] : 0u;
            const uint32_t jd = e >> 5, bit = e & 31, k = jd >> 1;
            const uint32_t below = (1u << bit) - 1u;
            uint32_t pos;
            if (DENSE) {
                pos = (((jd & 1) << 5) | bit) * 32 + k;   // tile-interleaved: lane-in-group * 32 + group
            } else {
                const uint32_t mlo = __shfl(cur_mv, (int)(2 * k), 64);
                const uint32_t mhi = __shfl(cur_mv, (int)(2 * k + 1), 64);
                const uint32_t before = __shfl(incl, (int)(k ? 2 * k - 1 : 0), 64);
                pos = (k ? before : 0u) + ((jd & 1) ? (uint32_t)__builtin_popcount(mlo) : 0u) +
                      (uint32_t)__builtin_popcount(((jd & 1) ? mhi : mlo) & below);
            }
            if (ent < total) bb[r] = c.bs[j][run0 + pos];
        }
    });
    const uint32_t cl = lit_byte(lit.lo, j), ch = lit_byte(lit.hi, j);
    const bool lo_open = j < lit.llo, hi_open = j < lit.lhi;   // the literal goes on after byte j
    Unroll<0, kRounds>::run([&](auto rc) {
        constexpr uint32_t r = decltype(rc)::value;
        if (r * 64 < total) {
            const uint32_t ent = r * 64 + lane;
            const uint32_t e = ent < total ? (uint32_t)sp->list[ent] : 0u;
            const uint32_t jd = e >> 5, bit = e & 31;
            const uint32_t plo_w = __shfl(plov, (int)jd, 64), phi_w = __shfl(phiv, (int)jd, 64);
            const uint32_t nxt_w = __shfl(next_mv, (int)jd, 64);
            if (ent < total) {
                const bool plo = (plo_w >> bit) & 1, phi = (phi_w >> bit) & 1;
                const bool more = j < K && (DENSE || ((nxt_w >> bit) & 1));   // the row has a byte j+1
                const uint32_t f = row_rule<MODE>(bb[r], cl, ch, plo, phi, more, lo_open, hi_open);
                const uint32_t m = 1u << bit;
                if (f & kRuleHit) atomicOr(&sp->hit[jd], m);
                if (f & kRuleKeepLo) atomicOr(&sp->lo[jd], m);
                if (f & kRuleKeepHi) atomicOr(&sp->hi[jd], m);
                if (COUNT && (f & kRuleEq)) atomicOr(&sp->eq[jd], m);
            }
        }
    });
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint32_t h = sp->hit[lane];
    outv = MODE == kModeBetween ? (outv & ~h) : (outv | h);
    plov = sp->lo[lane];
    phiv = MODE == kModeBetween ? sp->hi[lane] : 0u;
    eq_rows = COUNT ? sp->eq[lane] : 0u;
}

// The length rule of a level on lane-held words (32 rows per lane dword): rows
// still equal to the literal (plov / phiv) either have a next byte (m) or end.
// Returns the rows newly found in the tracked relation; klo / khi are all ones
// while the level is shorter than the lower / upper literal.
template <int MODE>
__device__ __forceinline__ uint32_t level_mask_vec(uint32_t& plov, uint32_t& phiv, uint32_t m, uint32_t klo,
                                                   uint32_t khi) {
    uint32_t hit;
    if (MODE == kModeLT || MODE == kModeBetween) hit = plov & ~m & klo;   // a proper prefix: below
    else if (MODE == kModeGT) hit = plov & m & ~klo;                     // equal, then more bytes: above
    else hit = plov & ~m & ~klo;                                         // equal over the whole literal
    plov &= m & klo;
    if (MODE == kModeBetween) {
        hit |= phiv & m & ~khi;
        phiv &= m & khi;
    }
    return hit;
}

// One tile, one wave.
//
// Byte 1: for each of the 32 groups (unrolled, the tile is in registers) the
// ballots of the byte-1 compares land, as 64-bit words, in lanes 2k and 2k+1 of
// three word vectors: `res` (rows decided in the relation; BETWEEN: rows in
// range so far), `plo` / `phi` (rows equal so far to the lower / upper literal).
// No branches, no scalar work per group.
//
// Byte 2's presence: the tile's M_2 words sit in the same lane layout (one dword
// per lane), so the length rules settle all 32 groups at once with a few
// bitwise vector operations.
//
// Later bytes: only groups with rows still pending are visited, four at a time
// (their reads issued before any is waited on).  Per level, a tile with many
// pending groups copies its run of the slice into LDS with one coalesced read;
// one with few gathers just the pending groups' bytes.  So later slices are read
// only for undecided groups -- Algorithm 3's early stop at 64-row granularity,
// tested wave-uniformly.
template <int MODE, int SHORT, bool DENSE, bool HAS_IN, bool COUNT>
__device__ __forceinline__ void process_tile(const DevCol& c, const ScanLit& lit, uint64_t* __restrict__ out,
                                             uint64_t t, uint32_t lane, const TileData& td, uint8_t* lds,
                                             Stats& st, bool live) {
    if (!live) return;   // past the wave's last tile (a prefetch slot with nothing to do)
    const uint64_t w0 = t * 32;
    const uint32_t K = c.K;
    const uint32_t clo = lit_byte(lit.lo, 1), chi = lit_byte(lit.hi, 1);
    const uint32_t dw[8] = {td.q0.x, td.q0.y, td.q0.z, td.q0.w, td.q1.x, td.q1.y, td.q1.z, td.q1.w};
    // rows this lane's result dword may report: selected by the incoming mask and
    // inside the column
    const uint64_t d = w0 * 2 + lane;
    // 32-bit compare of uniform values (tile indices fit: directory entries are
    // 32-bit): a 64-bit one needs a vector register for one side on this chip,
    // which is then held, or spilled, across the whole loop
    const bool full = (uint32_t)t < (uint32_t)(c.n / kTileRows);
    uint32_t actv = HAS_IN ? td.in : ~0u;
    if (!full) {
        const uint64_t r0 = d * 32;
        actv &= r0 + 32 <= c.n ? ~0u : (r0 < c.n ? (1u << (c.n - r0)) - 1u : 0u);
    }
    // SHORT bit 0 (bit 1): the lower (upper) literal is one byte long; SHORT < 0:
    // the lengths are read at run time
    constexpr bool kLoShort = SHORT >= 0 && (SHORT & 1) != 0;
    constexpr bool kHiShort = SHORT >= 0 && (SHORT & 2) != 0;
    // rows equal to a one-byte '<' or lower-BETWEEN literal on byte 1 are never
    // below it: their equal-so-far ballot is not needed
    constexpr bool kNeedLo = !((MODE == kModeLT || MODE == kModeBetween) && kLoShort);
    const uint32_t klo = SHORT < 0 ? (1 < lit.llo ? ~0u : 0u) : (kLoShort ? 0u : ~0u);
    const uint32_t khi = SHORT < 0 ? (1 < lit.lhi ? ~0u : 0u) : (kHiShort ? 0u : ~0u);
    const uint32_t span1 = chi - clo;   // BETWEEN: byte 1 in [clo, chi]
    // two registers per vector, alternating groups, so consecutive lane writes
    // do not chain
    uint32_t rq[2] = {0, 0}, pq[2] = {0, 0}, hq[2] = {0, 0};
    Unroll<0, 32>::run([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const uint32_t b = (dw[k >> 2] >> (8 * (k & 3))) & 0xffu;
        if (MODE == kModeLT) rq[k & 1] = put_word_at(rq[k & 1], k, ballot(b < clo));
        if (MODE == kModeGT) rq[k & 1] = put_word_at(rq[k & 1], k, ballot(b > clo));
        if (MODE == kModeBetween) rq[k & 1] = put_word_at(rq[k & 1], k, ballot(b - clo <= span1));
        if (kNeedLo) pq[k & 1] = put_word_at(pq[k & 1], k, ballot(b == clo));
        if (MODE == kModeBetween) hq[k & 1] = put_word_at(hq[k & 1], k, ballot(b == chi));
    });
    uint32_t outv = rq[0] | rq[1];
    uint32_t plov = (pq[0] | pq[1]) & actv;
    uint32_t phiv = (hq[0] | hq[1]) & actv;
    if (COUNT) {
        st.alg += kTileRows + 256 + (HAS_IN ? 256 : 0);
        st.full += full_read_bytes<DENSE>(c, lit, t, HAS_IN);
        st.rowbytes += wave_sum(__builtin_popcount(actv), lane);
        // M_2 words read: the groups with rows equal on byte 1
        if (!DENSE && K >= 2) st.alg += 8ull * __builtin_popcount(group_mask(plov | phiv));
    }
    // byte 2's presence settles the rows equal on byte 1 that end there
    {
        const uint32_t m2v = DENSE ? (K >= 2 ? ~0u : 0u) : td.m2;
        const uint32_t hit = level_mask_vec<MODE>(plov, phiv, m2v, klo, khi);
        outv = MODE == kModeBetween ? (outv & ~hit) : (outv | hit);
    }
    // later bytes, pending groups only
    // one-byte literals are settled by now (nothing stays pending); say so at
    // compile time so the later-byte code drops out
    constexpr bool kByte1Only = MODE == kModeBetween ? (kLoShort && kHiShort) : kLoShort;
    uint32_t pend = kByte1Only ? 0u : group_mask(plov | phiv);
    if constexpr (DENSE) {
        // ByteSlice: every row has every byte and slice j is tile-interleaved like
        // slice 1, so byte j of the tile is one 2 KB read into the same lane layout
        // and a level settles all pending groups with compares and lane writes
        for (uint32_t j = 2; pend != 0 && j <= K; ++j) {
            if (COUNT) {
                if (j == 2) st.deep_groups += __builtin_popcount(pend);
                st.alg += 64ull * __builtin_popcount(pend);
                st.rowbytes += wave_sum(__builtin_popcount(plov | phiv), lane);
            }
            {
                // few pending rows: gather just their bytes, one row per lane and
                // round (a single literal's byte compares on the whole 2 KB are
                // cheap enough that more than one round does not pay)
                constexpr uint32_t kMaxRows = MODE == kModeBetween ? kSparseRows : 64;
                const uint32_t prow = __builtin_popcount(plov | phiv);
                const uint32_t rincl = wave_incl_sum(prow, lane);
                const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)rincl, 63);
                if (total <= kMaxRows) {
                    uint32_t eq_rows = 0;
                    sparse_level<MODE, true, COUNT>(c, lit, t, j, t * kTileRows, 0u, 0u, 0u, outv, plov, phiv, lane,
                                                    reinterpret_cast<SparseLds*>(lds + kStageBytes), rincl - prow,
                                                    total, eq_rows);
                    pend = group_mask(plov | phiv);
                    continue;
                }
            }
            const auto rj = buffer_rsrc(c.bs[j] + t * kTileRows, kTileRows);
            const uint4 a0 = buffer_load16(rj, lane * 32), a1 = buffer_load16(rj, lane * 32 + 16);
            const uint32_t bw[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
            const uint32_t cjlo = lit_byte(lit.lo, j), cjhi = lit_byte(lit.hi, j);
            uint32_t xq[2] = {0, 0}, eq[2] = {0, 0}, yq[2] = {0, 0}, fq[2] = {0, 0};
            Unroll<0, 32>::run([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                if ((pend >> k) & 1u) {
                    const uint32_t b = (bw[k >> 2] >> (8 * (k & 3))) & 0xffu;
                    // xq: rows leaving the lower literal's tie in the tracked direction
                    if (MODE == kModeLT || MODE == kModeBetween) xq[k & 1] = put_word_at(xq[k & 1], k, ballot(b < cjlo));
                    if (MODE == kModeGT) xq[k & 1] = put_word_at(xq[k & 1], k, ballot(b > cjlo));
                    eq[k & 1] = put_word_at(eq[k & 1], k, ballot(b == cjlo));
                    if (MODE == kModeBetween) {
                        yq[k & 1] = put_word_at(yq[k & 1], k, ballot(b > cjhi));
                        fq[k & 1] = put_word_at(fq[k & 1], k, ballot(b == cjhi));
                    }
                }
            });
            uint32_t hit = MODE == kModeEQ ? 0u : (plov & (xq[0] | xq[1]));
            plov &= eq[0] | eq[1];
            if (MODE == kModeBetween) {
                hit |= phiv & (yq[0] | yq[1]);
                phiv &= fq[0] | fq[1];
            }
            hit |= level_mask_vec<MODE>(plov, phiv, j < K ? ~0u : 0u, j < lit.llo ? ~0u : 0u, j < lit.lhi ? ~0u : 0u);
            outv = MODE == kModeBetween ? (outv & ~hit) : (outv | hit);
            pend = group_mask(plov | phiv);
        }
        pend = 0;
    }
    uint32_t cur_mv = DENSE ? 0u : td.m2;   // this lane's dword of the tile's M_j words
    for (uint32_t j = 2; pend != 0 && j <= K; ++j) {
        if (COUNT && j == 2) st.deep_groups += __builtin_popcount(pend);
        const uint32_t next_mv = (!DENSE && j < K) ? (j == 2 ? td.m3 : load_mask_dword(c, j + 1, t, lane)) : 0u;
        uint32_t incl = 0;
        uint64_t run0;
        uint32_t runlen;
        // one lane prefix for two counts: this level's bytes (M_j bits, high half)
        // and the pending rows (low half); each sums to at most 2048
        const uint32_t prow = __builtin_popcount(plov | phiv);
        const uint32_t both = wave_incl_sum(((uint32_t)__builtin_popcount(cur_mv) << 16) | prow, lane);
        const uint32_t rincl = both & 0xffffu;
        const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)both, 63) & 0xffffu;
        if (DENSE) {
            run0 = t * kTileRows;
            runlen = kTileRows;
        } else {
            incl = both >> 16;
            run0 = j == 2 ? (uint32_t)__builtin_amdgcn_readfirstlane((int)td.dir2)
                          : c.dir[j][(t * kTileRows) >> c.dir_shift];
            runlen = (uint32_t)__builtin_amdgcn_readlane((int)both, 63) >> 16;
        }
        // few pending rows: one row per lane and round
        {
            if (total <= kSparseRows) {
                if (COUNT) {
                    st.rowbytes += total;
                    st.alg += wave_sum(((pend >> (lane >> 1)) & 1) ? __builtin_popcount(cur_mv) : 0u, lane);
                }
                uint32_t eq_rows = 0;
                sparse_level<MODE, false, COUNT>(c, lit, t, j, run0, cur_mv, next_mv, incl, outv, plov, phiv, lane,
                                                 reinterpret_cast<SparseLds*>(lds + kStageBytes), rincl - prow, total,
                                                 eq_rows);
                if (COUNT && j < K) st.alg += 8ull * __builtin_popcount(group_mask(eq_rows));
                pend = group_mask(plov | phiv);
                cur_mv = next_mv;
                continue;
            }
        }
        // stage the tile's run of BS_j when enough groups need it
        const bool staged = (uint32_t)__builtin_popcount(pend) >= lit.stage;
        const uint32_t cjlo = lit_byte(lit.lo, j), cjhi = lit_byte(lit.hi, j);
        uint32_t pend_next = 0;
        if (staged) {
            // the run is in LDS: read the pending groups' bytes at compile-time
            // group positions (eight reads in flight), compare into lane words,
            // and settle the level for the whole tile with vector operations
            const uint32_t sh = stage_run(c.bs[j], run0, runlen, lds, lane);
            if (COUNT) st.rowbytes += wave_sum(__builtin_popcount(plov | phiv), lane);
            uint32_t xq[2] = {0, 0}, eq[2] = {0, 0}, yq[2] = {0, 0}, fq[2] = {0, 0};
            Unroll<0, 4>::run([&](auto cc) {
                constexpr int c8 = decltype(cc)::value * 8;
                if ((pend >> c8) & 0xffu) {
                    uint32_t bb[8];
                    Unroll<0, 8>::run([&](auto ic) {
                        constexpr int i = decltype(ic)::value, k = c8 + i;
                        bb[i] = 0;
                        if ((pend >> k) & 1u) {
                            uint32_t pos;
                            if (DENSE) {
                                pos = 64 * k + lane;
                            } else {
                                const uint64_t mj = lane_word(cur_mv, k);
                                pos = (k ? (uint32_t)__builtin_amdgcn_readlane((int)incl, 2 * k - 1) : 0u) + mbcnt(mj);
                                if (COUNT) st.alg += __builtin_popcountll(mj);
                            }
                            bb[i] = lds[sh + pos];   // in bounds for every lane; pending lanes are used
                        }
                    });
                    Unroll<0, 8>::run([&](auto ic) {
                        constexpr int i = decltype(ic)::value, k = c8 + i;
                        if ((pend >> k) & 1u) {
                            const uint32_t bj = bb[i];
                            if (MODE == kModeLT || MODE == kModeBetween)
                                xq[k & 1] = put_word_at(xq[k & 1], k, ballot(bj < cjlo));
                            if (MODE == kModeGT) xq[k & 1] = put_word_at(xq[k & 1], k, ballot(bj > cjlo));
                            eq[k & 1] = put_word_at(eq[k & 1], k, ballot(bj == cjlo));
                            if (MODE == kModeBetween) {
                                yq[k & 1] = put_word_at(yq[k & 1], k, ballot(bj > cjhi));
                                fq[k & 1] = put_word_at(fq[k & 1], k, ballot(bj == cjhi));
                            }
                        }
                    });
                }
            });
            uint32_t hit = MODE == kModeEQ ? 0u : (plov & (xq[0] | xq[1]));
            plov &= eq[0] | eq[1];
            if (MODE == kModeBetween) {
                hit |= phiv & (yq[0] | yq[1]);
                phiv &= fq[0] | fq[1];
            }
            const uint32_t mnext = j < K ? (DENSE ? ~0u : next_mv) : 0u;
            if (COUNT && !DENSE && j < K) st.alg += 8ull * __builtin_popcount(group_mask(plov | phiv));
            hit |= level_mask_vec<MODE>(plov, phiv, mnext, j < lit.llo ? ~0u : 0u, j < lit.lhi ? ~0u : 0u);
            outv = MODE == kModeBetween ? (outv & ~hit) : (outv | hit);
            pend_next = group_mask(plov | phiv);
            pend = 0;
        }
        while (pend) {
            uint32_t ks[4], bb[4];
            uint32_t cnt = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                ks[i] = 0;
                bb[i] = 0;
                if (pend) {
                    const uint32_t k = __builtin_ctz(pend);
                    pend &= pend - 1;
                    ks[i] = k;
                    cnt = i + 1;
                    // row position of this lane's byte j within the tile's run
                    uint32_t pos;
                    if (DENSE) {
                        pos = 64 * k + lane;
                        if (COUNT) st.alg += 64;
                    } else {
                        const uint64_t mj = lane_word(cur_mv, k);
                        const uint32_t before =
                            k ? (uint32_t)__builtin_amdgcn_readlane((int)incl, (int)(2 * k - 1)) : 0u;
                        pos = before + mbcnt(mj);
                        if (COUNT) st.alg += __builtin_popcountll(mj);
                    }
                    const uint64_t P = lane_word(plov, k) | (MODE == kModeBetween ? lane_word(phiv, k) : 0ull);
                    if ((P >> lane) & 1) bb[i] = c.bs[j][run0 + pos];
                    if (COUNT) {
                        const uint64_t P = lane_word(plov, k) | (MODE == kModeBetween ? lane_word(phiv, k) : 0ull);
                        st.rowbytes += __builtin_popcountll(P);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if ((uint32_t)i < cnt) {
                    const uint32_t k = ks[i];
                    uint64_t plo = lane_word(plov, k);
                    uint64_t phi = MODE == kModeBetween ? lane_word(phiv, k) : 0ull;
                    uint64_t hit = 0;
                    byte_step<MODE>(plo, phi, hit, bb[i], cjlo, cjhi);
                    if ((plo | phi) != 0) {
                        uint64_t m = 0;
                        if (j < K) {
                            if (DENSE) {
                                m = ~0ull;
                            } else {
                                m = lane_word(next_mv, k);
                                if (COUNT) st.alg += 8;
                            }
                        }
                        level_step<MODE>(plo, phi, hit, m, j, lit.llo, lit.lhi);
                    }
                    if (hit) outv = put_word_at(outv, k, apply_hit<MODE>(lane_word(outv, k), hit));
                    // written back even when settled: the lane words stay exact for the next level
                    plov = put_word_at(plov, k, plo);
                    if (MODE == kModeBetween) phiv = put_word_at(phiv, k, phi);
                    if ((plo | phi) != 0) pend_next |= 1u << k;
                }
            }
        }
        pend = pend_next;
        cur_mv = next_mv;
    }
    // negation as a xor with a mask held in a scalar register (built in a vector
    // register it is kept, or spilled, across the whole loop)
    const uint32_t neg =
        MODE != kModeBetween ? (uint32_t)__builtin_amdgcn_readfirstlane((int)(lit.negate ? ~0u : 0u)) : 0u;
    outv = (outv ^ neg) & actv;
    if (full || d < ((c.n + 63) >> 6) * 2) reinterpret_cast<uint32_t*>(out)[d] = outv;
}

// Scan tiles t_begin, t_begin + stride, ... below t_end, three tiles' loads in
// flight: while one tile is scanned the next two are loading, and no register
// is copied between tiles (a copy would wait for the load it copies).  The loop
// has one exit, at the bottom, so every path through it issues the same loads
// and each tile's wait leaves the next two in flight; a slot past the end loads
// nothing and stores nothing.
template <int MODE, int SHORT, bool DENSE, bool HAS_IN, bool COUNT>
__device__ __forceinline__ void scan_slices_range(const DevCol& c, const ScanLit& lit,
                                                  const uint64_t* __restrict__ in_mask,
                                                  uint64_t* __restrict__ out, uint64_t t_begin, uint64_t t_end,
                                                  uint64_t stride, uint32_t lane, uint8_t* lds, Stats& st) {
    if (t_begin >= t_end) return;
    uint64_t t = t_begin;
    // 32-bit uniform counters decide which slots hold a tile: a 64-bit bound kept
    // live across the loop ended up in vector registers and spilled, and each
    // reload from scratch waited for every load in flight
    const uint32_t mine = (uint32_t)((t_end - t_begin + stride - 1) / stride);
    if constexpr (!DENSE && SHORT == 0 && MODE != kModeBetween) {
        // PP-VBS with a multi-byte literal: two tiles in flight, so that the later
        // levels' working set fits the registers of 8 waves per SIMD
        TileData a = load_tile<DENSE, HAS_IN>(c, in_mask, t, lane);
        TileData b = load_tile<DENSE, HAS_IN>(c, in_mask, t + stride, lane, 1 < mine);
        for (uint32_t i = 0; i < mine; i += 2) {
            process_tile<MODE, SHORT, DENSE, HAS_IN, COUNT>(c, lit, out, t, lane, a, lds, st, true);
            a = load_tile<DENSE, HAS_IN>(c, in_mask, t + 2 * stride, lane, i + 2 < mine);
            t += stride;
            process_tile<MODE, SHORT, DENSE, HAS_IN, COUNT>(c, lit, out, t, lane, b, lds, st, i + 1 < mine);
            b = load_tile<DENSE, HAS_IN>(c, in_mask, t + 2 * stride, lane, i + 3 < mine);
            t += stride;
        }
        return;
    }
    TileData a = load_tile<DENSE, HAS_IN>(c, in_mask, t, lane);
    TileData b = load_tile<DENSE, HAS_IN>(c, in_mask, t + stride, lane, 1 < mine);
    TileData d = load_tile<DENSE, HAS_IN>(c, in_mask, t + 2 * stride, lane, 2 < mine);
    for (uint32_t i = 0; i < mine; i += 3) {
        process_tile<MODE, SHORT, DENSE, HAS_IN, COUNT>(c, lit, out, t, lane, a, lds, st, true);
        a = load_tile<DENSE, HAS_IN>(c, in_mask, t + 3 * stride, lane, i + 3 < mine);
        t += stride;
        process_tile<MODE, SHORT, DENSE, HAS_IN, COUNT>(c, lit, out, t, lane, b, lds, st, i + 1 < mine);
        b = load_tile<DENSE, HAS_IN>(c, in_mask, t + 3 * stride, lane, i + 4 < mine);
        t += stride;
        process_tile<MODE, SHORT, DENSE, HAS_IN, COUNT>(c, lit, out, t, lane, d, lds, st, i + 2 < mine);
        d = load_tile<DENSE, HAS_IN>(c, in_mask, t + 3 * stride, lane, i + 5 < mine);
        t += stride;
    }
}

__device__ __forceinline__ void flush_stats(unsigned long long* counters, const Stats& st, uint32_t lane) {
    if (lane == 0) {
        atomicAdd(counters + 0, (unsigned long long)st.alg);
        atomicAdd(counters + 1, (unsigned long long)st.rowbytes);
        atomicAdd(counters + 2, (unsigned long long)st.deep_groups);
        atomicAdd(counters + 3, (unsigned long long)st.full);
    }
}

// ------------------------------------------------------------ Bit-Packed scan
// Codes are unpacked from registers with compile-time shifts; the predicate is
// one unsigned range test (code - a) <= span prepared on the host; no early stop.
struct PackedLit {
    uint32_t a, span, negate, none;
};

// Registers of one Bit-Packed tile: lane L's w dwords and its incoming-mask dword.
template <int W>
struct PackedTile {
    uint32_t v[W];
    uint32_t in;
};

// Loads of tile t (zeros, and no memory read, when `valid` is false).
template <int W, bool HAS_IN>
__device__ __forceinline__ PackedTile<W> load_packed(const DevCol& c, const uint64_t* __restrict__ in_mask,
                                                     uint64_t t, uint32_t lane, bool valid) {
    PackedTile<W> p;
    const auto r = buffer_rsrc(c.packed + (valid ? t * 64 * W : 0), valid ? 256u * W : 0u);
#pragma unroll
    for (int i = 0; i < W; ++i) p.v[i] = buffer_load4(r, (uint32_t)(i * 64 + lane) * 4);
    p.in = ~0u;
    if (HAS_IN) {
        const uint64_t nd = ((c.n + 63) >> 6) * 2, d0 = t * 64;
        const uint32_t avail = (valid && d0 < nd) ? (uint32_t)(nd - d0 < 64 ? nd - d0 : 64) * 4u : 0u;
        const void* base = avail ? (const void*)(reinterpret_cast<const uint32_t*>(in_mask) + d0) : (const void*)in_mask;
        p.in = buffer_load4(buffer_rsrc(base, avail), lane * 4);
    }
    return p;
}

// One tile: per group the range test's ballot goes into lanes 2k, 2k+1 of the
// result dwords; the incoming mask, the column's end and negation are applied
// lane-parallel before the 256-byte store.
template <int W, bool HAS_IN>
__device__ __forceinline__ void process_packed(const DevCol& c, const PackedLit& pl, uint64_t* __restrict__ out,
                                               uint64_t t, uint64_t t_end, uint32_t lane, const PackedTile<W>& p,
                                               uint64_t& alg) {
    if (t >= t_end) return;
    const uint64_t d = t * 64 + lane;
    const bool full = (t + 1) * kTileRows <= c.n;
    uint32_t actv = p.in;
    if (!full) {
        const uint64_t r0 = d * 32;
        actv &= r0 + 32 <= c.n ? ~0u : (r0 < c.n ? (1u << (c.n - r0)) - 1u : 0u);
    }
    alg += 256 * W + 256 + (HAS_IN ? 256 : 0);
    uint32_t oq[2] = {0, 0};
    if (!pl.none) {
        Unroll<0, 32>::run([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            constexpr uint32_t kMask = (W == 32) ? 0xffffffffu : ((1u << (W & 31)) - 1u);
            constexpr int bit = k * W, i = bit >> 5, sh = bit & 31;
            uint32_t code;
            if constexpr (sh + W <= 32)
                code = (p.v[i] >> sh) & kMask;
            else
                code = __builtin_amdgcn_alignbit(p.v[i + 1], p.v[i], sh) & kMask;
            oq[k & 1] = put_word_at(oq[k & 1], k, ballot(code - pl.a <= pl.span));
        });
    }
    const uint32_t x = oq[0] | oq[1];
    const uint32_t outv = pl.none ? 0u : (pl.negate ? (actv & ~x) : (actv & x));
    if (full || d < ((c.n + 63) >> 6) * 2) reinterpret_cast<uint32_t*>(out)[d] = outv;
}

// Tiles t_begin, t_begin + stride, ... below t_end; two tiles' registers in
// ping-pong, so one tile loads while the other is scanned.
template <int W, bool HAS_IN>
__device__ __forceinline__ void scan_packed_range(const DevCol& c, const PackedLit& pl,
                                                  const uint64_t* __restrict__ in_mask, uint64_t* __restrict__ out,
                                                  uint64_t t_begin, uint64_t t_end, uint64_t stride, uint32_t lane,
                                                  uint64_t& alg) {
    if (t_begin >= t_end) return;
    uint64_t t = t_begin;
    PackedTile<W> a = load_packed<W, HAS_IN>(c, in_mask, t, lane, true);
    PackedTile<W> b = load_packed<W, HAS_IN>(c, in_mask, t + stride, lane, t + stride < t_end);
    const uint64_t mine = (t_end - t_begin + stride - 1) / stride;
    for (uint64_t i = 0; i < mine; i += 2) {
        process_packed<W, HAS_IN>(c, pl, out, t, t_end, lane, a, alg);
        a = load_packed<W, HAS_IN>(c, in_mask, t + 2 * stride, lane, t + 2 * stride < t_end);
        t += stride;
        process_packed<W, HAS_IN>(c, pl, out, t, t_end, lane, b, alg);
        b = load_packed<W, HAS_IN>(c, in_mask, t + 2 * stride, lane, t + 2 * stride < t_end);
        t += stride;
    }
}

// ------------------------------------------------------------ lookup
// Value of one row (Sec. 3.3, lookup): gather the row's bytes, rebuild its
// code, decode it.  PP-VBS finds the position of byte j in BS_j from M_j and the
// directory instead of Algorithm 4's running cursors, so any row can be read on
// its own; the decode tables walk Algorithm 1's tree: a slot ends the code, a
// pointer descends, a leaf turns the remaining bytes into a slot number.
__device__ __forceinline__ uint32_t trie_rank(const DevCol& c, uint64_t code, uint32_t len) {
    uint32_t ch = c.trie_root;
    for (uint32_t j = 1;; ++j) {
        if (ch & kLeafFlag) {
            const uint32_t rest = len - j + 1;
            const uint64_t slot = rest >= 8 ? code : (code & ((1ull << (8 * rest)) - 1));
            return (ch & ~kLeafFlag) + (uint32_t)slot - 1u;
        }
        const uint32_t byte = (uint32_t)(code >> (8 * (len - j))) & 0xffu;
        const uint32_t* e = c.trie + ((uint64_t)ch * 256 + byte) * 2;
        if (j >= len) return e[0];
        ch = e[1];
    }
}

// Frequency rank of a categorical code (Algorithm 2's fill order inverted):
// levels below B are full, 255 * 256^(b-1) codes each, filled pointer-major;
// level B is filled slot-major.
__device__ __forceinline__ uint64_t categorical_rank(uint64_t code, uint32_t len, uint32_t B) {
    uint64_t base = 0;
    for (uint32_t b = 1; b < len; ++b) base += 255ull << (8 * (b - 1));
    const uint64_t slot = code & 0xffu, path = code >> 8;
    if (len < B) return base + path * 255 + (slot - 1);
    return base + (slot - 1) * (1ull << (8 * (B - 1))) + path;
}

__device__ __forceinline__ uint32_t lookup_row(const DevCol& c, uint64_t r) {
    const uint64_t pos1 = (r & ~(uint64_t)(kTileRows - 1)) + ((r & 63) << 5) + ((r >> 6) & 31);
    if (c.layout == BST_PPVBS) {
        uint64_t code = c.bs[1][pos1];
        uint32_t len = 1;
        const uint64_t g = r >> 6;
        const uint64_t below = (1ull << (r & 63)) - 1;
        for (uint32_t j = 2; j <= c.K; ++j) {
            const uint64_t w = c.m[j][g];
            if (!((w >> (r & 63)) & 1)) break;
            const uint64_t off = vbs_group_base(c, j, g) + __builtin_popcountll(w & below);
            code = (code << 8) | c.bs[j][off];
            len = j;
        }
        if (c.categorical) return c.dict[categorical_rank(code, len, c.K)];
        return c.dict[trie_rank(c, code, len)];
    }
    if (c.layout == BST_BYTESLICE) {
        uint64_t v = c.bs[1][pos1];
        for (uint32_t j = 2; j <= c.K; ++j) v = (v << 8) | c.bs[j][pos1];
        const uint32_t code = (uint32_t)(v >> (8 * c.K - c.width));
        return c.domain_mode ? code : c.dict[code];
    }
    const uint32_t w = c.width;
    const uint64_t bit = ((r >> 6) & 31) * w;
    const uint32_t* base = c.packed + (r >> 11) * 64 * w + (r & 63);
    const uint32_t i = (uint32_t)(bit >> 5), sh = (uint32_t)(bit & 31);
    uint64_t win = base[(uint64_t)i * 64];
    if (sh + w > 32) win |= (uint64_t)base[(uint64_t)(i + 1) * 64] << 32;
    const uint32_t code = (uint32_t)((win >> sh) & ((w == 32) ? 0xffffffffull : ((1ull << w) - 1)));
    return c.domain_mode ? code : c.dict[code];
}

// ------------------------------------------------------------ batch
// Many scans in one persistent launch: waves take `grab` tiles at a time from
// a shared counter over the concatenated tile ranges of all items.
struct BatchItem {
    DevCol c;
    ScanLit lit;
    PackedLit pl;
    const uint64_t* in_mask;
    uint64_t* out;
    uint64_t tile0;   // first global tile of this item
    uint32_t kind;    // dispatch code: see batch_kind()
    uint32_t pad;
};

struct BatchHeader {
    uint64_t total_tiles;
    uint32_t n_items;
    uint32_t pad;
};

// Item holding group tile `g` of a batch group: the last item with tile0 <= g.
__device__ __forceinline__ uint32_t batch_find(const BatchItem* __restrict__ items, uint32_t n_items, uint64_t g) {
    uint32_t lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (items[mid].tile0 <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

using BatchKernel = void (*)(const BatchHeader*, const BatchItem*, unsigned long long*, uint32_t);
// Persistent Bit-Packed batch kernel for code width w (nullptr outside 1..32).
BatchKernel batch_packed_kernel(uint32_t w, bool has_in);
// Persistent slice-layout batch kernel for one-byte literals; mi: 0 '<', 1 '>',
// 2 '=', 3 BETWEEN.
BatchKernel batch_short_kernel(int mi, bool dense, bool has_in);


// ------------------------------------------------------------ host helpers
struct DeviceProps {
    int cus = 256;
};
DeviceProps& props();
extern int64_t g_tune[BST_TUNE_NKEYS];

inline int hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) return set_error(BST_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return BST_OK;
}

inline uint32_t tile_grid(uint64_t ntiles, int64_t tuned) {
    uint64_t want = (ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    uint64_t cap = tuned > 0 ? (uint64_t)tuned : (uint64_t)props().cus * 8;
    return (uint32_t)std::max<uint64_t>(1, std::min(want, cap));
}

inline uint32_t elem_grid(uint64_t n) {
    uint64_t want = (n + kBlock - 1) / kBlock;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)props().cus * 16));
}

PackedLit packed_literal(const HostColumn& h, const ScanLit& s);
int launch_slices(const DevCol& c, const ScanLit& lit, const uint64_t* in, uint64_t* out,
                  unsigned long long* counters, hipStream_t st);
int launch_packed(const DevCol& c, const PackedLit& pl, const uint64_t* in, uint64_t* out,
                  unsigned long long* counters, hipStream_t st);
int run_scan(const bst_column* col, const ScanLit& lit, const uint64_t* in, uint64_t* out,
             unsigned long long* counters, hipStream_t st);
uint32_t batch_kind(const bst_column* col, const ScanLit& lit);
int enqueue_fill(uint64_t* out, const uint64_t* in, uint64_t n, int all, hipStream_t st);

}  // namespace dev
}  // namespace bst
