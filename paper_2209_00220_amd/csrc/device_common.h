#pragma once
// Device code shared by the gfx950 kernels of the ByteStore library.
//
// Device layouts (built by host_encode.cpp), all in tiles of 2048 rows:
//  * first byte slice BS_1 (PP-VBS, ByteSlice): in tile t, lane L of a wave owns
//    the 32 rows t*2048 + k*64 + L (k = 0..31), stored as 32 contiguous bytes at
//    t*2048 + L*32.  Two 16-byte loads per lane bring a whole tile in, and byte k
//    of every lane is exactly one 64-row group in row order, so a ballot over a
//    byte compare is one result word.
//  * later slices: ByteSlice BS_j dense in row order; PP-VBS BS_j compacted in
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

// Lanes 2K and 2K+1 of v take the uniform values lo and hi (v_writelane_b32 with
// SGPR data).  The values usually come straight from a VALU compare or
// readfirstlane, and a VALU read of an SGPR that a VALU instruction just wrote
// needs two wait states on this chip; the compiler cannot see into the asm, so
// the s_nop that provides them is part of it.
template <int K>
__device__ __forceinline__ uint32_t put_word(uint32_t v, uint32_t lo, uint32_t hi) {
    uint32_t r;
    const uint32_t slo = __builtin_amdgcn_readfirstlane(lo);
    const uint32_t shi = __builtin_amdgcn_readfirstlane(hi);
    asm("s_nop 1\n\tv_writelane_b32 %0, %1, %3\n\tv_writelane_b32 %0, %2, %4"
                 : "=v"(r)
                 : "s"(slo), "s"(shi), "i"(2 * K), "i"(2 * K + 1), "0"(v));
    return r;
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
// Phase 1 compares byte 1 of all 32 groups (no memory wait, the tile is in
// registers) and records the groups that still have pending rows.  Phase 2
// settles only those groups: M_2 words come from the tile's prefetched mask
// dwords, and the byte-2 gathers of up to four groups are issued before any of
// them is waited on; deeper bytes, rarer still, are read group by group.  So
// later slices are read only for groups whose rows are undecided -- the early
// stop of Algorithm 3 at 64-row granularity, tested wave-uniformly.

// Per-lane registers of one tile.
struct TileData {
    uint4 q0, q1;   // 32 first-slice bytes: byte k is row tile*2048 + 64k + lane
    uint32_t m2;    // PP-VBS: dword `lane` of the tile's 32 M_2 words (0 when unused)
    uint32_t in;    // dword `lane` of the tile's 32 incoming-mask words (all ones when none)
};

template <bool DENSE, bool HAS_IN>
__device__ __forceinline__ TileData load_tile(const DevCol& c, const uint64_t* __restrict__ in_mask, uint64_t t,
                                              uint32_t lane) {
    TileData d;
    const uint4* p = reinterpret_cast<const uint4*>(c.bs[1] + t * kTileRows) + lane * 2;
    d.q0 = p[0];
    d.q1 = p[1];
    d.m2 = 0;
    if (!DENSE && c.K >= 2) d.m2 = reinterpret_cast<const uint32_t*>(c.m[2])[t * 64 + lane];
    d.in = ~0u;
    if (HAS_IN) {
        const uint64_t dd = t * 64 + lane;
        d.in = dd < ((c.n + 63) >> 6) * 2 ? reinterpret_cast<const uint32_t*>(in_mask)[dd] : 0u;
    }
    return d;
}

// 64-bit value held by lanes 2k (low half) and 2k+1 (high half) of v; k uniform.
__device__ __forceinline__ uint64_t lane_word(uint32_t v, uint32_t k) {
    return (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)v, (int)(2 * k)) |
           ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)v, (int)(2 * k + 1)) << 32);
}

// Store the uniform 64-bit value w into lanes 2k and 2k+1 of v; k uniform.
__device__ __forceinline__ uint32_t set_lane_word(uint32_t v, uint32_t k, uint64_t w, uint32_t lane) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)w);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(w >> 32));
    return lane == 2 * k ? lo : (lane == 2 * k + 1 ? hi : v);
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

// 64-bit word held by lanes 2K and 2K+1 of v, K a compile-time constant.
template <int K>
__device__ __forceinline__ uint64_t lane_word_c(uint32_t v) {
    return (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)v, 2 * K) |
           ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)v, 2 * K + 1) << 32);
}

template <int K>
__device__ __forceinline__ uint32_t set_word_c(uint32_t v, uint64_t w) {
    return put_word<K>(v, (uint32_t)w, (uint32_t)(w >> 32));
}

// Inclusive prefix sum over the wave's lanes.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v, uint32_t lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(v, o, 64);
        if ((int)lane >= o) v += y;
    }
    return v;
}

constexpr uint32_t kStageBytes = 2080;   // 130 chunks of 16 bytes: a 2048-byte run plus alignment

// Copy bytes [start, start+len) of a slice into this wave's LDS buffer with
// 16-byte loads from the aligned-down start; returns start's offset in the buffer.
__device__ __forceinline__ uint32_t stage_run(const uint8_t* __restrict__ src, uint64_t start, uint32_t len,
                                              uint8_t* buf, uint32_t lane) {
    const uint64_t a = start & ~15ull;
    const uint64_t end = start + len;
#pragma unroll
    for (uint32_t i = lane; i < kStageBytes / 16; i += 64) {
        const uint64_t p = a + 16ull * i;
        if (p < end) *reinterpret_cast<uint4*>(buf + 16 * i) = *reinterpret_cast<const uint4*>(src + p);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return (uint32_t)(start - a);
}

// One tile, one wave, in two passes.
//
// Pass 1 walks the 32 groups (unrolled, first-slice bytes in registers) and
// settles each group as deep as it can without waiting on memory: byte 1, the
// presence of byte 2 (M_2, prefetched with the tile) and, when the launch
// stages them, bytes 2 and 3 read from this wave's LDS copy of the tile's part
// of BS_2 / BS_3 (one coalesced read each, made before the pass).  The host
// stages a slice when many groups are expected to need it; otherwise pass 1
// leaves those groups pending.
//
// Pass 2 finishes the pending groups byte by byte: with many of them it stages
// the slice in LDS, with few it gathers just their bytes, four groups in
// flight.  Pending rows and results live in VGPR lanes (2k, 2k+1) per group.
template <int MODE, int SHORT, bool DENSE, bool HAS_IN, bool COUNT>
__device__ __forceinline__ void process_tile(const DevCol& c, const ScanLit& lit, uint64_t* __restrict__ out,
                                             uint64_t t, uint32_t lane, const TileData& td, uint8_t* lds,
                                             Stats& st) {
    const uint64_t w0 = t * 32;
    const uint64_t nwords = (c.n + 63) >> 6;
    const uint32_t K = c.K;
    const uint32_t clo = lit_byte(lit.lo, 1), chi = lit_byte(lit.hi, 1);
    const uint32_t c2lo = lit_byte(lit.lo, 2), c2hi = lit_byte(lit.hi, 2);
    const uint32_t c3lo = lit_byte(lit.lo, 3), c3hi = lit_byte(lit.hi, 3);
    const bool negate = lit.negate != 0;
    const uint32_t dw[8] = {td.q0.x, td.q0.y, td.q0.z, td.q0.w, td.q1.x, td.q1.y, td.q1.z, td.q1.w};
    if (COUNT) {
        st.alg += kTileRows + 256 + (HAS_IN ? 256 : 0);
        st.full += full_read_bytes<DENSE>(c, lit, t, HAS_IN);
    }
    // slices staged for pass 1
    const bool s2 = (lit.stage & 1) && K >= 2;
    const bool s3 = s2 && (lit.stage & 2) && K >= 3;
    uint32_t m3v = 0, incl2 = 0, incl3 = 0, sh2 = 0, sh3 = 0;
    uint8_t* lds2 = lds;
    uint8_t* lds3 = lds + kStageBytes;
    if (s2) {
        if (!DENSE && K >= 3) m3v = reinterpret_cast<const uint32_t*>(c.m[3])[t * 64 + lane];
        if (DENSE) {
            sh2 = stage_run(c.bs[2], t * kTileRows, kTileRows, lds2, lane);
        } else {
            incl2 = wave_incl_sum(__builtin_popcount(td.m2), lane);
            sh2 = stage_run(c.bs[2], c.dir[2][(t * kTileRows) >> c.dir_shift],
                            (uint32_t)__builtin_amdgcn_readlane((int)incl2, 63), lds2, lane);
        }
    }
    if (s3) {
        if (DENSE) {
            sh3 = stage_run(c.bs[3], t * kTileRows, kTileRows, lds3, lane);
        } else {
            incl3 = wave_incl_sum(__builtin_popcount(m3v), lane);
            sh3 = stage_run(c.bs[3], c.dir[3][(t * kTileRows) >> c.dir_shift],
                            (uint32_t)__builtin_amdgcn_readlane((int)incl3, 63), lds3, lane);
        }
    }
    uint32_t m4v = 0;
    if (s3 && !DENSE && K >= 4) m4v = reinterpret_cast<const uint32_t*>(c.m[4])[t * 64 + lane];
    // byte 1: SHORT bit 0 (bit 1) says the lower (upper) literal is one byte long
    // (SHORT < 0: decided at run time)
    const uint64_t k1lo = SHORT < 0 ? (1 < lit.llo ? ~0ull : 0ull) : ((SHORT & 1) ? 0ull : ~0ull);
    const uint64_t k1hi = SHORT < 0 ? (1 < lit.lhi ? ~0ull : 0ull) : ((SHORT & 2) ? 0ull : ~0ull);
    // PP-VBS mask dwords are zero past the longest code; ByteSlice rows have all K bytes
    const uint64_t has2 = K >= 2 ? ~0ull : 0ull, has3 = K >= 3 ? ~0ull : 0ull, has4 = K >= 4 ? ~0ull : 0ull;
    // result words of groups k = 0, 1, 2, 3 (mod 4) build up in separate registers
    // (disjoint lanes) so the lane writes of consecutive groups do not chain
    uint32_t outq[4] = {0, 0, 0, 0};
    uint32_t plov = 0, phiv = 0, pend = 0;
    Unroll<0, 32>::run([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        // rows past the column's end (zero padding) are computed like any other and
        // cleared when the tile is stored; the instrumented build masks them here
        uint64_t act = ~0ull;
        if (COUNT) act = valid_mask(w0 + k, c.n);
        if (HAS_IN) act &= lane_word_c<k>(td.in);
        const uint32_t b = (dw[k >> 2] >> (8 * (k & 3))) & 0xffu;
        uint64_t res, plo, phi = 0;
        if (MODE == kModeLT) {
            res = ballot(b < clo) & act;
            plo = ballot(b == clo) & act;
        } else if (MODE == kModeGT) {
            res = ballot(b > clo) & act;
            plo = ballot(b == clo) & act;
        } else if (MODE == kModeEQ) {
            res = 0ull;
            plo = ballot(b == clo) & act;
        } else {
            res = act & ~(ballot(b < clo) | ballot(b > chi));
            plo = ballot(b == clo) & act;
            phi = ballot(b == chi) & act;
        }
        if (COUNT) st.rowbytes += __builtin_popcountll(act);
        if ((plo | phi) != 0) {
            uint64_t hit = 0;
            // the presence of byte 2 settles the rows equal on byte 1 that end here
            const uint64_t m2 = DENSE ? has2 : lane_word_c<k>(td.m2);
            if (COUNT && !DENSE && K >= 2) st.alg += 8;
            level_mask_step<MODE>(plo, phi, hit, m2, k1lo, k1hi);
            if (s2 && (plo | phi) != 0) {
                // byte 2 from LDS (read in every lane; only pending lanes are used)
                uint64_t P = plo | phi;
                const uint32_t off2 =
                    DENSE ? 64 * k + lane
                          : sh2 + (k ? (uint32_t)__builtin_amdgcn_readlane((int)incl2, 2 * k - 1) : 0u) + mbcnt(m2);
                if (COUNT) {
                    st.alg += DENSE ? 64 : __builtin_popcountll(m2);
                    st.rowbytes += __builtin_popcountll(P);
                    st.deep_groups += 1;
                }
                byte_step<MODE>(plo, phi, hit, (uint32_t)lds2[off2], c2lo, c2hi);
                if ((plo | phi) != 0) {
                    const uint64_t m3 = DENSE ? has3 : lane_word_c<k>(m3v);
                    if (COUNT && !DENSE && K >= 3) st.alg += 8;
                    level_mask_step<MODE>(plo, phi, hit, m3, lit.k2lo, lit.k2hi);
                    if (s3 && (plo | phi) != 0) {
                        // byte 3 from LDS
                        P = plo | phi;
                        const uint32_t off3 =
                            DENSE ? 64 * k + lane
                                  : sh3 + (k ? (uint32_t)__builtin_amdgcn_readlane((int)incl3, 2 * k - 1) : 0u) +
                                        mbcnt(m3);
                        if (COUNT) {
                            st.alg += DENSE ? 64 : __builtin_popcountll(m3);
                            st.rowbytes += __builtin_popcountll(P);
                        }
                        byte_step<MODE>(plo, phi, hit, (uint32_t)lds3[off3], c3lo, c3hi);
                        if ((plo | phi) != 0) {
                            const uint64_t m4 = DENSE ? has4 : lane_word_c<k>(m4v);
                            if (COUNT && !DENSE && K >= 4) st.alg += 8;
                            level_mask_step<MODE>(plo, phi, hit, m4, lit.k3lo, lit.k3hi);
                        }
                    }
                }
            }
            res = apply_hit<MODE>(res, hit);
            if ((plo | phi) != 0) {
                pend |= 1u << k;
                plov = set_word_c<k>(plov, plo);
                if (MODE == kModeBetween) phiv = set_word_c<k>(phiv, phi);
            }
        }
        outq[k & 3] = set_word_c<k>(outq[k & 3], res);
    });
    uint32_t outv = outq[0] | outq[1] | outq[2] | outq[3];
    // pass 2: bytes j0, j0+1, ... of the groups still pending
    const uint32_t j0 = s3 ? 4u : (s2 ? 3u : 2u);
    uint32_t cur_mv = 0;   // this lane's dword of the tile's M_j words (PP-VBS)
    if (!DENSE && pend != 0) {
        if (j0 == 2) cur_mv = td.m2;
        else if (j0 == 3) cur_mv = m3v;
        else cur_mv = m4v;
    }
    for (uint32_t j = j0; pend != 0 && j <= K; ++j) {
        uint32_t next_mv = 0;   // M_{j+1}: which rows have a byte after this one
        if (!DENSE && j < K) next_mv = reinterpret_cast<const uint32_t*>(c.m[j + 1])[t * 64 + lane];
        uint32_t incl = 0;
        uint64_t run0;
        if (DENSE) {
            run0 = t * kTileRows;
        } else {
            incl = wave_incl_sum(__builtin_popcount(cur_mv), lane);
            run0 = c.dir[j][(t * kTileRows) >> c.dir_shift];
        }
        const uint32_t cjlo = lit_byte(lit.lo, j), cjhi = lit_byte(lit.hi, j);
        uint32_t pend_next = 0;
        {
            while (pend) {
                uint32_t ks[4];
                uint32_t bb[4];
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
                        const uint64_t P = lane_word(plov, k) | (MODE == kModeBetween ? lane_word(phiv, k) : 0ull);
                        const bool mine = (P >> lane) & 1;
                        if (DENSE) {
                            if (mine) bb[i] = c.bs[j][run0 + 64 * k + lane];
                            if (COUNT) st.alg += 64;
                        } else {
                            const uint64_t mj = lane_word(cur_mv, k);
                            const uint32_t before = k ? (uint32_t)__builtin_amdgcn_readlane((int)incl, (int)(2 * k - 1)) : 0u;
                            if (mine) bb[i] = c.bs[j][run0 + before + mbcnt(mj)];
                            if (COUNT) st.alg += __builtin_popcountll(mj);
                        }
                        if (COUNT) {
                            st.rowbytes += __builtin_popcountll(P);
                            if (j == 2) st.deep_groups += 1;
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
                        if (hit) outv = set_lane_word(outv, k, apply_hit<MODE>(lane_word(outv, k), hit), lane);
                        if ((plo | phi) != 0) {
                            pend_next |= 1u << k;
                            plov = set_lane_word(plov, k, plo, lane);
                            if (MODE == kModeBetween) phiv = set_lane_word(phiv, k, phi, lane);
                        }
                    }
                }
            }
        }
        pend = pend_next;
        cur_mv = next_mv;
    }
    const uint64_t d = w0 * 2 + lane;
    // the rows this lane's result dword may report: selected by the incoming mask and
    // inside the column ('>=', '<=', '!=' complement within them)
    uint32_t actv = td.in;
    const bool full = (t + 1) * kTileRows <= c.n;
    if (!full) {
        const uint64_t r0 = d * 32;
        actv &= r0 + 32 <= c.n ? ~0u : (r0 < c.n ? (1u << (c.n - r0)) - 1u : 0u);
    }
    if (MODE != kModeBetween && negate) outv = actv & ~outv;
    else if (!full) outv &= actv;
    if (full || d < nwords * 2) reinterpret_cast<uint32_t*>(out)[d] = outv;
}

// Load and scan one tile (used by the batched kernel).
template <int MODE, bool DENSE, bool HAS_IN, bool COUNT>
__device__ __forceinline__ void scan_slices_tile(const DevCol& c, const ScanLit& lit,
                                                 const uint64_t* __restrict__ in_mask,
                                                 uint64_t* __restrict__ out, uint64_t t, uint32_t lane,
                                                 uint8_t* lds, Stats& st) {
    const TileData td = load_tile<DENSE, HAS_IN>(c, in_mask, t, lane);
    process_tile<MODE, -1, DENSE, HAS_IN, COUNT>(c, lit, out, t, lane, td, lds, st);
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

template <int W, bool HAS_IN>
__device__ __forceinline__ void scan_packed_tile(const DevCol& c, const PackedLit& pl,
                                                 const uint64_t* __restrict__ in_mask,
                                                 uint64_t* __restrict__ out, uint64_t t, uint32_t lane,
                                                 uint64_t& alg) {
    const uint64_t w0 = t * 32;
    uint32_t* out32 = reinterpret_cast<uint32_t*>(out);
    const uint64_t nwords = (c.n + 63) >> 6;
    if (HAS_IN) {
        const uint64_t d = w0 * 2 + lane;
        const uint32_t mine = d < nwords * 2 ? reinterpret_cast<const uint32_t*>(in_mask)[d] : 0u;
        if (ballot(mine != 0) == 0) {
            if (d < nwords * 2) out32[d] = 0;
            alg += 512;
            return;
        }
    }
    const uint32_t* base = c.packed + t * 64 * W + lane;
    uint32_t v[W];
#pragma unroll
    for (int i = 0; i < W; ++i) v[i] = base[i * 64];
    alg += 256 * W + 256 + (HAS_IN ? 256 : 0);
    uint32_t outv = 0;
    Unroll<0, 32>::run([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr uint32_t kMask = (W == 32) ? 0xffffffffu : ((1u << (W & 31)) - 1u);
        constexpr int bit = k * W, i = bit >> 5, sh = bit & 31;
        uint32_t code;
        if constexpr (sh + W <= 32)
            code = (v[i] >> sh) & kMask;
        else
            code = __builtin_amdgcn_alignbit(v[i + 1], v[i], sh) & kMask;
        const uint64_t g = w0 + k;
        uint64_t act = valid_mask(g, c.n);
        if (HAS_IN) act &= (g < nwords) ? in_mask[g] : 0ull;
        const uint64_t X = ballot(code - pl.a <= pl.span);
        const uint64_t res = pl.none ? 0ull : (pl.negate ? (act & ~X) : (act & X));
        outv = put_word<k>(outv, (uint32_t)res, (uint32_t)(res >> 32));
    });
    const uint64_t d = w0 * 2 + lane;
    if (d < nwords * 2) out32[d] = outv;
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
        return c.dict[trie_rank(c, code, len)];
    }
    if (c.layout == BST_BYTESLICE) {
        uint64_t v = c.bs[1][pos1];
        for (uint32_t j = 2; j <= c.K; ++j) v = (v << 8) | c.bs[j][r];
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
    uint32_t kind;    // dispatch code, see batch_kind()
    uint32_t pad;
};

struct BatchHeader {
    uint64_t total_tiles;
    uint32_t n_items;
    uint32_t pad;
};


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
