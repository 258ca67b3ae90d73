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

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// number of set bits of m below this lane
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// v_writelane_b32: lane LANE of the VGPR takes the uniform value v (an SGPR)
template <int LANE>
__device__ __forceinline__ uint32_t put_lane(uint32_t old, uint32_t v) {
    uint32_t r;
    const uint32_t s = __builtin_amdgcn_readfirstlane(v);
    asm("v_writelane_b32 %0, %1, %2" : "=v"(r) : "s"(s), "i"(LANE), "0"(old));
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
// Classify one 64-row group against a literal byte by byte (Sec. 3.3,
// Algorithm 3 generalised to every operator).  A row stays pending while its
// bytes equal the literal's; at byte j < l a pending row without a (j+1)-th
// byte is a proper prefix of the literal, hence smaller (the literal's rest is
// not all zero); at j = l a pending row is greater if it has byte l+1, else
// equal.  Bytes are compared unsigned.  The group stops as soon as no row is
// pending (a wave-uniform test), so later slices are only read for the rows
// still undecided.
//
// MODE kModeLT: returns rows with code < lit; kModeGT: code > lit;
// kModeEQ: code == lit.  Rows outside `act` are never reported.
template <int MODE, bool DENSE, bool COUNT>
__device__ __forceinline__ uint64_t classify_one(const DevCol& c, uint64_t lit6, uint32_t l, uint32_t b1,
                                                 uint64_t act, uint64_t g, uint32_t lane, Stats& st) {
    uint32_t cb = lit_byte(lit6, 1);
    uint64_t X = 0;
    uint64_t P = ballot(b1 == cb) & act;
    if (MODE == kModeLT) X = ballot(b1 < cb) & act;
    if (MODE == kModeGT) X = ballot(b1 > cb) & act;
    if (COUNT) st.rowbytes += __builtin_popcountll(act);
    const uint32_t K = c.K;
    bool deep = false;
    for (uint32_t j = 1; P != 0; ++j) {
        uint64_t mnext;
        if (j >= K) {
            mnext = 0;
        } else if (DENSE) {
            mnext = ~0ull;
        } else {
            mnext = c.m[j + 1][g];
            if (COUNT) st.alg += 8;
        }
        if (j >= l) {
            if (MODE == kModeGT) X |= P & mnext;
            if (MODE == kModeEQ) X |= P & ~mnext;
            break;
        }
        if (MODE == kModeLT) X |= P & ~mnext;
        P &= mnext;
        if (P == 0) break;
        // byte j+1 of the pending rows
        uint32_t bb = 0;
        const bool mine = (P >> lane) & 1;
        if (DENSE) {
            if (mine) bb = c.bs[j + 1][(g << 6) + lane];
            if (COUNT) st.alg += 64;
        } else {
            const uint64_t base = vbs_group_base(c, j + 1, g);
            if (mine) bb = c.bs[j + 1][base + mbcnt(mnext)];
            if (COUNT) st.alg += __builtin_popcountll(mnext);
        }
        if (COUNT) {
            st.rowbytes += __builtin_popcountll(P);
            deep = true;
        }
        cb = lit_byte(lit6, j + 1);
        const uint64_t lt = ballot(bb < cb) & P;
        const uint64_t gt = ballot(bb > cb) & P;
        const uint64_t eq = ballot(bb == cb) & P;
        if (MODE == kModeLT) X |= lt;
        if (MODE == kModeGT) X |= gt;
        (void)gt;
        (void)lt;
        P = eq;
    }
    if (COUNT && deep) st.deep_groups += 1;
    return X;
}

// BETWEEN: rows with lo <= code <= hi, both literals classified in one pass.
template <bool DENSE, bool COUNT>
__device__ __forceinline__ uint64_t classify_between(const DevCol& c, const ScanLit& lit, uint32_t b1,
                                                     uint64_t act, uint64_t g, uint32_t lane, Stats& st) {
    uint32_t clo = lit_byte(lit.lo, 1), chi = lit_byte(lit.hi, 1);
    uint64_t below = ballot(b1 < clo) & act;   // code < lo
    uint64_t above = ballot(b1 > chi) & act;   // code > hi
    uint64_t Plo = ballot(b1 == clo) & act;
    uint64_t Phi = ballot(b1 == chi) & act;
    if (COUNT) st.rowbytes += __builtin_popcountll(act);
    const uint32_t K = c.K;
    bool deep = false;
    for (uint32_t j = 1; (Plo | Phi) != 0; ++j) {
        uint64_t mnext;
        if (j >= K) {
            mnext = 0;
        } else if (DENSE) {
            mnext = ~0ull;
        } else {
            mnext = c.m[j + 1][g];
            if (COUNT) st.alg += 8;
        }
        if (j >= lit.llo) {
            Plo = 0;   // equal to lo or longer: not below lo
        } else {
            below |= Plo & ~mnext;
            Plo &= mnext;
        }
        if (j >= lit.lhi) {
            above |= Phi & mnext;
            Phi = 0;
        } else {
            Phi &= mnext;   // a proper prefix of hi is below hi
        }
        const uint64_t P = Plo | Phi;
        if (P == 0) break;
        uint32_t bb = 0;
        const bool mine = (P >> lane) & 1;
        if (DENSE) {
            if (mine) bb = c.bs[j + 1][(g << 6) + lane];
            if (COUNT) st.alg += 64;
        } else {
            const uint64_t base = vbs_group_base(c, j + 1, g);
            if (mine) bb = c.bs[j + 1][base + mbcnt(mnext)];
            if (COUNT) st.alg += __builtin_popcountll(mnext);
        }
        if (COUNT) {
            st.rowbytes += __builtin_popcountll(P);
            deep = true;
        }
        clo = lit_byte(lit.lo, j + 1);
        chi = lit_byte(lit.hi, j + 1);
        below |= ballot(bb < clo) & Plo;
        above |= ballot(bb > chi) & Phi;
        Plo = ballot(bb == clo) & Plo;
        Phi = ballot(bb == chi) & Phi;
    }
    if (COUNT && deep) st.deep_groups += 1;
    return act & ~below & ~above;
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

// One tile of a slice-layout scan, done by one wave.
template <int MODE, bool DENSE, bool HAS_IN, bool COUNT>
__device__ __forceinline__ void scan_slices_tile(const DevCol& c, const ScanLit& lit,
                                                 const uint64_t* __restrict__ in_mask,
                                                 uint64_t* __restrict__ out, uint64_t t, uint32_t lane,
                                                 Stats& st) {
    const uint64_t w0 = t * 32;
    uint32_t* out32 = reinterpret_cast<uint32_t*>(out);
    const uint64_t nwords = (c.n + 63) >> 6;
    if (HAS_IN) {
        // a tile whose incoming mask is all zero is not read at all
        const uint64_t d = w0 * 2 + lane;
        const uint32_t mine = d < nwords * 2 ? reinterpret_cast<const uint32_t*>(in_mask)[d] : 0u;
        if (ballot(mine != 0) == 0) {
            if (d < nwords * 2) out32[d] = 0;
            if (COUNT) st.alg += 256 + 256;
            return;
        }
    }
    const uint4* p = reinterpret_cast<const uint4*>(c.bs[1] + t * kTileRows) + lane * 2;
    const uint4 q0 = p[0], q1 = p[1];
    const uint32_t dw[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
    if (COUNT) {
        st.alg += kTileRows + 256 + (HAS_IN ? 256 : 0);
        st.full += full_read_bytes<DENSE>(c, lit, t, HAS_IN);
    }
    uint32_t outv = 0;
    Unroll<0, 32>::run([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const uint64_t g = w0 + k;
        uint64_t act = valid_mask(g, c.n);
        if (HAS_IN) act &= (g < nwords) ? in_mask[g] : 0ull;
        uint64_t res = 0;
        if (act != 0) {
            const uint32_t b1 = (dw[k >> 2] >> (8 * (k & 3))) & 0xffu;
            if (MODE == kModeBetween) {
                res = classify_between<DENSE, COUNT>(c, lit, b1, act, g, lane, st);
            } else {
                const uint64_t X = classify_one<MODE, DENSE, COUNT>(c, lit.lo, lit.llo, b1, act, g, lane, st);
                res = lit.negate ? (act & ~X) : X;
            }
        }
        outv = put_lane<2 * k>(outv, (uint32_t)res);
        outv = put_lane<2 * k + 1>(outv, (uint32_t)(res >> 32));
    });
    const uint64_t d = w0 * 2 + lane;
    if (d < nwords * 2) out32[d] = outv;
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
        outv = put_lane<2 * k>(outv, (uint32_t)res);
        outv = put_lane<2 * k + 1>(outv, (uint32_t)(res >> 32));
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
