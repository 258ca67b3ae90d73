#pragma once
// Device code shared by the gfx950 kernels of the ByteStore library.
//
// Device layouts (built by host_encode.cpp), all in tiles of 2048 rows:
//  * tile-interleaved slices (BS_1 of PP-VBS and ByteSlice): lane L of a wave
//    owns the 32 consecutive rows t*2048 + 32L + p (p = 0..31) of tile t, held
//    as eight dwords; row p is byte p / 8 of dword p % 8, dwords 0-3 at
//    t*2048 + 16L and dwords 4-7 at t*2048 + 1024 + 16L (slice_pos()).  Two
//    16-byte loads per lane bring a tile in, each covering 1 KB contiguously,
//    and a lane's 32 outcome bits form its result dword.
//  * ByteSlice slices after the first: the same eight dwords per lane, stored
//    contiguously at t*2048 + 32L (lane_slice_pos()), since only lanes with
//    rows still pending read them.
//  * PP-VBS BS_j (j >= 2) compacted in row order (only rows with a j-th byte),
//    bitmask M_j one uint64 per 64 rows, directory DIR_j = running count of
//    j-th bytes every 2^dir_shift rows.
//  * Bit-Packed: in tile t, lane L's 32 codes (rows t*2048 + 64k + L) packed
//    LSB first into w dwords; dword i of lane L at t*64*w + i*64 + L.
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

// Inclusive prefix sum over the wave's lanes: DPP row shifts within each
// 16-lane row, then row broadcasts across rows (lanes without a source add 0).
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v) {
    constexpr int kRowShr = 0x110, kRowBcast15 = 0x142, kRowBcast31 = 0x143;
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowShr + 1, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowShr + 2, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowShr + 4, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowShr + 8, 0xf, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowBcast15, 0xa, 0xf, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kRowBcast31, 0xc, 0xf, false);
    return v;
}

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

// Byte offset of row r in a tile-interleaved slice.
__device__ __forceinline__ uint64_t slice_pos(uint64_t r) {
    const uint32_t p = (uint32_t)r & 31, lane = (uint32_t)(r >> 5) & 63, i = p & 7;
    return (r & ~(uint64_t)(kTileRows - 1)) + (i >> 2) * 1024 + lane * 16 + (i & 3) * 4 + (p >> 3);
}

// Byte offset of row r in a ByteSlice slice after the first: the same rows per
// lane and bytes per dword, each lane's 32 bytes contiguous at 32L.
__device__ __forceinline__ uint64_t lane_slice_pos(uint64_t r) {
    const uint32_t p = (uint32_t)r & 31, lane = (uint32_t)(r >> 5) & 63;
    return (r & ~(uint64_t)(kTileRows - 1)) + lane * 32 + (p & 7) * 4 + (p >> 3);
}

struct Stats {
    uint64_t alg = 0, rowbytes = 0, deep_groups = 0, full = 0;
    uint64_t lines = 0;   // 128-byte lines holding the algorithmic bytes (each counted once)
};

// M_j word of 64-row group g (PP-VBS), and in `before` the j-th bytes of the
// groups before g in its directory block (the position of g's first j-th byte
// is the block's directory entry plus `before`).  A block of up to 8 words is
// one aligned 64-byte run, read with independent 16-byte loads, so the mask
// and the walk cost one round trip together, in the line the mask needs anyway.
__device__ __forceinline__ uint64_t vbs_word(const DevCol& c, uint32_t j, uint64_t g, uint64_t& before) {
    const uint32_t lw = c.dir_shift - 6;   // log2 of the M_j words per directory block
    const uint64_t b0 = (g >> lw) << lw;
    const uint32_t k = (uint32_t)(g - b0);
    const uint64_t* m = c.m[j] + b0;
    before = 0;
    if (lw == 0 || lw > 3) {
        for (uint32_t i = 0; i < k; ++i) before += __builtin_popcountll(m[i]);
        return m[k];
    }
    const uint32_t pairs = 1u << (lw - 1);   // 16-byte pairs in the block: 1, 2 or 4
    const ulonglong2* p = reinterpret_cast<const ulonglong2*>(m);
    ulonglong2 v[4];
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
        if (i < pairs) v[i] = p[i];
        else v[i] = make_ulonglong2(0, 0);
    }
    uint64_t w = 0;
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
        if (2 * i < k) before += __builtin_popcountll(v[i].x);
        if (2 * i + 1 < k) before += __builtin_popcountll(v[i].y);
        if (2 * i == k) w = v[i].x;
        if (2 * i + 1 == k) w = v[i].y;
    }
    return w;
}

// ------------------------------------------------------------ raw buffer access
// gfx9-family descriptor: no format, no swizzle.  A buffer load past
// num_records returns zeros without touching memory, so loads can be issued
// unconditionally: the hardware's in-order count of pending loads then matches
// the program order, and the compiler can wait for one tile's data while the
// next tiles' loads stay in flight.
//
// Streamed data (slices, masks, directories, incoming masks, packed words) is
// read with the non-temporal cache policy: a scan reads each byte once, and
// letting those reads allocate normally in the caches slows the whole stream
// down once result stores are interleaved with it (measured on this chip:
// 5.5-5.7 TB/s of reads with non-temporal loads against 4.4-4.7 TB/s without).
// Result words are stored non-temporally for the same reason.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kRawBufferWord3 = 0x00020000;
constexpr int kStream = 2;   // cache-policy operand of a buffer load: non-temporal

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRawBufferWord3);
}

__device__ __forceinline__ uint4 buffer_load16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, kStream);
    return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ uint32_t buffer_load4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, kStream);
}

// One dword of a result bitvector, stored non-temporally.
__device__ __forceinline__ void store_result_dword(uint64_t* out, uint64_t d, uint32_t v) {
    __builtin_nontemporal_store(v, reinterpret_cast<uint32_t*>(out) + d);
}

__device__ __forceinline__ void flush_stats(unsigned long long* counters, const Stats& st, uint32_t lane) {
    if (lane == 0) {
        atomicAdd(counters + 0, (unsigned long long)st.alg);
        atomicAdd(counters + 1, (unsigned long long)st.rowbytes);
        atomicAdd(counters + 2, (unsigned long long)st.deep_groups);
        atomicAdd(counters + 3, (unsigned long long)st.full);
        atomicAdd(counters + 4, (unsigned long long)(st.lines * 128));
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
    if (full || d < ((c.n + 63) >> 6) * 2) store_result_dword(out, d, outv);
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
// its own; the decode tables walk Algorithm 1's tree: a slot ends the code (and
// holds its value), a pointer descends, a leaf turns the remaining bytes into a
// slot number (a rank into the dictionary).
// Base rank of a leaf entry (its low bits; the slot digits, when stored, sit above).
__device__ __forceinline__ uint32_t leaf_base(const DevCol& c, uint32_t ch) {
    return ch & (c.leaf_digits ? ((1u << kLeafDigitsShift) - 1u) : ~kLeafFlag);
}

__device__ __forceinline__ uint32_t trie_value(const DevCol& c, uint64_t code, uint32_t len) {
    uint32_t ch = c.trie_root;
    for (uint32_t j = 1;; ++j) {
        if (ch & kLeafFlag) {   // a leaf: the remaining bytes number a slot of consecutive ranks
            const uint32_t rest = len - j + 1;
            const uint64_t slot = rest >= 8 ? code : (code & ((1ull << (8 * rest)) - 1));
            return c.dict[leaf_base(c, ch) + (uint32_t)slot - 1u];
        }
        const uint32_t byte = (uint32_t)(code >> (8 * (len - j))) & 0xffu;
        const uint32_t* e = c.trie + ((uint64_t)ch * 256 + byte) * 2;
        if (j >= len) return e[0];   // the code ends in this slot: its value
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
    const uint64_t pos1 = slice_pos(r);
    if (c.layout == BST_PPVBS) {
        uint64_t code = c.bs[1][pos1];
        uint32_t len = 1;
        const uint64_t g = r >> 6;
        const uint64_t below = (1ull << (r & 63)) - 1;
        const uint32_t lw = c.dir_shift - 6;
        // Once the code's prefix leads into a leaf of the decode trie, the leaf's
        // slot digits give the code's length, and the mask that would show the
        // code ends (M_{L+1}) need not be read.  `node`: the trie node of the next
        // digit to consume (a leaf entry once known), `known`: the length, or 0.
        const bool guided = c.leaf_digits && !c.categorical;
        uint32_t node = c.trie_root, known = 0;
        if (guided && (node & kLeafFlag)) known = (node >> kLeafDigitsShift) & 7u;
        for (uint32_t j = 2; j <= c.K; ++j) {
            if (known && j > known) break;
            uint64_t before;
            const uint64_t w = vbs_word(c, j, g, before);
            if (!((w >> (r & 63)) & 1)) break;
            if (guided && !known) {
                // the code goes on past byte j - 1: follow that digit's child
                node = c.trie[((uint64_t)node * 256 + (uint32_t)(code & 0xffu)) * 2 + 1];
                if (node & kLeafFlag) known = (j - 1) + ((node >> kLeafDigitsShift) & 7u);
            }
            const uint64_t off = c.dir[j][g >> lw] + before + __builtin_popcountll(w & below);
            code = (code << 8) | c.bs[j][off];
            len = j;
        }
        if (c.categorical) return c.dict[categorical_rank(code, len, c.K)];
        if (guided) {
            // the walk above already reached the code's last node: a leaf turns
            // its slot digits into a dictionary rank, an internal node's slot
            // entry holds the value
            if (node & kLeafFlag) {
                const uint32_t beta = (node >> kLeafDigitsShift) & 7u;
                const uint64_t slot = code & ((1ull << (8 * beta)) - 1);
                return c.dict[leaf_base(c, node) + (uint32_t)slot - 1u];
            }
            return c.trie[((uint64_t)node * 256 + (uint32_t)(code & 0xffu)) * 2];
        }
        return trie_value(c, code, len);
    }
    if (c.layout == BST_BYTESLICE) {
        uint64_t v = c.bs[1][pos1];
        const uint64_t posj = lane_slice_pos(r);
        for (uint32_t j = 2; j <= c.K; ++j) v = (v << 8) | c.bs[j][posj];
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

// Workgroups of a tile-parallel launch: one wave per tile up to `per_cu`
// workgroups per CU (or the tuned count).  Few resident waves keep the number of
// concurrent HBM streams low, which this chip serves faster: the slice scans
// measured best at 3 workgroups (12 waves) per CU, Bit-Packed at 2.
inline uint32_t tile_grid(uint64_t ntiles, int64_t tuned, uint32_t per_cu = 3) {
    uint64_t want = (ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    uint64_t cap = tuned > 0 ? (uint64_t)tuned : (uint64_t)props().cus * per_cu;
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
uint32_t lookup_grid(uint64_t m);
int enqueue_fill(uint64_t* out, const uint64_t* in, uint64_t n, int all, hipStream_t st);

}  // namespace dev
}  // namespace bst
