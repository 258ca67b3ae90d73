// Fills, bitvector helpers, compaction, lookup, the advisor's timing loop and
// the device half of the C ABI.
#include <mutex>
#include <vector>

#include "device_common.h"

using namespace bst;
using namespace bst::dev;

namespace bst {
namespace dev {

// ------------------------------------------------------------ fills
// ALL / NONE predicates: out = (in_mask or every row) / 0.
__global__ __launch_bounds__(kBlock) void k_fill(uint64_t* __restrict__ out, const uint64_t* __restrict__ in_mask,
                                                 uint64_t n, int all) {
    const uint64_t nwords = (n + 63) >> 6;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t v = all ? valid_mask(w, n) : 0ull;
        if (all && in_mask) v &= in_mask[w];
        out[w] = v;
    }
}

__global__ __launch_bounds__(kBlock) void k_bv_binop(const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                                                     uint64_t* __restrict__ out, uint64_t n, int op) {
    const uint64_t nwords = (n + 63) >> 6;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += (uint64_t)gridDim.x * blockDim.x) {
        // 0: a AND b, 1: a OR b, 2: a AND NOT b, 3: NOT a (b unused)
        uint64_t v = op == 0 ? (a[w] & b[w]) : op == 1 ? (a[w] | b[w]) : op == 2 ? (a[w] & ~b[w]) : ~a[w];
        out[w] = v & valid_mask(w, n);
    }
}

__global__ void k_zero_u64(unsigned long long* p, int count) {
    if ((int)threadIdx.x < count) p[threadIdx.x] = 0;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// The traffic of a scan that settles every row on its first byte, without the
// compares: a wave reads 2048-byte tiles (two 16-byte loads per lane, the
// layout and cache policy of BS_1), the next tile's loads in flight while the
// current one is folded, and stores one dword per lane (the tile's 256-byte
// result) non-temporally; grid-stride over the tiles with the scans' launch
// shape.
__global__ __launch_bounds__(kBlock) void k_stream_probe(const uint8_t* __restrict__ src, uint64_t ntiles,
                                                         uint32_t* __restrict__ dst) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t wave = uniform(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
    const uint64_t nwaves = (uint64_t)gridDim.x * kWavesPerBlock;
    auto load = [&](uint64_t t, uint4& a, uint4& b) {
        // a tile past the end reads as zeros (an empty buffer range)
        const auto r = buffer_rsrc(src + (t < ntiles ? t : 0) * kTileRows, t < ntiles ? (uint32_t)kTileRows : 0u);
        a = buffer_load16(r, lane * 16);
        b = buffer_load16(r, 1024 + lane * 16);
    };
    uint4 a, b;
    load(wave, a, b);
    for (uint64_t t = wave; t < ntiles; t += nwaves) {
        uint4 na, nb;
        load(t + nwaves, na, nb);
        const uint32_t v = a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w;
        __builtin_nontemporal_store(v, dst + t * 64 + lane);
        a = na;
        b = nb;
    }
}

// Rows of dword d of a bitvector (rows 32d .. 32d+31) that lie inside an
// n-row column.
__device__ __forceinline__ uint32_t dword_rows(uint64_t d, uint64_t n) {
    const uint64_t r0 = d * 32;
    return r0 + 32 <= n ? ~0u : (r0 < n ? (1u << (uint32_t)(n - r0)) - 1u : 0u);
}

// Dwords d .. d+3 of a bitvector of ndw dwords (zeros past its end), with the
// default cache policy: the compaction reads the bitvector twice, and its
// second pass finds it in the caches.  A quad that runs past the end is read a
// dword at a time, so that the range check of the buffer descriptor applies
// to each dword.
__device__ __forceinline__ uint4 load_quad(__amdgpu_buffer_rsrc_t r, uint64_t d, uint64_t ndw) {
    if (d + 4 <= ndw) {
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)(d * 4), 0, 0);
        return make_uint4(v.x, v.y, v.z, v.w);
    }
    if (d >= ndw) return make_uint4(0u, 0u, 0u, 0u);
    const int o = (int)(d * 4);
    return make_uint4(__builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0), __builtin_amdgcn_raw_buffer_load_b32(r, o + 4, 0, 0),
                      __builtin_amdgcn_raw_buffer_load_b32(r, o + 8, 0, 0),
                      __builtin_amdgcn_raw_buffer_load_b32(r, o + 12, 0, 0));
}

__device__ __forceinline__ uint32_t quad_popc(const uint4& v, uint64_t d, uint64_t n) {
    return (uint32_t)(__builtin_popcount(v.x & dword_rows(d, n)) + __builtin_popcount(v.y & dword_rows(d + 1, n)) +
                      __builtin_popcount(v.z & dword_rows(d + 2, n)) + __builtin_popcount(v.w & dword_rows(d + 3, n)));
}

// Set bits of an n-row bitvector: 16-byte loads, four in flight per thread.
__global__ __launch_bounds__(kBlock) void k_bv_popcount(const uint64_t* __restrict__ bv, uint64_t n,
                                                        unsigned long long* __restrict__ count) {
    __shared__ uint32_t part[kWavesPerBlock];
    const uint64_t ndw = ((n + 63) >> 6) * 2;   // dwords of the bitvector
    const auto r = buffer_rsrc(bv, (uint32_t)(ndw * 4));
    const uint64_t nq = (ndw + 3) / 4;          // its 16-byte quads
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t s = 0;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += 4 * stride) {
        uint4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = load_quad(r, (q + k * stride) * 4, ndw);
#pragma unroll
        for (int k = 0; k < 4; ++k) s += quad_popc(v[k], (q + k * stride) * 4, n);
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    // one atomic per block: same-address atomics serialise
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int i = 0; i < kWavesPerBlock; ++i) t += part[i];
        if (t) atomicAdd(count, (unsigned long long)t);
    }
}

// ------------------------------------------------------------ compaction
// Ascending row IDs of the set bits in three launches: every wave counts the
// set bits of one chunk of kChunkTiles consecutive 2048-row tiles, one
// workgroup turns the chunk counts into exclusive offsets (and the total),
// then every wave reads its chunk again and writes the IDs from its offset.
// The chunk counts are the only workspace.  The counting pass reads a quad of
// dwords per lane (16 lanes per tile), so one load instruction of a wave
// covers four tiles; the writing pass finds the bitvector in the caches.
constexpr uint32_t kChunkTiles = 64;
constexpr uint32_t kChunkLoads = 4;   // load instructions in flight per wave (16 tiles)
constexpr uint32_t kScanBlock = 1024;

__device__ __forceinline__ uint32_t quad_rows_popc(const uint4& v, uint64_t d, uint64_t n, uint4& m) {
    m = make_uint4(v.x & dword_rows(d, n), v.y & dword_rows(d + 1, n), v.z & dword_rows(d + 2, n),
                   v.w & dword_rows(d + 3, n));
    return (uint32_t)(__builtin_popcount(m.x) + __builtin_popcount(m.y) + __builtin_popcount(m.z) +
                      __builtin_popcount(m.w));
}

// First dword of the quad lane `lane` reads at step `s` of chunk `w`.
__device__ __forceinline__ uint64_t chunk_quad(uint64_t w, uint32_t s, uint32_t lane) {
    return ((uint64_t)w * kChunkTiles + 4 * s + (lane >> 4)) * 64 + (lane & 15) * 4;
}

__global__ __launch_bounds__(kBlock) void k_chunk_popc(const uint64_t* __restrict__ bv, uint64_t n, uint64_t nchunks,
                                                       uint64_t* __restrict__ chunk_counts) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t w = uniform(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
    if (w >= nchunks) return;
    const uint64_t ndw = ((n + 63) >> 6) * 2;
    const auto r = buffer_rsrc(bv, (uint32_t)(ndw * 4));
    uint32_t c = 0;
    for (uint32_t s = 0; s < kChunkTiles / 4; s += kChunkLoads) {
        uint4 v[kChunkLoads];
#pragma unroll
        for (uint32_t k = 0; k < kChunkLoads; ++k) v[k] = load_quad(r, chunk_quad(w, s + k, lane), ndw);
#pragma unroll
        for (uint32_t k = 0; k < kChunkLoads; ++k) {
            uint4 m;
            c += quad_rows_popc(v[k], chunk_quad(w, s + k, lane), n, m);
        }
    }
    c = wave_sum(c);
    if (lane == 0) chunk_counts[w] = c;
}

// Exclusive scan of v over the workgroup (kScanBlock threads); *total gets the sum.
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t* part, uint64_t* total) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(incl, o, 64);
        if ((int)lane >= o) incl += y;
    }
    if (lane == 63) part[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        uint64_t p = lane < kScanBlock / 64 ? part[lane] : 0;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            const uint64_t y = __shfl_up(p, o, 64);
            if ((int)lane >= o) p += y;
        }
        if (lane < kScanBlock / 64) part[lane] = p;   // inclusive over waves
    }
    __syncthreads();
    const uint64_t before = wave ? part[wave - 1] : 0;
    *total = part[kScanBlock / 64 - 1];
    return before + incl - v;
}

// In-place exclusive scan of the chunk counts by one workgroup (each thread
// takes a run of consecutive counts); the total goes to *total_out.
__global__ __launch_bounds__(kScanBlock) void k_scan_chunks(uint64_t* __restrict__ cc, uint64_t nchunks,
                                                            unsigned long long* __restrict__ total_out) {
    __shared__ uint64_t part[kScanBlock / 64];
    const uint64_t per = (nchunks + kScanBlock - 1) / kScanBlock;
    const uint64_t b = threadIdx.x * per, e = std::min<uint64_t>(nchunks, b + per);
    uint64_t sum = 0;
    for (uint64_t i = b; i < e; ++i) sum += cc[i];
    uint64_t total;
    uint64_t run = block_excl_scan(sum, part, &total);
    for (uint64_t i = b; i < e; ++i) {
        const uint64_t v = cc[i];
        cc[i] = run;
        run += v;
    }
    if (threadIdx.x == 0) *total_out = total;
}

// The writes go a tile at a time, lane L taking dword L of the tile (its 32
// rows), so the IDs one store instruction writes fall within the tile's run;
// sixteen tiles' dwords are loaded at once.
constexpr uint32_t kWriteTilesPerLoad = 16;

__global__ __launch_bounds__(kBlock) void k_write_ids(const uint64_t* __restrict__ bv, uint64_t n, uint64_t nchunks,
                                                      const uint64_t* __restrict__ chunk_offsets,
                                                      uint32_t* __restrict__ ids, uint64_t cap,
                                                      uint32_t* __restrict__ status) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t w = uniform(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
    if (w >= nchunks) return;
    const uint64_t ndw = ((n + 63) >> 6) * 2;
    const auto r = buffer_rsrc(bv, (uint32_t)(ndw * 4));
    uint64_t base = chunk_offsets[w];   // the IDs of the chunk's earlier tiles end here
    bool over = false;
    for (uint32_t t0 = 0; t0 < kChunkTiles; t0 += kWriteTilesPerLoad) {
        uint32_t v[kWriteTilesPerLoad];
#pragma unroll
        for (uint32_t k = 0; k < kWriteTilesPerLoad; ++k) {
            const uint64_t d = ((uint64_t)w * kChunkTiles + t0 + k) * 64 + lane;
            v[k] = d < ndw ? __builtin_amdgcn_raw_buffer_load_b32(r, (int)(d * 4), 0, 0) : 0u;
        }
#pragma unroll
        for (uint32_t k = 0; k < kWriteTilesPerLoad; ++k) {
            const uint64_t d = ((uint64_t)w * kChunkTiles + t0 + k) * 64 + lane;
            uint32_t bits = v[k] & dword_rows(d, n);
            const uint32_t c = (uint32_t)__builtin_popcount(bits);
            const uint32_t incl = wave_incl_sum(c);
            uint64_t pos = base + (incl - c);
            const uint32_t row0 = (uint32_t)(d * 32);
            while (bits) {
                const uint32_t b = __builtin_ctz(bits);
                bits &= bits - 1;
                if (pos < cap) ids[pos] = row0 + b; else over = true;
                ++pos;
            }
            base += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        }
    }
    if (over && status) atomicOr(status, BST_DEV_OVERFLOW);
}


// all_or_none: with a device count above cap, look up nothing and flag the overflow
__global__ __launch_bounds__(kBlock) void k_lookup(const DevCol c, const uint32_t* __restrict__ ids, uint64_t m,
                                                   const unsigned long long* __restrict__ dev_m, uint64_t cap,
                                                   uint32_t* __restrict__ out, uint32_t* __restrict__ status,
                                                   int all_or_none) {
    uint64_t cnt = m;
    if (dev_m) {
        const uint64_t dm = (uint64_t)*dev_m;
        if (all_or_none && dm > cap) {
            if (status && blockIdx.x == 0 && threadIdx.x == 0) atomicOr(status, BST_DEV_OVERFLOW);
            return;
        }
        cnt = std::min<uint64_t>(dm, cap);
    }
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t r = ids[i];
        if (r >= c.n) {
            out[i] = 0;
            if (status) atomicOr(status, BST_DEV_BAD_ROW);
            continue;
        }
        out[i] = lookup_row(c, r);
    }
}

DeviceProps& props() {
    static DeviceProps p;
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            p.cus = cus;
    });
    return p;
}

int64_t g_tune[BST_TUNE_NKEYS] = {0, 0, 0, 16, 4, 1, 16384};

PackedLit packed_literal(const HostColumn& h, const ScanLit& s) {
    PackedLit p{0, 0, (uint32_t)s.negate, 0};
    const uint64_t maxc = (h.width >= 32) ? 0xffffffffull : ((1ull << h.width) - 1);
    switch (s.mode) {
        case kModeNone:
            p.none = 1;
            break;
        case kModeAll:
            p.a = 0;
            p.span = 0xffffffffu;
            p.negate = 0;
            break;
        case kModeLT:   // code < lo  <=>  code in [0, lo-1]
            if (s.lo == 0) { p.a = 1; p.span = 0; p.none = !s.negate; if (s.negate) { p.a = 0; p.span = 0xffffffffu; p.negate = 0; } }
            else { p.a = 0; p.span = (uint32_t)(s.lo - 1); }
            break;
        case kModeGT:   // code > lo  <=>  code in [lo+1, max]
            if (s.lo >= maxc) { p.none = !s.negate; if (s.negate) { p.a = 0; p.span = 0xffffffffu; p.negate = 0; } }
            else { p.a = (uint32_t)(s.lo + 1); p.span = (uint32_t)(maxc - s.lo - 1); }
            break;
        case kModeEQ:
            p.a = (uint32_t)s.lo;
            p.span = 0;
            break;
        case kModeBetween:
            if (s.lo > s.hi) { p.none = 1; break; }
            p.a = (uint32_t)s.lo;
            p.span = (uint32_t)(s.hi - s.lo);
            break;
    }
    return p;
}

// Workgroups of a lookup launch: 4 per CU by default (measured a few percent
// faster than 16 per CU on random row IDs), or the tuned count.
uint32_t lookup_grid(uint64_t m) {
    if (g_tune[BST_TUNE_LOOKUP_GRID] > 0) return (uint32_t)g_tune[BST_TUNE_LOOKUP_GRID];
    const uint64_t want = (m + kBlock - 1) / kBlock;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)props().cus * 4));
}

int enqueue_fill(uint64_t* out, const uint64_t* in, uint64_t n, int all, hipStream_t st) {
    const uint64_t nwords = (n + 63) >> 6;
    hipLaunchKernelGGL(k_fill, dim3(elem_grid(nwords)), dim3(kBlock), 0, st, out, in, n, all);
    return hip_check(hipGetLastError(), "fill launch");
}

int run_scan(const bst_column* col, const ScanLit& lit, const uint64_t* in, uint64_t* out,
             unsigned long long* counters, hipStream_t st) {
    const DevCol& c = col->dev;
    if (c.n == 0) return BST_OK;
    if (lit.mode == kModeNone || lit.mode == kModeAll) return enqueue_fill(out, in, c.n, lit.mode == kModeAll ? 1 : 0, st);
    if (c.layout == BST_BITPACKED) return launch_packed(c, packed_literal(*col->host, lit), in, out, counters, st);
    ScanLit tuned = lit;
    choose_gather(&tuned, (int)g_tune[BST_TUNE_GATHER_ROWS]);
    return launch_slices(c, tuned, in, out, counters, st);
}

uint32_t batch_kind(const bst_column* col, const ScanLit& lit) {
    if (col->dev.layout == BST_BITPACKED) return 16 + col->dev.width;
    int mi = lit.mode == kModeLT ? 0 : lit.mode == kModeGT ? 1 : lit.mode == kModeEQ ? 2 : 3;
    // bit 3: every literal is one byte long, so byte 1 and M_2 settle every row
    const bool one = lit.llo == 1 && (lit.mode != kModeBetween || lit.lhi == 1);
    return (uint32_t)((col->dev.layout == BST_BYTESLICE ? 1 : 0) | (mi << 1) | (one ? 8 : 0));
}

}  // namespace dev
}  // namespace bst

extern "C" {

int bst_device_count(void) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return 0;
    return n;
}

int bst_upload(const bst_host_column* hc, void* const dev_bufs[BST_NBUF], void* stream, bst_column** out) {
    if (!hc || !dev_bufs || !out) return set_error(BST_EINVAL, "NULL argument");
    const HostColumn& h = hc->c;
    hipStream_t st = (hipStream_t)stream;
    for (int s = 0; s < BST_NBUF; ++s) {
        if (h.buf[s].empty()) continue;
        if (!dev_bufs[s]) return set_error(BST_EINVAL, "missing device buffer for slot " + std::to_string(s));
        if (reinterpret_cast<uintptr_t>(dev_bufs[s]) % 16)
            return set_error(BST_EINVAL, "device buffer for slot " + std::to_string(s) + " is not 16-byte aligned");
        int rc = hip_check(hipMemcpyAsync(dev_bufs[s], h.buf[s].data(), h.buf[s].size(), hipMemcpyHostToDevice, st),
                           "upload");
        if (rc) return rc;
    }
    bst_column* col = new (std::nothrow) bst_column;
    if (!col) return set_error(BST_ENOMEM, "out of host memory");
    memset(&col->dev, 0, sizeof(col->dev));
    col->hc = hc;
    col->host = &h;
    DevCol& c = col->dev;
    c.layout = h.layout;
    c.width = h.width;
    c.K = h.K;
    c.dir_shift = 0;
    while ((1u << c.dir_shift) < h.dir_stride) ++c.dir_shift;
    c.domain_mode = h.domain_mode;
    c.trie_root = h.trie_root;
    c.categorical = h.categorical;
    c.leaf_digits = h.leaf_digits;
    c.n = h.n;
    c.ntiles = h.ntiles;
    c.bs[1] = (const uint8_t*)dev_bufs[BST_BUF_BS1];
    for (uint32_t j = 2; j <= BST_KMAX; ++j) {
        c.bs[j] = (const uint8_t*)dev_bufs[BST_BUF_BS2 + j - 2];
        c.m[j] = (const uint64_t*)dev_bufs[BST_BUF_M2 + j - 2];
        c.dir[j] = (const uint32_t*)dev_bufs[BST_BUF_DIR2 + j - 2];
    }
    c.packed = (const uint32_t*)dev_bufs[BST_BUF_PACKED];
    c.dict = (const uint32_t*)dev_bufs[BST_BUF_DICT];
    c.trie = (const uint32_t*)dev_bufs[BST_BUF_TRIE];
    int rc = hip_check(hipGetDevice(&col->device), "upload device");
    if (rc) {
        delete col;
        return rc;
    }
    *out = col;
    return BST_OK;
}

void bst_column_free(bst_column* col) { delete col; }

int bst_column_info_get(const bst_column* col, bst_column_info* info) {
    if (!col) return set_error(BST_EINVAL, "NULL column");
    return bst_host_info(col->hc, info);
}

int bst_scan(const bst_column* col, bst_pred pred, const uint64_t* in_mask, uint64_t* out_bv,
             uint32_t* dev_status, void* stream) {
    (void)dev_status;
    if (!col) return set_error(BST_EINVAL, "NULL column");
    if (col->dev.n && !out_bv) return set_error(BST_EINVAL, "NULL output bitvector");
    ScanLit lit;
    int rc = rewrite_predicate(*col->host, pred, &lit);
    if (rc) return rc;
    return run_scan(col, lit, in_mask, out_bv, nullptr, (hipStream_t)stream);
}

int bst_scan_codes(const bst_column* col, int op, uint64_t code_lo, uint32_t len_lo, uint64_t code_hi,
                   uint32_t len_hi, const uint64_t* in_mask, uint64_t* out_bv, void* stream) {
    if (!col) return set_error(BST_EINVAL, "NULL column");
    if (col->dev.n && !out_bv) return set_error(BST_EINVAL, "NULL output bitvector");
    ScanLit lit;
    int rc = code_literal(*col->host, op, code_lo, len_lo, code_hi, len_hi, &lit);
    if (rc) return rc;
    if (lit.mode == kModeBetween && lit.lo > lit.hi) lit.mode = kModeNone;
    return run_scan(col, lit, in_mask, out_bv, nullptr, (hipStream_t)stream);
}

int bst_scan_stats(const bst_column* col, bst_pred pred, const uint64_t* in_mask, uint64_t* out_bv,
                   uint64_t* dev_counters, void* stream) {
    if (!col || !dev_counters) return set_error(BST_EINVAL, "NULL argument");
    if (col->dev.n && !out_bv) return set_error(BST_EINVAL, "NULL output bitvector");
    ScanLit lit;
    int rc = rewrite_predicate(*col->host, pred, &lit);
    if (rc) return rc;
    return run_scan(col, lit, in_mask, out_bv, (unsigned long long*)dev_counters, (hipStream_t)stream);
}

int bst_lookup(const bst_column* col, const uint32_t* row_ids, uint64_t m, uint32_t* out_values,
               uint32_t* dev_status, void* stream) {
    if (!col) return set_error(BST_EINVAL, "NULL column");
    if (m == 0) return BST_OK;
    if (!row_ids || !out_values) return set_error(BST_EINVAL, "NULL argument");
    if (col->host->codes_only) return set_error(BST_EUNSUPPORTED, "lookup on a column built from explicit codes");
    const uint32_t grid = lookup_grid(m);
    hipLaunchKernelGGL(k_lookup, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, col->dev, row_ids, m,
                       (const unsigned long long*)nullptr, m, out_values, dev_status, 0);
    return hip_check(hipGetLastError(), "lookup launch");
}

int bst_lookup_counted(const bst_column* col, const uint32_t* row_ids, const uint64_t* dev_count, uint64_t cap,
                       uint32_t* out_values, uint32_t* dev_status, void* stream) {
    if (!col) return set_error(BST_EINVAL, "NULL column");
    if (cap == 0) return BST_OK;
    if (!row_ids || !dev_count || !out_values) return set_error(BST_EINVAL, "NULL argument");
    if (col->host->codes_only) return set_error(BST_EUNSUPPORTED, "lookup on a column built from explicit codes");
    hipLaunchKernelGGL(k_lookup, dim3(lookup_grid(cap)), dim3(kBlock), 0, (hipStream_t)stream, col->dev, row_ids, cap,
                       (const unsigned long long*)dev_count, cap, out_values, dev_status, 1);
    return hip_check(hipGetLastError(), "lookup launch");
}

uint64_t bst_compact_workspace_bytes(uint64_t n_rows) {
    const uint64_t nt = (n_rows + kTileRows - 1) / kTileRows;
    return 8 * std::max<uint64_t>(1, (nt + kChunkTiles - 1) / kChunkTiles);
}

int bst_bv_compact(const uint64_t* bv, uint64_t n_rows, uint32_t* out_ids, uint64_t cap, uint64_t* dev_count,
                   void* workspace, uint32_t* dev_status, void* stream) {
    if (!dev_count || !workspace || (n_rows && !bv) || (cap && !out_ids)) return set_error(BST_EINVAL, "NULL argument");
    if (n_rows > 0xffffffffull) return set_error(BST_ERANGE, "row IDs are 32-bit: at most 2^32 - 1 rows");
    hipStream_t st = (hipStream_t)stream;
    const uint64_t nt = (n_rows + kTileRows - 1) / kTileRows;
    if (nt == 0) {
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, (unsigned long long*)dev_count, 1);
        return hip_check(hipGetLastError(), "compact launch");
    }
    const uint64_t nchunks = (nt + kChunkTiles - 1) / kChunkTiles;   // at most 2^15 (n < 2^32)
    const uint32_t grid = (uint32_t)((nchunks + kWavesPerBlock - 1) / kWavesPerBlock);
    uint64_t* cc = (uint64_t*)workspace;
    hipLaunchKernelGGL(k_chunk_popc, dim3(grid), dim3(kBlock), 0, st, bv, n_rows, nchunks, cc);
    hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(kScanBlock), 0, st, cc, nchunks, (unsigned long long*)dev_count);
    hipLaunchKernelGGL(k_write_ids, dim3(grid), dim3(kBlock), 0, st, bv, n_rows, nchunks, cc, out_ids, cap, dev_status);
    return hip_check(hipGetLastError(), "compact launch");
}

int bst_lookup_bv(const bst_column* col, const uint64_t* bv, uint32_t* out_values, uint64_t cap, uint64_t* dev_count,
                  uint32_t* ids_tmp, void* workspace, uint32_t* dev_status, void* stream) {
    if (!col) return set_error(BST_EINVAL, "NULL column");
    if (col->host->codes_only) return set_error(BST_EUNSUPPORTED, "lookup on a column built from explicit codes");
    int rc = bst_bv_compact(bv, col->dev.n, ids_tmp, cap, dev_count, workspace, dev_status, stream);
    if (rc) return rc;
    if (cap == 0) return BST_OK;
    if (!out_values) return set_error(BST_EINVAL, "NULL output");
    const uint32_t grid = lookup_grid(cap);
    hipLaunchKernelGGL(k_lookup, dim3(grid), dim3(kBlock), 0, (hipStream_t)stream, col->dev, ids_tmp, cap,
                       (const unsigned long long*)dev_count, cap, out_values, dev_status, 0);
    return hip_check(hipGetLastError(), "lookup launch");
}

}  // extern "C"

// ---- lookup of qualifying rows without caller-provided device memory ----
// The compaction workspace and the row-ID staging of bst_lookup_bv live in one
// file-scope device array.  Host code never passes `scratch` itself to a kernel
// or copy: there the name is a host-side stand-in, not the device address.  The
// address is taken per device with hipGetSymbolAddress (each GPU holds its own
// copy) and kept for the process.
namespace {
constexpr uint64_t kStaticMaxRows = 1ull << 29;   // rows of the scanned column
constexpr uint64_t kStaticMaxIds = 1ull << 21;    // selected rows looked up per call
constexpr uint64_t kStaticTiles = kStaticMaxRows / kTileRows;
constexpr uint64_t kStaticCompactBytes = 8 * ((kStaticTiles + kChunkTiles - 1) / kChunkTiles);   // bst_compact_workspace_bytes
constexpr uint64_t kStaticIdsOffset = (kStaticCompactBytes + 255) / 256 * 256;
constexpr uint64_t kScratchBytes = kStaticIdsOffset + 4 * kStaticMaxIds;   // 8.4 MB
constexpr int kMaxDevices = 64;

struct StaticScratch {
    std::mutex mu;
    void* ptr[kMaxDevices] = {};
};
StaticScratch& static_scratch() {
    static StaticScratch* s = new StaticScratch;   // never destroyed
    return *s;
}
}  // namespace

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// Device address of the current device's scratch array, taken on the first call
// on that device.
static int scratch_address(void** out) {
    int dev = 0;
    int rc = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (rc) return rc;
    if (dev < 0 || dev >= kMaxDevices) return set_error(BST_EUNSUPPORTED, "device index beyond the scratch table");
    StaticScratch& s = static_scratch();
    std::lock_guard<std::mutex> lock(s.mu);
    if (!s.ptr[dev]) {
        void* p = nullptr;
        rc = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (rc) return rc;
        if (!p) return set_error(BST_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        s.ptr[dev] = p;
    }
    *out = s.ptr[dev];
    return BST_OK;
}

extern "C" {

uint64_t bst_lookup_bv_static_max_rows(void) { return kStaticMaxRows; }
uint64_t bst_lookup_bv_static_max_ids(void) { return kStaticMaxIds; }

int bst_lookup_bv_static(const bst_column* col, const uint64_t* bv, uint32_t* out_values, uint64_t cap,
                         uint64_t* dev_count, uint32_t* dev_status, void* stream) {
    if (!col) return set_error(BST_EINVAL, "NULL column");
    if (col->dev.n > kStaticMaxRows)
        return set_error(BST_ERANGE, "bst_lookup_bv_static takes columns of at most 2^29 rows; use bst_lookup_bv");
    if (cap > kStaticMaxIds)
        return set_error(BST_ERANGE, "bst_lookup_bv_static looks up at most 2^21 rows per call; use bst_lookup_bv");
    void* base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    // every scratch location a kernel reads is written earlier in the same
    // call, so nothing needs clearing between calls
    uint8_t* sp = static_cast<uint8_t*>(base);
    return bst_lookup_bv(col, bv, out_values, cap, dev_count, reinterpret_cast<uint32_t*>(sp + kStaticIdsOffset), sp,
                         dev_status, stream);
}

int bst_bv_and(const uint64_t* a, const uint64_t* b, uint64_t* out, uint64_t n_rows, void* stream) {
    if (n_rows == 0) return BST_OK;
    if (!a || !b || !out) return set_error(BST_EINVAL, "NULL argument");
    hipLaunchKernelGGL(k_bv_binop, dim3(elem_grid((n_rows + 63) / 64)), dim3(kBlock), 0, (hipStream_t)stream, a, b, out,
                       n_rows, 0);
    return hip_check(hipGetLastError(), "bv_and launch");
}

int bst_bv_or(const uint64_t* a, const uint64_t* b, uint64_t* out, uint64_t n_rows, void* stream) {
    if (n_rows == 0) return BST_OK;
    if (!a || !b || !out) return set_error(BST_EINVAL, "NULL argument");
    hipLaunchKernelGGL(k_bv_binop, dim3(elem_grid((n_rows + 63) / 64)), dim3(kBlock), 0, (hipStream_t)stream, a, b, out,
                       n_rows, 1);
    return hip_check(hipGetLastError(), "bv_or launch");
}

int bst_bv_andnot(const uint64_t* a, const uint64_t* b, uint64_t* out, uint64_t n_rows, void* stream) {
    if (n_rows == 0) return BST_OK;
    if (!a || !b || !out) return set_error(BST_EINVAL, "NULL argument");
    hipLaunchKernelGGL(k_bv_binop, dim3(elem_grid((n_rows + 63) / 64)), dim3(kBlock), 0, (hipStream_t)stream, a, b, out,
                       n_rows, 2);
    return hip_check(hipGetLastError(), "bv_andnot launch");
}

int bst_bv_not(const uint64_t* a, uint64_t* out, uint64_t n_rows, void* stream) {
    if (n_rows == 0) return BST_OK;
    if (!a || !out) return set_error(BST_EINVAL, "NULL argument");
    hipLaunchKernelGGL(k_bv_binop, dim3(elem_grid((n_rows + 63) / 64)), dim3(kBlock), 0, (hipStream_t)stream, a, a, out,
                       n_rows, 3);
    return hip_check(hipGetLastError(), "bv_not launch");
}

int bst_bv_popcount(const uint64_t* bv, uint64_t n_rows, uint64_t* dev_count, void* stream) {
    if (!dev_count || (n_rows && !bv)) return set_error(BST_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, (unsigned long long*)dev_count, 1);
    if (n_rows)
        // 2 workgroups per CU: each ends with one atomic on the count, and those
        // serialise (about 9 ns apiece measured here: 16 per CU took 59 us for a
        // 500M-row bitvector, 2 per CU 22 us)
        hipLaunchKernelGGL(k_bv_popcount, dim3(std::min<uint32_t>(elem_grid((n_rows + 63) / 64), (uint32_t)props().cus * 2)),
                           dim3(kBlock), 0, st, bv, n_rows,
                           (unsigned long long*)dev_count);
    return hip_check(hipGetLastError(), "popcount launch");
}

// ---- streaming probe ---------------------------------------------------------
int bst_stream_probe(const void* src, uint64_t bytes, void* dst, void* stream) {
    if (!src || !dst) return set_error(BST_EINVAL, "NULL argument");
    if (bytes % kTileRows) return set_error(BST_EINVAL, "probe size must be a multiple of 2048 bytes");
    if (reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
        return set_error(BST_EINVAL, "probe buffers must be 16-byte aligned");
    const uint64_t ntiles = bytes / kTileRows;
    if (!ntiles) return BST_OK;
    hipLaunchKernelGGL(k_stream_probe, dim3(tile_grid(ntiles, g_tune[BST_TUNE_SCAN_GRID])), dim3(kBlock), 0,
                       (hipStream_t)stream, (const uint8_t*)src, ntiles, (uint32_t*)dst);
    return hip_check(hipGetLastError(), "probe launch");
}

// ---- advisor -------------------------------------------------------------
int bst_advise(const bst_column* const* cands, int n_cand, int op, const uint32_t* lits, const double* sels, int n_lit,
               int repeats, uint64_t* scratch_bv, double* times_out, double* auc_out, int* chosen, void* stream) {
    if (!cands || n_cand < 1 || !lits || !sels || n_lit < 1 || !scratch_bv || !auc_out || !chosen)
        return set_error(BST_EINVAL, "bad argument");
    if (op != BST_LT && op != BST_EQ) return set_error(BST_EINVAL, "profiling op must be BST_LT or BST_EQ");
    if (repeats < 1) repeats = 1;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    int rc = hip_check(hipEventCreate(&e0), "event");
    if (rc) return rc;
    rc = hip_check(hipEventCreate(&e1), "event");
    if (rc) {
        (void)hipEventDestroy(e0);
        return rc;
    }
    std::vector<int> layouts(n_cand);
    std::vector<double> t(n_lit), samples(repeats);
    for (int ci = 0; ci < n_cand && !rc; ++ci) {
        const bst_column* col = cands[ci];
        if (!col) { rc = set_error(BST_EINVAL, "NULL candidate"); break; }
        layouts[ci] = (int)col->dev.layout;
        for (int li = 0; li < n_lit && !rc; ++li) {
            bst_pred p{op, lits[li], lits[li]};
            ScanLit lit;
            rc = rewrite_predicate(*col->host, p, &lit);
            if (rc) break;
            rc = run_scan(col, lit, nullptr, scratch_bv, nullptr, st);   // warm-up
            for (int r = 0; r < repeats && !rc; ++r) {
                rc = hip_check(hipEventRecord(e0, st), "event record");
                if (!rc) rc = run_scan(col, lit, nullptr, scratch_bv, nullptr, st);
                if (!rc) rc = hip_check(hipEventRecord(e1, st), "event record");
                if (!rc) rc = hip_check(hipEventSynchronize(e1), "event sync");
                float ms = 0;
                if (!rc) rc = hip_check(hipEventElapsedTime(&ms, e0, e1), "event time");
                samples[r] = ms * 1000.0;
            }
            if (rc) break;
            std::sort(samples.begin(), samples.end());
            t[li] = samples[repeats / 2];
            if (times_out) times_out[(size_t)ci * n_lit + li] = t[li];
        }
        if (!rc) rc = bst_auc(sels, t.data(), n_lit, &auc_out[ci]);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    return bst_choose(layouts.data(), auc_out, n_cand, chosen);
}

int bst_tune_set(int key, int64_t value) {
    if (key < 0 || key >= BST_TUNE_NKEYS) return set_error(BST_EINVAL, "bad tuning key");
    if (key == BST_TUNE_BATCH_STREAMS && (value < 1 || value > 4))
        return set_error(BST_EINVAL, "batch streams must be 1..4");
    if (key == BST_TUNE_BATCH_SOLO_TILES && value < 1) return set_error(BST_EINVAL, "solo tiles must be >= 1");
    g_tune[key] = value;
    return BST_OK;
}

int64_t bst_tune_get(int key) {
    if (key < 0 || key >= BST_TUNE_NKEYS) return -1;
    return g_tune[key];
}

}  // extern "C"

