// Host side of the ByteStore library: dictionary, prefix-preserving encoding
// (Algorithm 1), the three device layouts, literal rewriting and the advisor's
// host arithmetic.  Everything here is exact integer work, parallel over rows.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <numeric>
#include <thread>

#include "internal.h"

namespace bst {

static thread_local std::string g_last_error;

int set_error(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

// ------------------------------------------------------------ parallel helper
static uint32_t host_threads(uint32_t req) {
    if (req) return std::min<uint32_t>(req, 256);
    unsigned hc = std::thread::hardware_concurrency();
    return hc ? std::min<uint32_t>(hc, 64) : 1;
}

// Run fn(lo, hi, t) over [0, n) split into `parts` contiguous chunks aligned to `align`.
static void parallel_chunks(uint64_t n, uint32_t parts, uint64_t align,
                            const std::function<void(uint64_t, uint64_t, uint32_t)>& fn) {
    if (parts <= 1 || n <= align) {
        fn(0, n, 0);
        return;
    }
    uint64_t units = (n + align - 1) / align;
    if (parts > units) parts = (uint32_t)units;
    uint64_t per = (units + parts - 1) / parts;
    std::vector<std::thread> th;
    th.reserve(parts);
    for (uint32_t t = 0; t < parts; ++t) {
        uint64_t lo = std::min(n, (uint64_t)t * per * align);
        uint64_t hi = std::min(n, (uint64_t)(t + 1) * per * align);
        if (lo >= hi) continue;
        th.emplace_back([=, &fn] { fn(lo, hi, t); });
    }
    for (auto& x : th) x.join();
}

// ------------------------------------------------------------ dictionary
static int build_dict(const uint32_t* x, uint64_t n, uint32_t T, Dict& d) {
    d.n = n;
    d.A.clear();
    d.Q.clear();
    d.rank.assign(n, 0);
    if (n == 0) return BST_OK;
    // maximum value
    std::vector<uint32_t> pmax(T, 0);
    parallel_chunks(n, T, 1 << 16, [&](uint64_t lo, uint64_t hi, uint32_t t) {
        uint32_t m = 0;
        for (uint64_t i = lo; i < hi; ++i) m = std::max(m, x[i]);
        pmax[t] = m;
    });
    uint64_t vmax = *std::max_element(pmax.begin(), pmax.end());
    uint64_t span = vmax + 1;
    if (span <= (1ull << 28) && span * (uint64_t)T * 4 <= (3ull << 30)) {
        // counting: one histogram per thread, merged per value range
        std::vector<std::vector<uint32_t>> hist(T);
        parallel_chunks(n, T, 1 << 16, [&](uint64_t lo, uint64_t hi, uint32_t t) {
            hist[t].assign(span, 0);
            uint32_t* h = hist[t].data();
            for (uint64_t i = lo; i < hi; ++i) h[x[i]]++;
        });
        std::vector<uint64_t> total(span, 0);
        parallel_chunks(span, T, 4096, [&](uint64_t lo, uint64_t hi, uint32_t) {
            for (auto& h : hist) {
                if (h.empty()) continue;
                for (uint64_t v = lo; v < hi; ++v) total[v] += h[v];
            }
        });
        hist.clear();
        hist.shrink_to_fit();
        std::vector<uint32_t> rank_of(span, 0);
        uint64_t nd = 0;
        for (uint64_t v = 0; v < span; ++v)
            if (total[v]) {
                rank_of[v] = (uint32_t)nd++;
            }
        d.A.resize(nd);
        d.Q.resize(nd);
        for (uint64_t v = 0; v < span; ++v)
            if (total[v]) {
                d.A[rank_of[v]] = (uint32_t)v;
                d.Q[rank_of[v]] = total[v];
            }
        parallel_chunks(n, T, 1 << 16, [&](uint64_t lo, uint64_t hi, uint32_t) {
            for (uint64_t i = lo; i < hi; ++i) d.rank[i] = rank_of[x[i]];
        });
        return BST_OK;
    }
    // sorting: bucket by the top 8 bits, sort buckets in parallel
    std::vector<uint32_t> tmp(n);
    std::vector<std::vector<uint64_t>> cnt(T, std::vector<uint64_t>(256, 0));
    const int sh = 24;
    parallel_chunks(n, T, 1 << 16, [&](uint64_t lo, uint64_t hi, uint32_t t) {
        for (uint64_t i = lo; i < hi; ++i) cnt[t][x[i] >> sh]++;
    });
    std::vector<uint64_t> bstart(257, 0);
    std::vector<std::vector<uint64_t>> off(T, std::vector<uint64_t>(256, 0));
    {
        uint64_t acc = 0;
        for (int b = 0; b < 256; ++b) {
            bstart[b] = acc;
            for (uint32_t t = 0; t < T; ++t) {
                off[t][b] = acc;
                acc += cnt[t][b];
            }
        }
        bstart[256] = acc;
    }
    parallel_chunks(n, T, 1 << 16, [&](uint64_t lo, uint64_t hi, uint32_t t) {
        auto& o = off[t];
        for (uint64_t i = lo; i < hi; ++i) tmp[o[x[i] >> sh]++] = x[i];
    });
    std::atomic<int> next{0};
    std::vector<std::vector<uint32_t>> uv(256);
    std::vector<std::vector<uint64_t>> uc(256);
    auto worker = [&] {
        for (;;) {
            int b = next.fetch_add(1);
            if (b >= 256) break;
            uint32_t* p = tmp.data() + bstart[b];
            uint64_t len = bstart[b + 1] - bstart[b];
            std::sort(p, p + len);
            for (uint64_t i = 0; i < len;) {
                uint64_t j = i + 1;
                while (j < len && p[j] == p[i]) ++j;
                uv[b].push_back(p[i]);
                uc[b].push_back(j - i);
                i = j;
            }
        }
    };
    {
        std::vector<std::thread> th;
        for (uint32_t t = 0; t < T; ++t) th.emplace_back(worker);
        for (auto& t : th) t.join();
    }
    tmp.clear();
    tmp.shrink_to_fit();
    {
        uint64_t total = 0;
        for (int b = 0; b < 256; ++b) total += uv[b].size();
        d.A.reserve(total);
        d.Q.reserve(total);
    }
    for (int b = 0; b < 256; ++b) {
        d.A.insert(d.A.end(), uv[b].begin(), uv[b].end());
        d.Q.insert(d.Q.end(), uc[b].begin(), uc[b].end());
        std::vector<uint32_t>().swap(uv[b]);
        std::vector<uint64_t>().swap(uc[b]);
    }
    // ranks: a directory over the top bits (about log2 of the distinct count, at
    // most 24) narrows each search to the entries that share them (first[p] =
    // entries below p << shift; nd < 2^32), so it stays in a cache line or two
    // instead of walking the whole sorted array
    const uint32_t* A = d.A.data();
    const uint64_t nd = d.A.size();
    int bits = 8;
    while (bits < 24 && (1ull << bits) < nd) ++bits;
    const int shift = 32 - bits;
    std::vector<uint32_t> first((1u << bits) + 1, (uint32_t)nd);
    for (uint64_t k = nd; k-- > 0;) first[A[k] >> shift] = (uint32_t)k;
    for (uint64_t p = first.size() - 1; p-- > 0;) first[p] = std::min(first[p], first[p + 1]);
    parallel_chunks(n, T, 1 << 16, [&](uint64_t lo, uint64_t hi, uint32_t) {
        for (uint64_t i = lo; i < hi; ++i) {
            const uint32_t p = x[i] >> shift;
            d.rank[i] = (uint32_t)(std::lower_bound(A + first[p], A + first[p + 1], x[i]) - A);
        }
    });
    return BST_OK;
}

// ------------------------------------------------------------ Algorithm 1
// Prefix-preserving encoding for numerical columns: a 256-way tree built depth
// first; each internal node's 255 slots hold the most frequent values of its
// range in value order, the values between slots recurse under pointers, and at
// the depth cut (parent level 2) or when a range fits one node the values take
// consecutive slot numbers.  The recursion also emits the decode tables: per
// internal node and byte, {rank of the value in that slot, child descriptor}.
struct PpeBuilder {
    const std::vector<uint64_t>& Q;
    std::vector<uint64_t>& C;
    std::vector<uint8_t>& L;
    std::vector<uint32_t>& trie;   // 512 uint32 per node: (slot rank, child) x 256; the
                                   // encoder replaces each slot rank by the slot's value
    std::vector<uint32_t> idx;     // scratch for the top-255 selection
    bool leaf_digits = false;      // leaf entries also carry their slot digits

    static uint32_t digits(uint64_t count) {   // smallest beta with 256^beta >= count
        uint32_t beta = 0;
        unsigned __int128 cap = 1;
        while (cap < count) {
            cap *= 256;
            ++beta;
        }
        return beta;
    }

    void shift_in(uint64_t lo, uint64_t hi, uint32_t digit) {
        for (uint64_t i = lo; i < hi; ++i) C[i] = (C[i] << 8) + digit;
    }

    uint32_t encode(uint32_t b, uint64_t s, uint64_t e) {
        if (e - s < 256 || b >= 2) {
            uint32_t beta = digits(e - s + 1);
            for (uint64_t i = s; i < e; ++i) {
                C[i] = (beta ? (C[i] << (8 * beta)) : C[i]) + 1 + (i - s);
                L[i] = (uint8_t)(b + beta);
            }
            // a leaf: base rank s, and (when it fits) the digits of its slot
            // numbers, which fix the length of every code below it
            return kLeafFlag | (uint32_t)s | (leaf_digits ? beta << kLeafDigitsShift : 0u);
        }
        uint32_t node = (uint32_t)(trie.size() / 512);
        trie.resize(trie.size() + 512, 0);
        // the 255 largest frequencies in [s, e); ties prefer the smaller index
        idx.resize(e - s);
        std::iota(idx.begin(), idx.end(), (uint32_t)s);
        auto cmp = [&](uint32_t a, uint32_t c) { return Q[a] != Q[c] ? Q[a] > Q[c] : a < c; };
        std::nth_element(idx.begin(), idx.begin() + 254, idx.end(), cmp);
        std::vector<uint32_t> I(idx.begin(), idx.begin() + 255);
        std::sort(I.begin(), I.end());
        for (uint32_t t = 0; t < 255; ++t) {
            L[I[t]] = (uint8_t)(b + 1);
            C[I[t]] = (C[I[t]] << 8) + t + 1;
            trie[(size_t)node * 512 + 2 * (t + 1)] = I[t];
        }
        uint32_t kids[256];
        for (uint32_t t = 0; t < 254; ++t) {
            shift_in(I[t] + 1, I[t + 1], t + 1);
            kids[t + 1] = encode(b + 1, I[t] + 1, I[t + 1]);
        }
        shift_in(s, I[0], 0);
        kids[0] = encode(b + 1, s, I[0]);
        shift_in((uint64_t)I[254] + 1, e, 255);
        kids[255] = encode(b + 1, (uint64_t)I[254] + 1, e);
        for (uint32_t p = 0; p < 256; ++p) trie[(size_t)node * 512 + 2 * p + 1] = kids[p];
        return node;
    }
};

// ------------------------------------------------------------ layouts
static inline uint64_t bs1_pos(uint64_t r) {
    // tile-interleaved slice: lane L = (r / 32) % 64 of a tile owns its 32
    // consecutive rows as eight dwords, row p = r % 32 in byte p / 8 of dword
    // p % 8; dwords 0-3 of the lanes fill the tile's first 1 KB, dwords 4-7 its second
    const uint64_t p = r & 31, lane = (r >> 5) & 63, i = p & 7;
    return (r & ~(uint64_t)(kTileRows - 1)) + (i >> 2) * 1024 + lane * 16 + (i & 3) * 4 + (p >> 3);
}

static inline uint64_t bsj_pos(uint64_t r) {
    // ByteSlice slices after the first: lane L = (r / 32) % 64 of a tile owns its
    // 32 rows as 32 contiguous bytes at 32L (row p = r % 32 in byte p / 8 of dword
    // p % 8), so a lane that needs its bytes of the slice reads one 32-byte span
    const uint64_t p = r & 31, lane = (r >> 5) & 63;
    return (r & ~(uint64_t)(kTileRows - 1)) + lane * 32 + (p & 7) * 4 + (p >> 3);
}

static int log2_exact(uint32_t v) {
    int s = 0;
    while ((1u << s) < v) ++s;
    return ((1u << s) == v) ? s : -1;
}

// VBS layout from per-distinct codes and per-row ranks.
static void build_vbs(HostColumn& c, const uint32_t* rank, uint32_t T) {
    const uint64_t n = c.n, nt = c.ntiles, npad = nt * kTileRows;
    const uint32_t K = c.K, D = c.dir_stride;
    const uint64_t nwords = nt * kGroupsPerTile, ndir = npad / D + 1;
    c.buf[BST_BUF_BS1].assign(npad, 0);
    for (uint32_t j = 2; j <= K; ++j) {
        c.buf[BST_BUF_M2 + j - 2].assign(nwords * 8, 0);
        c.buf[BST_BUF_DIR2 + j - 2].assign(ndir * 4, 0);
    }
    // pass 1: rows with a j-th byte per chunk of tiles
    const uint32_t parts = std::max<uint32_t>(1, std::min<uint32_t>(T, (uint32_t)std::max<uint64_t>(1, nt)));
    std::vector<std::array<uint64_t, BST_KMAX + 1>> cnt(parts);
    for (auto& a : cnt) a.fill(0);
    std::vector<uint64_t> plo(parts, 0);
    parallel_chunks(n, parts, kTileRows, [&](uint64_t lo, uint64_t hi, uint32_t t) {
        plo[t] = lo;
        for (uint64_t r = lo; r < hi; ++r) {
            uint32_t len = c.clen[rank[r]];
            for (uint32_t j = 1; j <= len; ++j) cnt[t][j]++;
        }
    });
    std::vector<std::array<uint64_t, BST_KMAX + 1>> start(parts);
    std::array<uint64_t, BST_KMAX + 1> tot;
    tot.fill(0);
    for (uint32_t t = 0; t < parts; ++t) {
        start[t] = tot;
        for (uint32_t j = 1; j <= BST_KMAX; ++j) tot[j] += cnt[t][j];
    }
    for (uint32_t j = 1; j <= BST_KMAX; ++j) c.rows_by_len[j] = tot[j] - (j < BST_KMAX ? tot[j + 1] : 0);
    c.rows_by_len[0] = 0;
    // without length-carrying decode leaves, every code shorter than K ends at a 0 in M_{len+1}
    for (uint32_t j = 0; j <= BST_KMAX; ++j) c.rows_end_by_mask[j] = j < K ? c.rows_by_len[j] : 0;
    for (uint32_t j = 2; j <= K; ++j) c.buf[BST_BUF_BS2 + j - 2].assign(tot[j] + 64, 0);
    // pass 2: bytes, masks, directories
    parallel_chunks(n, parts, kTileRows, [&](uint64_t lo, uint64_t hi, uint32_t t) {
        std::array<uint64_t, BST_KMAX + 1> pos = start[t];
        uint8_t* bs1 = c.buf[BST_BUF_BS1].data();
        for (uint64_t r = lo; r < hi; ++r) {
            if ((r % D) == 0)
                for (uint32_t j = 2; j <= K; ++j)
                    reinterpret_cast<uint32_t*>(c.buf[BST_BUF_DIR2 + j - 2].data())[r / D] = (uint32_t)pos[j];
            uint32_t k = rank[r];
            uint64_t code = c.code[k];
            uint32_t len = c.clen[k];
            bs1[bs1_pos(r)] = (uint8_t)(code >> (8 * (len - 1)));
            for (uint32_t j = 2; j <= len; ++j) {
                c.buf[BST_BUF_BS2 + j - 2][pos[j]++] = (uint8_t)(code >> (8 * (len - j)));
                reinterpret_cast<uint64_t*>(c.buf[BST_BUF_M2 + j - 2].data())[r >> 6] |= 1ull << (r & 63);
            }
        }
    });
    // directory entries past the last row (padding positions) hold the totals
    for (uint32_t j = 2; j <= K; ++j) {
        uint32_t* dir = reinterpret_cast<uint32_t*>(c.buf[BST_BUF_DIR2 + j - 2].data());
        for (uint64_t q = (n + D - 1) / D; q < ndir; ++q) dir[q] = (uint32_t)tot[j];
    }
}

// ByteSlice: code left-aligned in K bytes; BS_1 tile-interleaved like PP-VBS's
// BS_1, later slices with each lane's 32 bytes contiguous (bsj_pos).
static void build_byteslice(HostColumn& c, const uint32_t* vals, uint32_t T) {
    const uint64_t n = c.n, npad = c.ntiles * kTileRows;
    const uint32_t K = c.K, w = c.width;
    c.buf[BST_BUF_BS1].assign(npad, 0);
    for (uint32_t j = 2; j <= K; ++j) c.buf[BST_BUF_BS2 + j - 2].assign(npad, 0);
    parallel_chunks(n, T, kTileRows, [&](uint64_t lo, uint64_t hi, uint32_t) {
        for (uint64_t r = lo; r < hi; ++r) {
            uint64_t v = (uint64_t)vals[r] << (8 * K - w);
            // every slice holds a lane's 32 rows in the same registers as BS_1; later
            // slices keep each lane's bytes together (read lane by lane, only by
            // lanes with rows still pending)
            c.buf[BST_BUF_BS1][bs1_pos(r)] = (uint8_t)(v >> (8 * (K - 1)));
            const uint64_t pj = bsj_pos(r);
            for (uint32_t j = 2; j <= K; ++j) c.buf[BST_BUF_BS2 + j - 2][pj] = (uint8_t)(v >> (8 * (K - j)));
        }
    });
}

// Bit-Packed: in each tile, lane L's 32 codes (rows tile*2048 + k*64 + L) are
// packed back to back, LSB first, into w dwords; dword i of lane L is stored at
// tile*64*w + i*64 + L so one wave reads dword i of all lanes contiguously.
static void build_bitpacked(HostColumn& c, const uint32_t* vals, uint32_t T) {
    const uint64_t n = c.n, nt = c.ntiles;
    const uint32_t w = c.width;
    c.buf[BST_BUF_PACKED].assign(nt * 64 * w * 4, 0);
    uint32_t* out = reinterpret_cast<uint32_t*>(c.buf[BST_BUF_PACKED].data());
    parallel_chunks(nt, T, 1, [&](uint64_t tlo, uint64_t thi, uint32_t) {
        for (uint64_t t = tlo; t < thi; ++t) {
            uint32_t* base = out + t * 64 * w;
            for (uint32_t lane = 0; lane < 64; ++lane) {
                for (uint32_t k = 0; k < 32; ++k) {
                    uint64_t r = t * kTileRows + (uint64_t)k * 64 + lane;
                    uint64_t code = r < n ? vals[r] : 0;
                    uint64_t bit = (uint64_t)k * w;
                    uint32_t i = (uint32_t)(bit >> 5), sh = (uint32_t)(bit & 31);
                    base[(uint64_t)i * 64 + lane] |= (uint32_t)(code << sh);
                    if (sh + w > 32) base[(uint64_t)(i + 1) * 64 + lane] |= (uint32_t)(code >> (32 - sh));
                }
            }
        }
    });
}

static uint32_t bits_for(uint64_t nd) {
    uint32_t w = 1;
    while (w < 32 && (1ull << w) < nd) ++w;
    return w;
}

void choose_gather(ScanLit* s, int rows) {
    // pending rows per 32-row lane that a level gathers straight from its slice;
    // a tile with a lane holding more stages the level's run in LDS
    s->gather = (uint32_t)std::max(0, std::min(rows, 4));
}

// Categorical PPE (Sec. 3.1, Algorithm 2): the distinct values, taken in
// descending frequency (ties: smaller value first), fill a balanced 256-way tree
// breadth first.  Level b holds the codes (c << 8) + i for every pointer path c
// of b - 1 bytes and slot i = 1..255; every level but the last is full, and the
// last level is filled slot by slot (i outer, c inner) so its values spread over
// all of its nodes.  code/clen are indexed by sorted dictionary position;
// by_code[alpha] = dictionary position of the alpha-th most frequent value.
static int categorical_codes(const std::vector<uint64_t>& Q, std::vector<uint64_t>& code, std::vector<uint8_t>& clen,
                             uint32_t* K, std::vector<uint32_t>& by_code) {
    const uint64_t n = Q.size();
    code.assign(n, 0);
    clen.assign(n, 0);
    by_code.resize(n);
    std::iota(by_code.begin(), by_code.end(), 0u);
    std::stable_sort(by_code.begin(), by_code.end(), [&](uint32_t a, uint32_t b) { return Q[a] > Q[b]; });
    uint32_t B = 0;   // levels: smallest B with 256^B >= n + 1
    for (unsigned __int128 cap = 1; cap < (unsigned __int128)n + 1; cap *= 256) ++B;
    if (B == 0) B = 1;
    if (B > BST_KMAX) return set_error(BST_ERANGE, "code longer than BST_KMAX bytes");
    uint64_t alpha = 0;
    for (uint32_t b = 1; b < B && alpha < n; ++b) {
        const uint64_t paths = 1ull << (8 * (b - 1));
        for (uint64_t p = 0; p < paths && alpha < n; ++p)
            for (uint32_t i = 1; i < 256 && alpha < n; ++i, ++alpha) {
                code[by_code[alpha]] = (p << 8) + i;
                clen[by_code[alpha]] = (uint8_t)b;
            }
    }
    const uint64_t paths = 1ull << (8 * (B - 1));
    for (uint32_t i = 1; i < 256 && alpha < n; ++i)
        for (uint64_t p = 0; p < paths && alpha < n; ++p, ++alpha) {
            code[by_code[alpha]] = (p << 8) + i;
            clen[by_code[alpha]] = (uint8_t)B;
        }
    *K = B;
    return BST_OK;
}

static int encode_column(const Dict& d, int layout, uint32_t width, uint32_t dir_stride, uint32_t T,
                         HostColumn& c) {
    if (layout < BST_BITPACKED || layout > BST_PPVBS_CATEGORICAL) return set_error(BST_EINVAL, "bad layout");
    const bool categorical = layout == BST_PPVBS_CATEGORICAL;
    if (categorical) layout = BST_PPVBS;
    if (dir_stride == 0) dir_stride = kDefaultDirStride;
    if (log2_exact(dir_stride) < 6 || dir_stride > kTileRows)
        return set_error(BST_EINVAL, "dir_stride must be a power of two in [64, 2048]");
    if (width > 32) return set_error(BST_EINVAL, "width must be in [0, 32]");
    if (d.A.size() >= (1ull << 31)) return set_error(BST_ERANGE, "too many distinct values");
    c.layout = (uint32_t)layout;
    c.n = d.n;
    c.nd = d.A.size();
    c.ntiles = (c.n + kTileRows - 1) / kTileRows;
    c.dir_stride = dir_stride;
    T = host_threads(T);
    if (layout == BST_PPVBS && categorical) {
        c.domain_mode = 0;
        c.categorical = 1;
        c.dict = d.A;
        uint32_t K = 1;
        std::vector<uint32_t> by_code;   // values in code (frequency) order
        int rc = categorical_codes(d.Q, c.code, c.clen, &K, by_code);
        if (rc) return rc;
        for (uint32_t k = 0; k < c.nd; ++k) by_code[k] = d.A[by_code[k]];
        c.K = K;
        c.width = 8 * K;
        c.buf[BST_BUF_DICT].resize(c.nd * 4);
        if (c.nd) memcpy(c.buf[BST_BUF_DICT].data(), by_code.data(), c.nd * 4);
        build_vbs(c, d.rank.data(), T);
        return BST_OK;
    }
    if (layout == BST_PPVBS) {
        c.domain_mode = 0;
        c.dict = d.A;
        c.code.assign(c.nd, 0);
        c.clen.assign(c.nd, 0);
        std::vector<uint32_t> trie;
        PpeBuilder pb{d.Q, c.code, c.clen, trie, {}, c.nd < kLeafDigitsMaxValues};
        c.trie_root = pb.encode(0, 0, c.nd);
        c.leaf_digits = pb.leaf_digits ? 1u : 0u;
        uint32_t K = 1;
        for (uint8_t l : c.clen) K = std::max<uint32_t>(K, l);
        if (K > BST_KMAX) return set_error(BST_ERANGE, "code longer than BST_KMAX bytes");
        c.K = K;
        c.width = 8 * K;
        c.buf[BST_BUF_DICT].resize(c.nd * 4);
        if (c.nd) memcpy(c.buf[BST_BUF_DICT].data(), c.dict.data(), c.nd * 4);
        // codes that end in a slot: only for them does a lookup read M_{len+1} to see
        // the code end (a leaf entry carries the length of the codes below it)
        std::vector<uint8_t> in_slot(c.nd, 0);
        for (size_t k = 0; k < trie.size(); k += 2)
            if (k % 512 != 0) in_slot[trie[k]] = 1;
        c.buf[BST_BUF_TRIE].resize(trie.size() * 4);
        build_vbs(c, d.rank.data(), T);
        if (c.leaf_digits) {
            for (uint32_t j = 0; j <= BST_KMAX; ++j) c.rows_end_by_mask[j] = 0;
            for (uint64_t i = 0; i < c.nd; ++i)
                if (in_slot[i] && c.clen[i] < K) c.rows_end_by_mask[c.clen[i]] += d.Q[i];
        }
        // slot entries carry the slot's value rather than its rank, so a lookup of
        // a code that ends in a slot needs no dictionary read
        for (size_t k = 0; k < trie.size(); k += 2)
            if (k % 512 != 0) trie[k] = c.dict[trie[k]];
        if (!trie.empty()) memcpy(c.buf[BST_BUF_TRIE].data(), trie.data(), trie.size() * 4);
        return BST_OK;
    }
    // fixed-length codes
    const uint32_t* vals;
    std::vector<uint32_t> tmp;
    if (width == 0) {
        c.domain_mode = 0;
        c.width = bits_for(c.nd);
        c.dict = d.A;
        c.code.resize(c.nd);
        std::iota(c.code.begin(), c.code.end(), 0ull);
        c.buf[BST_BUF_DICT].resize(c.nd * 4);
        if (c.nd) memcpy(c.buf[BST_BUF_DICT].data(), c.dict.data(), c.nd * 4);
        vals = d.rank.data();
    } else {
        c.domain_mode = 1;
        c.width = width;
        if (c.nd && width < 32 && (uint64_t)d.A.back() >= (1ull << width))
            return set_error(BST_ERANGE, "a value does not fit the domain width");
        c.code.assign(d.A.begin(), d.A.end());
        tmp.resize(c.n);
        parallel_chunks(c.n, T, 1 << 16, [&](uint64_t lo, uint64_t hi, uint32_t) {
            for (uint64_t i = lo; i < hi; ++i) tmp[i] = d.A[d.rank[i]];
        });
        vals = tmp.data();
    }
    c.clen.assign(c.nd, (uint8_t)((c.width + 7) / 8));
    if (layout == BST_BYTESLICE) {
        c.K = (c.width + 7) / 8;
        build_byteslice(c, vals, T);
    } else {
        c.K = 1;
        build_bitpacked(c, vals, T);
    }
    return BST_OK;
}

// ------------------------------------------------------------ literals
// Code of dictionary entry k in the column's code space, padded for the kernels.
static void padded_code(const HostColumn& c, uint64_t k, uint64_t* code6, uint32_t* len) {
    if (c.layout == BST_BITPACKED) {   // the plain code: a rank, or the value in domain mode
        *code6 = k;
        *len = 0;
        return;
    }
    if (c.layout == BST_BYTESLICE) {
        uint64_t v = k << (8 * c.K - c.width);
        *code6 = v << (8 * (BST_KMAX - c.K));
        *len = c.K;
        return;
    }
    uint32_t L = c.clen[k];
    *code6 = c.code[k] << (8 * (BST_KMAX - L));
    *len = L;
}

int rewrite_predicate(const HostColumn& c, const bst_pred& p, ScanLit* out) {
    if (p.op < BST_LT || p.op > BST_BETWEEN) return set_error(BST_EINVAL, "bad predicate op");
    if (c.categorical && p.op != BST_EQ && p.op != BST_NE)
        return set_error(BST_EINVAL, "a categorical column supports '=' and '!=' scans only");
    // code space: dictionary entries 0..count-1 (domain mode: every w-bit value)
    const bool dom = (c.layout != BST_PPVBS) && c.domain_mode;
    const uint64_t count = dom ? (1ull << c.width) : c.nd;
    auto lb = [&](uint64_t x) -> uint64_t {   // entries < x
        if (dom) return std::min<uint64_t>(x, count);
        return (uint64_t)(std::lower_bound(c.dict.begin(), c.dict.end(), (uint32_t)x) - c.dict.begin());
    };
    auto ub = [&](uint64_t x) -> uint64_t {   // entries <= x
        if (dom) return std::min<uint64_t>(x + 1, count);
        return (uint64_t)(std::upper_bound(c.dict.begin(), c.dict.end(), (uint32_t)x) - c.dict.begin());
    };
    auto code = [&](uint64_t k, uint64_t* v, uint32_t* l) { padded_code(c, k, v, l); };
    ScanLit s{};
    s.mode = kModeNone;
    const uint64_t x = p.lo;
    const uint64_t l0 = lb(x), u0 = ub(x);
    const bool present = u0 > l0;
    switch (p.op) {
        case BST_LT:   // rank < l0
            if (l0 == 0) s.mode = kModeNone;
            else if (l0 == count) s.mode = kModeAll;
            else { s.mode = kModeLT; code(l0, &s.lo, &s.llo); }
            break;
        case BST_LE:   // rank < u0
            if (u0 == 0) s.mode = kModeNone;
            else if (u0 == count) s.mode = kModeAll;
            else if (present) { s.mode = kModeGT; s.negate = 1; code(l0, &s.lo, &s.llo); }
            else { s.mode = kModeLT; code(l0, &s.lo, &s.llo); }
            break;
        case BST_GT:   // rank >= u0
            if (u0 == count) s.mode = kModeNone;
            else if (u0 == 0) s.mode = kModeAll;
            else if (present) { s.mode = kModeGT; code(l0, &s.lo, &s.llo); }
            else { s.mode = kModeLT; s.negate = 1; code(u0, &s.lo, &s.llo); }
            break;
        case BST_GE:   // rank >= l0
            if (l0 == count) s.mode = kModeNone;
            else if (l0 == 0) s.mode = kModeAll;
            else { s.mode = kModeLT; s.negate = 1; code(l0, &s.lo, &s.llo); }
            break;
        case BST_EQ:
            if (!present) s.mode = kModeNone;
            else { s.mode = kModeEQ; code(l0, &s.lo, &s.llo); }
            break;
        case BST_NE:
            if (!present) s.mode = kModeAll;
            else { s.mode = kModeEQ; s.negate = 1; code(l0, &s.lo, &s.llo); }
            break;
        case BST_BETWEEN: {
            if (p.lo > p.hi) { s.mode = kModeNone; break; }
            uint64_t a = l0, b1 = ub(p.hi);   // ranks a .. b1-1
            if (a >= b1) s.mode = kModeNone;
            else if (a == 0 && b1 == count) s.mode = kModeAll;
            else {
                s.mode = kModeBetween;
                code(a, &s.lo, &s.llo);
                code(b1 - 1, &s.hi, &s.lhi);
            }
            break;
        }
    }
    if (count == 0) s.mode = kModeNone;   // an empty column selects nothing
    *out = s;
    return BST_OK;
}

int code_literal(const HostColumn& c, int op, uint64_t lo, uint32_t llo, uint64_t hi, uint32_t lhi,
                 ScanLit* out) {
    if (op < BST_LT || op > BST_BETWEEN) return set_error(BST_EINVAL, "bad op");
    ScanLit s{};
    auto pad = [&](uint64_t v, uint32_t l, uint64_t* o, uint32_t* ol) -> int {
        if (c.layout == BST_BITPACKED) {
            if (c.width < 64 && v >= (1ull << c.width)) return set_error(BST_ERANGE, "code exceeds width");
            *o = v;
            *ol = 0;
            return BST_OK;
        }
        if (l < 1 || l > BST_KMAX) return set_error(BST_EINVAL, "code length must be 1..6");
        if (l < 8 && (v >> (8 * l)) != 0) return set_error(BST_EINVAL, "code wider than its length");
        *o = v << (8 * (BST_KMAX - l));
        *ol = l;
        return BST_OK;
    };
    int rc = pad(lo, llo, &s.lo, &s.llo);
    if (rc) return rc;
    switch (op) {
        case BST_LT: s.mode = kModeLT; break;
        case BST_GE: s.mode = kModeLT; s.negate = 1; break;
        case BST_GT: s.mode = kModeGT; break;
        case BST_LE: s.mode = kModeGT; s.negate = 1; break;
        case BST_EQ: s.mode = kModeEQ; break;
        case BST_NE: s.mode = kModeEQ; s.negate = 1; break;
        case BST_BETWEEN:
            s.mode = kModeBetween;
            rc = pad(hi, lhi, &s.hi, &s.lhi);
            if (rc) return rc;
            break;
    }
    *out = s;
    return BST_OK;
}

}  // namespace bst

using namespace bst;

// ====================================================================== ABI
extern "C" {

const char* bst_last_error(void) { return g_last_error.c_str(); }

int bst_version(void) { return 10000; }

int bst_dict_build(const uint32_t* values, uint64_t n, uint32_t n_threads, bst_dict** out) {
    if (!out || (n && !values)) return set_error(BST_EINVAL, "NULL argument");
    if (n >= (1ull << 32)) return set_error(BST_EINVAL, "n_rows must be < 2^32");
    bst_dict* d = new (std::nothrow) bst_dict;
    if (!d) return set_error(BST_ENOMEM, "out of host memory");
    try {
        int rc = build_dict(values, n, host_threads(n_threads), d->d);
        if (rc) {
            delete d;
            return rc;
        }
    } catch (const std::bad_alloc&) {
        delete d;
        return set_error(BST_ENOMEM, "out of host memory");
    }
    *out = d;
    return BST_OK;
}

void bst_dict_free(bst_dict* d) { delete d; }

int bst_dict_info(const bst_dict* d, uint64_t* n_rows, uint64_t* n_distinct) {
    if (!d) return set_error(BST_EINVAL, "NULL dict");
    if (n_rows) *n_rows = d->d.n;
    if (n_distinct) *n_distinct = d->d.A.size();
    return BST_OK;
}

int bst_dict_values(const bst_dict* d, uint32_t* values_out, uint64_t* counts_out) {
    if (!d) return set_error(BST_EINVAL, "NULL dict");
    if (values_out && !d->d.A.empty()) memcpy(values_out, d->d.A.data(), d->d.A.size() * 4);
    if (counts_out && !d->d.Q.empty()) memcpy(counts_out, d->d.Q.data(), d->d.Q.size() * 8);
    return BST_OK;
}

int bst_encode(const bst_dict* d, int layout, uint32_t width, uint32_t dir_stride, uint32_t n_threads,
               bst_host_column** out) {
    if (!d || !out) return set_error(BST_EINVAL, "NULL argument");
    bst_host_column* c = new (std::nothrow) bst_host_column;
    if (!c) return set_error(BST_ENOMEM, "out of host memory");
    try {
        int rc = encode_column(d->d, layout, width, dir_stride, n_threads, c->c);
        if (rc) {
            delete c;
            return rc;
        }
    } catch (const std::bad_alloc&) {
        delete c;
        return set_error(BST_ENOMEM, "out of host memory");
    }
    *out = c;
    return BST_OK;
}

int bst_encode_host(const uint32_t* values, uint64_t n, int layout, uint32_t width, bst_host_column** out) {
    bst_dict* d = nullptr;
    int rc = bst_dict_build(values, n, 0, &d);
    if (rc) return rc;
    rc = bst_encode(d, layout, width, 0, 0, out);
    bst_dict_free(d);
    return rc;
}

int bst_encode_codes(const uint64_t* codes, const uint8_t* lengths, uint64_t n, uint32_t k_max,
                     bst_host_column** out) {
    if (!out || (n && (!codes || !lengths))) return set_error(BST_EINVAL, "NULL argument");
    if (k_max < 1 || k_max > BST_KMAX) return set_error(BST_EINVAL, "k_max must be 1..6");
    if (n >= (1ull << 32)) return set_error(BST_EINVAL, "n_rows must be < 2^32");
    // distinct codes, as padded integers, define the "values" (their ranks)
    std::vector<std::pair<uint64_t, uint8_t>> dc;
    dc.reserve(n);
    for (uint64_t r = 0; r < n; ++r) {
        uint8_t l = lengths[r];
        if (l < 1 || l > k_max) return set_error(BST_EINVAL, "code length outside 1..k_max");
        if (l < 8 && (codes[r] >> (8 * l)) != 0) return set_error(BST_EINVAL, "code wider than its length");
        dc.push_back({codes[r] << (8 * (k_max - l)), l});
    }
    std::sort(dc.begin(), dc.end());
    dc.erase(std::unique(dc.begin(), dc.end()), dc.end());
    for (size_t i = 1; i < dc.size(); ++i)
        if (dc[i].first == dc[i - 1].first)
            return set_error(BST_EINVAL, "two codes coincide once padded (prefix rule violated)");
    bst_host_column* hc = new (std::nothrow) bst_host_column;
    if (!hc) return set_error(BST_ENOMEM, "out of host memory");
    HostColumn& c = hc->c;
    c.layout = BST_PPVBS;
    c.codes_only = true;
    c.n = n;
    c.nd = dc.size();
    c.ntiles = (n + kTileRows - 1) / kTileRows;
    c.K = k_max;
    c.width = 8 * k_max;
    c.dir_stride = kDefaultDirStride;
    c.code.resize(c.nd);
    c.clen.resize(c.nd);
    c.dict.resize(c.nd);
    for (size_t i = 0; i < dc.size(); ++i) {
        c.code[i] = dc[i].first >> (8 * (k_max - dc[i].second));
        c.clen[i] = dc[i].second;
        c.dict[i] = (uint32_t)i;
    }
    std::vector<uint32_t> rank(n);
    for (uint64_t r = 0; r < n; ++r) {
        uint64_t p = codes[r] << (8 * (k_max - lengths[r]));
        rank[r] = (uint32_t)(std::lower_bound(dc.begin(), dc.end(), std::make_pair(p, (uint8_t)0)) - dc.begin());
    }
    build_vbs(c, rank.data(), 1);
    std::vector<uint64_t> counts(c.nd, 0);
    for (uint64_t r = 0; r < n; ++r) counts[rank[r]]++;
    *out = hc;
    return BST_OK;
}

void bst_free_host(bst_host_column* c) { delete c; }

int bst_host_info(const bst_host_column* hc, bst_column_info* info) {
    if (!hc || !info) return set_error(BST_EINVAL, "NULL argument");
    const HostColumn& c = hc->c;
    memset(info, 0, sizeof(*info));
    info->layout = c.layout;
    info->width_bits = c.width;
    info->k_max = c.K;
    info->dir_stride = c.dir_stride;
    info->domain_mode = c.domain_mode;
    info->categorical = c.categorical;
    info->n_rows = c.n;
    info->n_distinct = c.nd;
    for (int s = 0; s < BST_NBUF; ++s) {
        info->bytes[s] = c.buf[s].size();
        info->total_bytes += c.buf[s].size();
        if (s != BST_BUF_DICT && s != BST_BUF_TRIE) info->layout_bytes += c.buf[s].size();
    }
    for (int j = 0; j <= BST_KMAX; ++j) info->rows_by_len[j] = c.rows_by_len[j];
    for (int j = 0; j <= BST_KMAX; ++j) info->rows_end_by_mask[j] = c.rows_end_by_mask[j];
    return BST_OK;
}

int bst_host_code_table(const bst_host_column* hc, uint64_t* codes, uint8_t* lengths) {
    if (!hc) return set_error(BST_EINVAL, "NULL column");
    const HostColumn& c = hc->c;
    if (codes && c.nd) memcpy(codes, c.code.data(), c.nd * 8);
    if (lengths && c.nd) memcpy(lengths, c.clen.data(), c.nd);
    return BST_OK;
}

int bst_host_paper_view(const bst_host_column* hc, int part, int j, void* out, uint64_t* bytes) {
    if (!hc || !bytes) return set_error(BST_EINVAL, "NULL argument");
    const HostColumn& c = hc->c;
    const uint64_t n = c.n;
    if (part == 0) {
        if (c.layout == BST_BITPACKED || j < 1 || j > (int)c.K) return set_error(BST_EINVAL, "no such slice");
        uint64_t len = (j == 1 || c.layout == BST_BYTESLICE) ? n : c.buf[BST_BUF_BS2 + j - 2].size() - 64;
        *bytes = len;
        if (!out) return BST_OK;
        uint8_t* o = (uint8_t*)out;
        const uint8_t* src = c.buf[j == 1 ? BST_BUF_BS1 : BST_BUF_BS2 + j - 2].data();
        if (j == 1)   // tile-interleaved slices back to row order
            for (uint64_t r = 0; r < n; ++r) o[r] = src[bs1_pos(r)];
        else if (c.layout == BST_BYTESLICE)
            for (uint64_t r = 0; r < n; ++r) o[r] = src[bsj_pos(r)];
        else
            memcpy(o, src, len);
        return BST_OK;
    }
    if (part == 1) {
        if (c.layout != BST_PPVBS || j < 2 || j > (int)c.K) return set_error(BST_EINVAL, "no such mask");
        uint64_t nw = (n + 63) / 64;
        *bytes = nw * 8;
        if (out) memcpy(out, c.buf[BST_BUF_M2 + j - 2].data(), nw * 8);
        return BST_OK;
    }
    if (part == 2) {
        if (c.layout != BST_BITPACKED) return set_error(BST_EINVAL, "not a Bit-Packed column");
        const uint32_t w = c.width;
        uint64_t nw = (n * w + 63) / 64;
        *bytes = nw * 8;
        if (!out) return BST_OK;
        uint64_t* o = (uint64_t*)out;
        memset(o, 0, nw * 8);
        const uint32_t* pk = reinterpret_cast<const uint32_t*>(c.buf[BST_BUF_PACKED].data());
        for (uint64_t r = 0; r < n; ++r) {
            uint64_t t = r / kTileRows, lane = r & 63, k = (r >> 6) & 31;
            uint64_t bit = k * w;
            uint64_t i = bit >> 5, sh = bit & 31;
            const uint32_t* base = pk + t * 64 * w;
            uint64_t win = base[i * 64 + lane];
            if (sh + w > 32) win |= (uint64_t)base[(i + 1) * 64 + lane] << 32;
            uint64_t code = (win >> sh) & ((w == 64) ? ~0ull : ((1ull << w) - 1));
            uint64_t sb = r * w;
            o[sb >> 6] |= code << (sb & 63);
            if ((sb & 63) + w > 64) o[(sb >> 6) + 1] |= code >> (64 - (sb & 63));
        }
        return BST_OK;
    }
    return set_error(BST_EINVAL, "bad part");
}

// ---- advisor host arithmetic (Algorithm 5) --------------------------------
int bst_profile_literals(const bst_dict* dd, int op, int count, uint32_t* lits, double* sels) {
    if (!dd || count < 1 || !lits) return set_error(BST_EINVAL, "bad argument");
    const Dict& d = dd->d;
    const uint64_t nd = d.A.size();
    if (nd == 0) return set_error(BST_EINVAL, "empty column");
    const double n = (double)d.n;
    if (op == BST_LT) {
        // '<' selectivity of A_k is (rows below A_k) / n; pick the nearest to each target
        std::vector<uint64_t> below(nd);
        uint64_t acc = 0;
        for (uint64_t k = 0; k < nd; ++k) {
            below[k] = acc;
            acc += d.Q[k];
        }
        for (int i = 1; i <= count; ++i) {
            double target = (i - 0.5) / count;
            // first k with below[k]/n >= target, then compare with its left neighbour
            uint64_t lo = 0, hi = nd;
            while (lo < hi) {
                uint64_t mid = (lo + hi) / 2;
                if ((double)below[mid] / n >= target) hi = mid; else lo = mid + 1;
            }
            uint64_t best = lo < nd ? lo : nd - 1;
            if (lo > 0) {
                double dl = std::fabs((double)below[lo - 1] / n - target);
                double dr = lo < nd ? std::fabs((double)below[lo] / n - target) : 1e300;
                if (dl <= dr) best = lo - 1;
            }
            lits[i - 1] = d.A[best];
            if (sels) sels[i - 1] = (double)below[best] / n;
        }
        return BST_OK;
    }
    if (op == BST_EQ) {
        std::vector<uint32_t> ord(nd);
        std::iota(ord.begin(), ord.end(), 0u);
        std::stable_sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) { return d.Q[a] > d.Q[b]; });
        for (int i = 0; i < count; ++i) {
            uint64_t pos = (count == 1) ? 0 : (uint64_t)std::llround((double)i * (double)(nd - 1) / (double)(count - 1));
            uint32_t k = ord[pos];
            lits[i] = d.A[k];
            if (sels) sels[i] = (double)d.Q[k] / n;
        }
        return BST_OK;
    }
    return set_error(BST_EINVAL, "profiling op must be BST_LT or BST_EQ");
}

int bst_auc(const double* s, const double* t, int n, double* out) {
    if (!out || n < 0 || (n && (!s || !t))) return set_error(BST_EINVAL, "bad argument");
    std::vector<std::pair<double, double>> pts;
    pts.reserve((size_t)n);
    for (int i = 0; i < n; ++i) pts.push_back({s[i], t[i]});
    std::sort(pts.begin(), pts.end(), [](auto& a, auto& b) { return a.first < b.first; });
    std::vector<double> xs, ys;
    for (size_t i = 0; i < pts.size();) {
        size_t j = i;
        double sum = 0;
        while (j < pts.size() && pts[j].first == pts[i].first) sum += pts[j++].second;
        xs.push_back(pts[i].first);
        ys.push_back(sum / (double)(j - i));
        i = j;
    }
    if (xs.size() < 2) {
        double m = 0;
        for (double y : ys) m += y;
        *out = ys.empty() ? 0.0 : m / (double)ys.size();
        return BST_OK;
    }
    double a = 0;
    for (size_t i = 1; i < xs.size(); ++i) a += (xs[i] - xs[i - 1]) * (ys[i] + ys[i - 1]) * 0.5;
    *out = a;
    return BST_OK;
}

int bst_choose(const int* layouts, const double* aucs, int n, int* chosen) {
    if (!layouts || !aucs || !chosen || n < 1) return set_error(BST_EINVAL, "bad argument");
    static const int pref[3] = {BST_BYTESLICE, BST_PPVBS, BST_BITPACKED};
    int best = -1;
    for (int p = 0; p < 3; ++p)
        for (int i = 0; i < n; ++i)
            if (layouts[i] == pref[p] && (best < 0 || aucs[i] < aucs[best])) best = i;
    for (int i = 0; i < n; ++i)   // layouts outside the three known ones come last
        if (best < 0) best = i;
    *chosen = best;
    return BST_OK;
}

}  // extern "C"
