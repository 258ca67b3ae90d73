// Internal definitions shared by the host encoder and the HIP kernels.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/bytestore.h"

namespace bst {

constexpr uint32_t kTileRows = BST_TILE_ROWS;   // rows per tile (32 groups of 64)
constexpr uint32_t kGroupsPerTile = kTileRows / 64;
constexpr uint32_t kLeafFlag = 0x80000000u;     // decode-table child entry is a leaf
// With fewer than 2^28 distinct values a leaf entry also carries, in bits 28-30,
// the digits its slot numbers take (so the length of every code below it).
constexpr uint32_t kLeafDigitsShift = 28;
constexpr uint64_t kLeafDigitsMaxValues = 1ull << 28;
constexpr uint32_t kDefaultDirStride = 512;

// Error reporting (thread-local message behind bst_last_error()).
int set_error(int code, const std::string& msg);

// ---------------------------------------------------------------- host side
struct Dict {
    uint64_t n = 0;
    std::vector<uint32_t> A;     // sorted distinct values
    std::vector<uint64_t> Q;     // their counts
    std::vector<uint32_t> rank;  // per row
};

struct HostColumn {
    uint32_t layout = 0, width = 0, K = 1, dir_stride = kDefaultDirStride, domain_mode = 0;
    uint32_t categorical = 0;        // PP-VBS codes from Algorithm 2; dict then in code order
    uint64_t n = 0, nd = 0, ntiles = 0;
    bool codes_only = false;
    std::vector<uint32_t> dict;      // sorted distinct values (dictionary mode, PP-VBS)
    std::vector<uint64_t> code;      // per distinct value: code (PP-VBS unpadded, else fixed)
    std::vector<uint8_t> clen;       // per distinct value: code length in bytes
    std::vector<uint8_t> buf[BST_NBUF];
    uint64_t rows_by_len[BST_KMAX + 1] = {0};
    uint64_t rows_end_by_mask[BST_KMAX + 1] = {0};   // rows whose lookup reads M_{len+1}
    uint32_t trie_root = kLeafFlag;
    uint32_t leaf_digits = 0;        // leaf entries carry their slot digits (kLeafDigitsShift)
};

// A literal in code space as the kernels take it.
struct ScanLit {
    int32_t mode;        // see LitMode
    int32_t negate;      // result = valid & ~X instead of X
    uint64_t lo, hi;     // slice layouts: codes padded to BST_KMAX bytes; Bit-Packed: plain codes
    uint32_t llo, lhi;   // code lengths in bytes (slice layouts)
    uint32_t gather;     // pending rows per 32-row lane a level gathers directly (0..4);
                         // a tile with a lane holding more stages the level's run in LDS
    uint32_t pad;
};

enum LitMode : int32_t {
    kModeNone = 0,     // no row passes
    kModeAll = 1,      // every (in_mask) row passes
    kModeLT = 2,       // X = rows with code <  lo
    kModeGT = 3,       // X = rows with code >  lo
    kModeEQ = 4,       // X = rows with code == lo
    kModeBetween = 5,  // X = rows with lo <= code <= hi
};

// Rewrite a value predicate into code space for a column (host, exact).
int rewrite_predicate(const HostColumn& c, const bst_pred& p, ScanLit* out);
// Set ScanLit.gather: a level gathers each pending row's byte straight from the
// slice while no 32-row lane of the tile has more than `rows` (0..4) pending
// rows, and otherwise copies the tile's run of BS_j into LDS with one read.
void choose_gather(ScanLit* s, int rows);
// Literal from explicit codes (op in code space).
int code_literal(const HostColumn& c, int op, uint64_t lo, uint32_t llo, uint64_t hi, uint32_t lhi,
                 ScanLit* out);

// ---------------------------------------------------------------- device side
struct DevCol {
    uint32_t layout, width, K, dir_shift;
    uint32_t domain_mode, trie_root;
    uint32_t categorical;                // Algorithm 2 codes: decode arithmetically, dict by frequency
    uint32_t leaf_digits;                // trie leaf entries carry their slot digits
    uint64_t n, ntiles;
    const uint8_t* bs[BST_KMAX + 1];     // bs[1..K]
    const uint64_t* m[BST_KMAX + 1];     // m[2..K]
    const uint32_t* dir[BST_KMAX + 1];   // dir[2..K]
    const uint32_t* packed;
    const uint32_t* dict;
    const uint32_t* trie;                // pairs {slot rank, child}, 256 per node
};

}  // namespace bst

struct bst_dict {
    bst::Dict d;
};
struct bst_host_column {
    bst::HostColumn c;
};
struct bst_column {
    const bst_host_column* hc;
    const bst::HostColumn* host;
    bst::DevCol dev;
    int device;
};
