/*
 * bytestore.h -- C ABI of the MI355X (gfx950) ByteStore scan / lookup library.
 *
 * ByteStore (arXiv 2209.00220) stores each dictionary-encoded column in the
 * layout that scans it fastest: PP-VBS (prefix-preserving variable byte
 * slice, Sec. 3), ByteSlice (Sec. 2.5) or Bit-Packed (Sec. 2.3), chosen per
 * column by an experiment-driven advisor (Sec. 4, Algorithm 5).  The two
 * operations on a stored column are the scan, which turns a predicate into a
 * result bitvector, and the lookup, which returns plain values of selected
 * rows (Sec. 2.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns an int status: BST_OK (0) or a negative BST_E*
 *   code.  bst_last_error() returns a thread-local message for the last
 *   failure on the calling thread.  No C++ exception crosses this boundary.
 * - The library never allocates device memory.  Device buffers (layout
 *   buffers, bitvectors, row IDs, outputs, workspaces) are allocated by the
 *   caller and passed as plain device pointers; their required sizes come
 *   from the *_bytes / info functions.  Host objects (bst_dict,
 *   bst_host_column, bst_column, bst_batch) are library-owned and freed by
 *   their *_free function.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Device work is enqueued asynchronously on it; results are valid after
 *   the caller synchronises the stream.
 * - Argument errors are reported synchronously.  Errors only the device can
 *   see (a row ID past the end, an output capacity exceeded) are OR-ed into
 *   the caller's 32-bit device word *dev_status (bits BST_DEV_*), which the
 *   caller clears beforehand and reads after synchronising; dev_status may be
 *   NULL where noted.
 * - Bitvectors are arrays of ceil(n_rows / 64) uint64 words, LSB first: row
 *   r is bit r % 64 of word r / 64.  Bits past the last row are written 0.
 * - Row IDs are uint32 (n_rows < 2^32); values are uint32 compared unsigned.
 */
#ifndef BYTESTORE_H
#define BYTESTORE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define BST_OK 0
#define BST_EINVAL (-1)       /* bad argument (NULL pointer, bad enum, size) */
#define BST_ENOMEM (-2)       /* host allocation failed                      */
#define BST_EHIP (-3)         /* a HIP runtime call failed                   */
#define BST_ERANGE (-4)       /* value out of the column's domain or limits  */
#define BST_EUNSUPPORTED (-5) /* operation not defined for this layout       */

/* ---- asynchronous device status bits ---------------------------------- */
#define BST_DEV_BAD_ROW 1u  /* a row ID >= n_rows was looked up (its output is 0) */
#define BST_DEV_OVERFLOW 2u /* more selected rows than the output capacity        */

/* ---- layouts, operators, limits --------------------------------------- */
typedef enum {
    BST_BITPACKED = 0,
    BST_BYTESLICE = 1,
    BST_PPVBS = 2,
    /* PP-VBS over the categorical PPE of Algorithm 2 (Sec. 3.1): codes follow
     * descending frequency, not value order, so only '=' and '!=' scans apply
     * (other operators return BST_EINVAL).  Accepted by the encode calls; the
     * column then reports layout BST_PPVBS with categorical = 1. */
    BST_PPVBS_CATEGORICAL = 3
} bst_layout;

/* Sec. 2.2: scans take =, !=, >, <, <=, >= and BETWEEN (lo <= v <= hi). */
typedef enum {
    BST_LT = 0, BST_LE = 1, BST_GT = 2, BST_GE = 3, BST_EQ = 4, BST_NE = 5, BST_BETWEEN = 6
} bst_op;

/* A predicate on plain values: `v op lo`, or lo <= v <= hi for BETWEEN. */
typedef struct {
    int32_t op;
    uint32_t lo;
    uint32_t hi;
} bst_pred;

#define BST_KMAX 6          /* longest PP-VBS code in bytes (2 levels + 4-byte leaf) */
#define BST_TILE_ROWS 2048  /* rows per tile of the device layouts                   */
#define BST_BATCH_ROUND_ROBIN 0xFFFFFFFFu /* tiles_per_grab: static round-robin tiles */

/* Device buffer slots of a stored column (bst_column_info.bytes[slot]). */
enum {
    BST_BUF_BS1 = 0,     /* byte slice 1, tile-interleaved (PP-VBS, ByteSlice)      */
    BST_BUF_BS2 = 1,     /* byte slices 2..6 (slot BST_BUF_BS2 + j - 2)            */
    BST_BUF_M2 = 6,      /* PP-VBS bitmasks M_2..M_6, uint64 words (slot + j - 2)   */
    BST_BUF_DIR2 = 11,   /* PP-VBS directories for BS_2..BS_6, uint32 (slot + j - 2) */
    BST_BUF_PACKED = 16, /* Bit-Packed words, uint32, lane-interleaved              */
    BST_BUF_DICT = 17,   /* sorted distinct values, uint32 (dictionary mode)        */
    BST_BUF_TRIE = 18,   /* PP-VBS decode tables, uint32                            */
    BST_NBUF = 19
};

typedef struct bst_dict bst_dict;               /* host: sorted distinct values + ranks */
typedef struct bst_host_column bst_host_column; /* host: one encoded layout             */
typedef struct bst_column bst_column;           /* a layout resident in device memory   */
typedef struct bst_batch bst_batch;             /* a prepared batch of scans            */

typedef struct {
    uint32_t layout;      /* bst_layout                                            */
    uint32_t width_bits;  /* fixed code width (ByteSlice, Bit-Packed)              */
    uint32_t k_max;       /* bytes of the longest code (slices used)               */
    uint32_t dir_stride;  /* rows per PP-VBS directory entry                       */
    uint32_t domain_mode; /* 1: code = value; 0: code = dictionary rank / PPE code */
    uint32_t categorical; /* 1: PP-VBS codes from Algorithm 2 (= and != only)        */
    uint64_t n_rows;
    uint64_t n_distinct;
    uint64_t bytes[BST_NBUF];          /* device bytes each slot needs (0 = unused) */
    uint64_t total_bytes;              /* sum of bytes[]                            */
    uint64_t rows_by_len[BST_KMAX + 1]; /* PP-VBS: rows whose code has exactly j bytes */
    uint64_t layout_bytes;             /* bytes of the layout proper (slices, masks,
                                          directories, packed words)                */
    uint64_t rows_end_by_mask[BST_KMAX + 1]; /* PP-VBS: of rows_by_len[j] (j < k_max),
                                          the rows whose code length a lookup learns
                                          only by reading M_{j+1}; the others end in
                                          a decode-table leaf that fixes the length */
} bst_column_info;

/* ---- diagnostics -------------------------------------------------------- */
const char* bst_last_error(void);
int bst_version(void);
/* Number of visible HIP devices (0 when none); never fails. */
int bst_device_count(void);

/* ---- dictionary (Sec. 2.2: order-preserving dictionary) ---------------- */
/*
 * Build the dictionary of a column: its distinct values A_0 < ... < A_{d-1},
 * their counts Q_i (the input of Algorithm 1) and each row's rank.  `values`
 * (n host uint32) is copied; n < 2^32.  n_threads 0 = all host cores.
 * Errors: BST_EINVAL (values NULL with n > 0, n >= 2^32), BST_ENOMEM.
 */
int bst_dict_build(const uint32_t* values, uint64_t n, uint32_t n_threads, bst_dict** out);
void bst_dict_free(bst_dict* d);
int bst_dict_info(const bst_dict* d, uint64_t* n_rows, uint64_t* n_distinct);
/* Copy the sorted distinct values and/or their counts (either pointer may be NULL). */
int bst_dict_values(const bst_dict* d, uint32_t* values_out, uint64_t* counts_out);

/* ---- encoding (Sec. 2.3, 2.5, 3.1-3.2; Algorithm 1) --------------------- */
/*
 * Encode the dictionary's column into one layout, in host memory.
 *  layout BST_PPVBS   : Algorithm 1 (PPE for numerical columns) over the
 *                       distinct values, stored as VBS: BS_1 for every row,
 *                       BS_j / M_j (j >= 2) only for codes with a j-th byte,
 *                       a directory of running BS_j positions every
 *                       dir_stride rows and the decode tables.  `width` unused.
 *  layout BST_BYTESLICE: fixed w-bit codes, ceil(w/8) byte slices, left-aligned.
 *  layout BST_BITPACKED: fixed w-bit codes packed back to back.
 *  width 0 selects dictionary mode (code = rank, w = bits for d ranks); width
 *  w in [1, 32] selects domain mode (code = value; every value must be < 2^w,
 *  else BST_ERANGE).
 *  dir_stride: 0 = default (512); else a power of two in [64, 2048].
 * Errors: BST_EINVAL, BST_ERANGE, BST_ENOMEM.
 */
int bst_encode(const bst_dict* d, int layout, uint32_t width, uint32_t dir_stride,
               uint32_t n_threads, bst_host_column** out);
/* Convenience: bst_dict_build + bst_encode + bst_dict_free. */
int bst_encode_host(const uint32_t* values, uint64_t n, int layout, uint32_t width,
                    bst_host_column** out);
/*
 * Test support: a PP-VBS column from explicit per-row codes (codes[r] is an
 * unpadded code of lengths[r] in [1, k_max] bytes), bypassing Algorithm 1, for
 * the worked examples of Sec. 3.3.  The column's "values" are the ranks of the
 * distinct padded codes.  Codes must satisfy the prefix rule (a code that is a
 * proper prefix of another leaves a non-zero remainder), else BST_EINVAL.
 */
int bst_encode_codes(const uint64_t* codes, const uint8_t* lengths, uint64_t n, uint32_t k_max,
                     bst_host_column** out);
void bst_free_host(bst_host_column* c);
int bst_host_info(const bst_host_column* c, bst_column_info* info);
/*
 * Per distinct value i (dictionary order): its code and code length in bytes
 * (PP-VBS: the Algorithm 1 code, unpadded; ByteSlice / Bit-Packed: the fixed
 * code).  Arrays of n_distinct entries; either may be NULL.
 */
int bst_host_code_table(const bst_host_column* c, uint64_t* codes, uint8_t* lengths);
/*
 * The layout in the paper's row order, for inspection:
 *  part 0, j in [1, k_max]: byte slice BS_j (n bytes; PP-VBS j >= 2: one byte per
 *          row that has a j-th byte, in row order);
 *  part 1, j in [2, k_max]: PP-VBS bitmask M_j as ceil(n/64) uint64 words;
 *  part 2, j = 0: Bit-Packed LSB-first stream as ceil(n*w/64) uint64 words.
 * `out` NULL returns the byte count in *bytes.
 */
int bst_host_paper_view(const bst_host_column* c, int part, int j, void* out, uint64_t* bytes);

/* ---- residency --------------------------------------------------------- */
/*
 * Copy a host column into caller-allocated device buffers (dev_bufs[slot] of
 * at least info.bytes[slot] bytes, 16-byte aligned; unused slots may be NULL)
 * with hipMemcpyAsync on `stream`, and return a handle that pairs the device
 * pointers with the host metadata used to rewrite literals.  The host column
 * must outlive the handle; the device buffers stay owned by the caller.
 * Errors: BST_EINVAL for a missing or misaligned buffer.
 */
int bst_upload(const bst_host_column* c, void* const dev_bufs[BST_NBUF], void* stream,
               bst_column** out);
void bst_column_free(bst_column* col);
int bst_column_info_get(const bst_column* col, bst_column_info* info);

/* ---- scan (Sec. 2.2, Sec. 3.3 / Algorithm 3, Lemma 1) ------------------ */
/*
 * out_bv[r] = in_mask[r] AND (value_r op literal), bit-exact, for all rows.
 * The value literal is rewritten on the host into the column's code space
 * (order-preserving codes, Sec. 2.2); literals absent from the dictionary are
 * handled through the neighbouring codes, and always-true / always-false
 * predicates become a fill.  in_mask NULL = all rows (predicate pipelining,
 * Sec. 3.3: pass the previous scan's result).  out_bv: ceil(n/64) words,
 * may alias in_mask.  Errors: BST_EINVAL (bad op, NULL out_bv with n > 0).
 */
int bst_scan(const bst_column* col, bst_pred pred, const uint64_t* in_mask, uint64_t* out_bv,
             uint32_t* dev_status, void* stream);
/*
 * Scan with literals already in code space (the form Algorithm 3 takes):
 * PP-VBS / ByteSlice: code_lo / code_hi are codes of len_lo / len_hi bytes,
 * compared as if zero-padded (Sec. 3.1); Bit-Packed: plain w-bit codes
 * (lengths ignored).  code_hi / len_hi only for BETWEEN.
 */
int bst_scan_codes(const bst_column* col, int op, uint64_t code_lo, uint32_t len_lo,
                   uint64_t code_hi, uint32_t len_hi, const uint64_t* in_mask,
                   uint64_t* out_bv, void* stream);
/*
 * Instrumented scan: same result as bst_scan, and adds to dev_counters[0..4]
 * (uint64, device): [0] algorithmic bytes (slice bytes, mask words and
 * bitvector words the early-stopping scan must touch, counted per 64-row
 * group), [1] code bytes examined summed over rows (Lemma 1 bounds each row by
 * min(l(v), l(c))), [2] 64-row groups that needed a byte beyond BS_1,
 * [3] bytes a scan without early stop would touch, [4] the bytes of [0] at
 * 128-byte granularity: 128 x the lines (by offset in their buffer) that hold
 * them, each line counted once per tile and level.
 */
int bst_scan_stats(const bst_column* col, bst_pred pred, const uint64_t* in_mask,
                   uint64_t* out_bv, uint64_t* dev_counters, void* stream);

/* ---- lookup (Sec. 2.2, Sec. 3.3 / Algorithm 4) ------------------------- */
/*
 * out_values[i] = value of row row_ids[i], i < m (device arrays).  A row ID
 * >= n_rows yields 0 and sets BST_DEV_BAD_ROW in *dev_status (may be NULL).
 */
int bst_lookup(const bst_column* col, const uint32_t* row_ids, uint64_t m, uint32_t* out_values,
               uint32_t* dev_status, void* stream);
/*
 * Lookup by a device-resident row-ID list whose length is itself on the device
 * (as bst_bv_compact leaves it): out_values[i] = value of row row_ids[i] for
 * i < *dev_count, when *dev_count <= cap.  So the IDs of one compaction serve
 * lookups of several columns of the same rows with no host read of the count.
 * All or nothing: when *dev_count > cap nothing is written and BST_DEV_OVERFLOW
 * is set in *dev_status (may be NULL); the caller looks up again with a cap
 * of at least the count.  A row ID >= n_rows yields 0 and sets BST_DEV_BAD_ROW.
 */
int bst_lookup_counted(const bst_column* col, const uint32_t* row_ids, const uint64_t* dev_count, uint64_t cap,
                       uint32_t* out_values, uint32_t* dev_status, void* stream);
/* Workspace bytes bst_bv_compact / bst_lookup_bv need for n_rows rows. */
uint64_t bst_compact_workspace_bytes(uint64_t n_rows);
/*
 * Row IDs of the set bits of bv in ascending order (Sec. 3.3, the outer loop of
 * Algorithm 4): out_ids[0..count) with count = popcount(bv) written to
 * *dev_count (device uint64).  Writes at most cap IDs; more sets
 * BST_DEV_OVERFLOW.  workspace: bst_compact_workspace_bytes(n_rows) bytes.
 */
int bst_bv_compact(const uint64_t* bv, uint64_t n_rows, uint32_t* out_ids, uint64_t cap,
                   uint64_t* dev_count, void* workspace, uint32_t* dev_status, void* stream);
/*
 * Lookup driven by a result bitvector (the paper's lookup input): the values
 * of the selected rows in ascending row order, count in *dev_count.  ids_tmp:
 * device uint32[cap] for the row IDs; workspace as for bst_bv_compact.
 */
int bst_lookup_bv(const bst_column* col, const uint64_t* bv, uint32_t* out_values, uint64_t cap,
                  uint64_t* dev_count, uint32_t* ids_tmp, void* workspace, uint32_t* dev_status,
                  void* stream);

/*
 * bst_lookup_bv without caller-provided device memory, for callers that cannot
 * allocate (code under stream capture, tight serving loops, hosts that forbid
 * allocation): the compaction workspace and the row-ID staging live in a device
 * array the library holds per GPU (8.4 MB, reserved on that GPU until the
 * process ends).  The caller passes only inputs and outputs, as for
 * bst_lookup_bv.  Limits: columns of at most bst_lookup_bv_static_max_rows()
 * rows (2^29) and cap at most bst_lookup_bv_static_max_ids() (2^21); larger
 * ones return BST_ERANGE.  The array belongs to the current device, and every
 * call on one GPU shares it: calls whose work overlaps on one GPU (other
 * streams, other host threads) race and must be ordered by the caller.
 */
int bst_lookup_bv_static(const bst_column* col, const uint64_t* bv, uint32_t* out_values, uint64_t cap,
                         uint64_t* dev_count, uint32_t* dev_status, void* stream);
uint64_t bst_lookup_bv_static_max_rows(void);
uint64_t bst_lookup_bv_static_max_ids(void);

/* ---- bitvector helpers (Sec. 2.2: conjunctions and disjunctions of scan
 * results are bitwise operations on their bitvectors) ----------------------
 * All take ceil(n_rows/64) device words per vector, write `out` (which may
 * alias an input) with the bits past n_rows cleared, and return BST_EINVAL for
 * a NULL pointer when n_rows > 0. */
int bst_bv_and(const uint64_t* a, const uint64_t* b, uint64_t* out, uint64_t n_rows, void* stream);
int bst_bv_or(const uint64_t* a, const uint64_t* b, uint64_t* out, uint64_t n_rows, void* stream);
/* out = a AND NOT b */
int bst_bv_andnot(const uint64_t* a, const uint64_t* b, uint64_t* out, uint64_t n_rows, void* stream);
/* out = NOT a (within the first n_rows) */
int bst_bv_not(const uint64_t* a, uint64_t* out, uint64_t n_rows, void* stream);
/* *dev_count (device uint64) = number of set bits among the first n_rows. */
int bst_bv_popcount(const uint64_t* bv, uint64_t n_rows, uint64_t* dev_count, void* stream);

/* ---- layout advisor (Sec. 4, Algorithm 5) ------------------------------ */
/*
 * The profiling literals of Algorithm 5, chosen from the dictionary so their
 * selectivities span the feasible range: op BST_LT (numerical columns): for
 * i = 1..count the distinct value whose '<' selectivity is nearest
 * (i - 0.5)/count; op BST_EQ (categorical): count values evenly spaced in
 * descending-frequency order.  lits_out / sels_out: count entries each.
 */
int bst_profile_literals(const bst_dict* d, int op, int count, uint32_t* lits_out,
                         double* sels_out);
/* Area under the piecewise-linear time-vs-selectivity curve (duplicates averaged). */
int bst_auc(const double* sels, const double* times, int n, double* auc_out);
/* Index of the smallest area among n candidates; ties prefer ByteSlice, then PP-VBS,
   then Bit-Packed (Algorithm 5 keeps ByteSlice when its area is not larger). */
int bst_choose(const int* layouts, const double* aucs, int n, int* chosen);
/*
 * Algorithm 5 for one column: time `op` scans with each literal on every
 * candidate (the same column resident in different layouts), `repeats` times
 * each on `stream` with HIP events (median kept), integrate time over
 * selectivity and choose.  scratch_bv: ceil(n/64) device words.
 * times_out: n_cand * n_lit microseconds (may be NULL); auc_out: n_cand.
 */
int bst_advise(const bst_column* const* cands, int n_cand, int op, const uint32_t* lits,
               const double* sels, int n_lit, int repeats, uint64_t* scratch_bv,
               double* times_out, double* auc_out, int* chosen, void* stream);

/* ---- batched scans (many predicates over many columns, one launch) ----- */
/* Device workspace bytes for a batch of n_items scans. */
uint64_t bst_batch_workspace_bytes(int n_items);
/*
 * Prepare scans item i: cols[i] with preds[i], optional in_masks[i] (NULL
 * entry or NULL array = none), writing outs[i].  Literals are rewritten on the
 * host and the work list (item, tile) is uploaded into `workspace` on the
 * first launch, by an asynchronous copy from a pinned staging ring that the
 * library allocates once (8 MiB) and keeps until the process ends; the launch
 * does not wait for the stream.  The arrays are copied; columns, `workspace`
 * and the device buffers must stay alive until the launched work has run.
 */
int bst_batch_prepare(const bst_column* const* cols, const bst_pred* preds,
                      const uint64_t* const* in_masks, uint64_t* const* outs, int n_items,
                      void* workspace, bst_batch** out);
/*
 * Run every scan of the batch.  An item of at least BST_TUNE_BATCH_SOLO_TILES
 * tiles (as set when the batch was prepared) runs as the single-column scan
 * launch would run it.  The other items are grouped by kernel variant (layout,
 * operator or code width, one-byte literal, incoming mask), and each group is
 * one persistent launch of up to `grid` workgroups (0 = tuned default; never
 * more waves than the group has tiles) whose waves take at least
 * `tiles_per_grab` (0 = tuned default) consecutive 2048-row tiles at a time
 * from the group's queue -- more when the group is large, so that a wave takes
 * about four times per group; a group too small to give every wave
 * `tiles_per_grab` tiles is spread evenly over its waves instead.
 * tiles_per_grab = BST_BATCH_ROUND_ROBIN takes no counter: the group's tiles
 * (its items' tiles concatenated) go round robin over the launch's waves, so
 * each item is read as a single-column scan reads it.  With
 * BST_TUNE_BATCH_STREAMS = s > 1 the launches are spread over s streams (largest
 * first, to the least loaded): helper streams of the library fork off
 * `stream` after the counter reset and join back into it before the call
 * returns, so later work on `stream` still sees every result; such launches
 * (and captures) from several host threads on one device take turns on the
 * helper streams.  The items must be independent (no item's incoming mask is
 * another item's output).  With
 * use_graph != 0 the launch sequence is captured once into a HIP graph (the
 * streams become parallel branches) and replayed on later calls with the same
 * grid, grab size and stream count.  Errors: BST_EINVAL for a NULL batch,
 * BST_EHIP for a failed launch or capture.
 */
int bst_batch_launch(bst_batch* b, uint32_t grid, uint32_t tiles_per_grab, int use_graph,
                     void* stream);
void bst_batch_free(bst_batch* b);

/* ---- measurement ------------------------------------------------------- */
/*
 * Streaming probe, a measurement aid rather than an operation of the paper:
 * read `bytes` of `src` (a multiple of 2048) in 2048-byte tiles and write
 * bytes/8 to `dst` (both device memory, 16-byte aligned), with the launch
 * shape, tile layout and cache policies of the slice scans.  That is the
 * traffic of a scan in which byte 1 settles every row (Sec. 3.3's early stop
 * at its best) without the compares, so its rate bounds what such a scan can
 * reach on this chip.  Errors: BST_EINVAL for a NULL pointer, a size that is
 * not a multiple of 2048 or a misaligned buffer.
 */
int bst_stream_probe(const void* src, uint64_t bytes, void* dst, void* stream);

/* ---- launch tuning ----------------------------------------------------- */
enum {
    BST_TUNE_SCAN_GRID = 0,    /* workgroups of a single-column scan launch (0 = auto) */
    BST_TUNE_LOOKUP_GRID = 1,  /* workgroups of a lookup launch (0 = auto)             */
    BST_TUNE_BATCH_GRID = 2,   /* default workgroups of a batch launch (0 = auto)      */
    BST_TUNE_BATCH_GRAB = 3,   /* default tiles per grab of a batch launch             */
    BST_TUNE_GATHER_ROWS = 4,  /* pending rows per 32-row lane (0..4, default 4) whose
                                  later bytes a scan gathers one by one; a tile with
                                  a lane holding more copies the level's run of the
                                  slice into LDS with one read instead                */
    BST_TUNE_BATCH_STREAMS = 5,/* streams a batch's groups are spread over (1..4,
                                  default 1): the caller's stream and library-owned
                                  helper streams forked from it and joined back   */
    BST_TUNE_BATCH_SOLO_TILES = 6, /* batch items of at least this many 2048-row tiles
                                  (read when a batch is prepared; >= 1, default
                                  16384) run as single-column scan launches with
                                  their own launch shape instead of joining a
                                  persistent group launch                          */
    BST_TUNE_NKEYS = 7
};
/* Tuning values are process-wide, read when a launch is enqueued (the solo
 * threshold when a batch is prepared); set them while no other host thread
 * launches.  bst_tune_set: BST_EINVAL for an unknown key or a value out of
 * range; bst_tune_get: -1 for an unknown key. */
int bst_tune_set(int key, int64_t value);
int64_t bst_tune_get(int key);

#ifdef __cplusplus
}
#endif
#endif /* BYTESTORE_H */
