// Batched scans: many predicates over many columns in one persistent launch.
#include <vector>

#include "device_common.h"

using namespace bst;
using namespace bst::dev;

namespace bst {
namespace dev {

// Each layout / operator / width variant is its own out-of-line function, so
// the dispatching kernel stays small and every variant is compiled on its own.
template <int MODE, bool DENSE, bool HAS_IN>
__device__ __noinline__ void batch_slices_tile(const BatchItem& it, uint64_t t, uint32_t lane, uint8_t* lds) {
    Stats st;
    scan_slices_tile<MODE, DENSE, HAS_IN, false>(it.c, it.lit, it.in_mask, it.out, t, lane, lds, st);
}

template <int W, bool HAS_IN>
__device__ __noinline__ void batch_packed_tile(const BatchItem& it, uint64_t t, uint32_t lane) {
    uint64_t alg = 0;
    scan_packed_tile<W, HAS_IN>(it.c, it.pl, it.in_mask, it.out, t, lane, alg);
}

__device__ __forceinline__ void scan_any_tile(const BatchItem& it, uint64_t t, uint32_t lane, uint8_t* lds) {
    const bool has_in = it.in_mask != nullptr;
    const uint32_t kind = it.kind;
    if (kind < 16) {
        // slice layouts: bit 0 dense (ByteSlice), bits 1..2 literal mode
        const bool dense = kind & 1;
        const int mi = (kind >> 1) & 3;
#define BST_SLICE_CASE(MI, MODE)                                                 \
    if (mi == MI) {                                                              \
        if (dense) {                                                             \
            if (has_in) batch_slices_tile<MODE, true, true>(it, t, lane, lds);       \
            else batch_slices_tile<MODE, true, false>(it, t, lane, lds);             \
        } else {                                                                 \
            if (has_in) batch_slices_tile<MODE, false, true>(it, t, lane, lds);      \
            else batch_slices_tile<MODE, false, false>(it, t, lane, lds);            \
        }                                                                        \
        return;                                                                  \
    }
        BST_SLICE_CASE(0, kModeLT)
        BST_SLICE_CASE(1, kModeGT)
        BST_SLICE_CASE(2, kModeEQ)
        BST_SLICE_CASE(3, kModeBetween)
#undef BST_SLICE_CASE
        return;
    }
    switch (kind - 16) {
#define BST_W(W)                                               \
    case W:                                                    \
        if (has_in) batch_packed_tile<W, true>(it, t, lane);  \
        else batch_packed_tile<W, false>(it, t, lane);        \
        return;
        BST_W(1) BST_W(2) BST_W(3) BST_W(4) BST_W(5) BST_W(6) BST_W(7) BST_W(8)
        BST_W(9) BST_W(10) BST_W(11) BST_W(12) BST_W(13) BST_W(14) BST_W(15) BST_W(16)
        BST_W(17) BST_W(18) BST_W(19) BST_W(20) BST_W(21) BST_W(22) BST_W(23) BST_W(24)
        BST_W(25) BST_W(26) BST_W(27) BST_W(28) BST_W(29) BST_W(30) BST_W(31) BST_W(32)
#undef BST_W
        default:
            return;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_batch(const BatchHeader* __restrict__ hdr,
                                                       const BatchItem* __restrict__ items,
                                                       unsigned long long* __restrict__ counter, uint32_t grab) {
    __shared__ __attribute__((aligned(16))) uint8_t stage[kWavesPerBlock][kStageBytes];
    uint8_t* lds = stage[threadIdx.x >> 6];
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t total = hdr->total_tiles;
    const uint32_t n_items = hdr->n_items;
    for (;;) {
        uint64_t start = 0;
        if (lane == 0) start = atomicAdd(counter, (unsigned long long)grab);
        start = ((uint64_t)uniform((uint32_t)(start >> 32)) << 32) | uniform((uint32_t)start);
        if (start >= total) break;
        const uint64_t stop = std::min<uint64_t>(total, start + grab);
        // item holding `start`: last item with tile0 <= start
        uint32_t lo = 0, hi = n_items - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (items[mid].tile0 <= start) lo = mid; else hi = mid - 1;
        }
        uint32_t cur = lo;
        for (uint64_t gt = start; gt < stop; ++gt) {
            while (cur + 1 < n_items && items[cur + 1].tile0 <= gt) ++cur;
            const BatchItem& it = items[cur];
            scan_any_tile(it, gt - it.tile0, lane, lds);
        }
    }
}

__global__ void k_reset_counter(unsigned long long* counter) {
    if (threadIdx.x == 0) *counter = 0;
}

}  // namespace dev
}  // namespace bst

struct bst_batch {
    std::vector<BatchItem> items;
    BatchHeader hdr;
    std::vector<std::pair<uint64_t*, std::pair<const uint64_t*, int>>> fills;   // (out, (in, all)) for ALL/NONE items
    std::vector<uint64_t> fill_rows;
    void* ws = nullptr;
    bool uploaded = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t graph_grid = 0, graph_grab = 0;
    hipStream_t graph_stream = nullptr;
};

extern "C" {

// ---- batch ---------------------------------------------------------------
uint64_t bst_batch_workspace_bytes(int n_items) {
    if (n_items < 0) return 0;
    return 256 + (uint64_t)n_items * sizeof(BatchItem) + 256;
}

int bst_batch_prepare(const bst_column* const* cols, const bst_pred* preds, const uint64_t* const* in_masks,
                      uint64_t* const* outs, int n_items, void* workspace, bst_batch** out) {
    if (!cols || !preds || !outs || n_items < 1 || !workspace || !out) return set_error(BST_EINVAL, "bad argument");
    bst_batch* b = new (std::nothrow) bst_batch;
    if (!b) return set_error(BST_ENOMEM, "out of host memory");
    b->ws = workspace;
    uint64_t tiles = 0;
    for (int i = 0; i < n_items; ++i) {
        const bst_column* col = cols[i];
        if (!col) {
            delete b;
            return set_error(BST_EINVAL, "NULL column in batch");
        }
        ScanLit lit;
        int rc = rewrite_predicate(*col->host, preds[i], &lit);
        if (rc) {
            delete b;
            return rc;
        }
        const uint64_t* in = in_masks ? in_masks[i] : nullptr;
        if (col->dev.n == 0) continue;
        if (!outs[i]) {
            delete b;
            return set_error(BST_EINVAL, "NULL output in batch");
        }
        if (lit.mode == kModeNone || lit.mode == kModeAll) {
            b->fills.push_back({outs[i], {in, lit.mode == kModeAll ? 1 : 0}});
            b->fill_rows.push_back(col->dev.n);
            continue;
        }
        BatchItem it;
        memset(&it, 0, sizeof(it));
        it.c = col->dev;
        it.lit = lit;
        choose_staging(*col->host, &it.lit, (int)g_tune[BST_TUNE_STAGE_PCT]);
        it.pl = packed_literal(*col->host, lit);
        it.in_mask = in;
        it.out = outs[i];
        it.tile0 = tiles;
        it.kind = batch_kind(col, lit);
        tiles += col->dev.ntiles;
        b->items.push_back(it);
    }
    b->hdr.total_tiles = tiles;
    b->hdr.n_items = (uint32_t)b->items.size();
    *out = b;
    return BST_OK;
}

static int batch_enqueue(bst_batch* b, uint32_t grid, uint32_t grab, hipStream_t st) {
    char* ws = (char*)b->ws;
    BatchHeader* hdr = (BatchHeader*)ws;
    unsigned long long* counter = (unsigned long long*)(ws + 128);
    BatchItem* items = (BatchItem*)(ws + 256);
    for (size_t i = 0; i < b->fills.size(); ++i) {
        int rc = enqueue_fill(b->fills[i].first, b->fills[i].second.first, b->fill_rows[i], b->fills[i].second.second, st);
        if (rc) return rc;
    }
    if (!b->items.empty()) {
        hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, counter);
        hipLaunchKernelGGL(k_scan_batch, dim3(grid), dim3(kBlock), 0, st, (const BatchHeader*)hdr,
                           (const BatchItem*)items, counter, grab);
    }
    return hip_check(hipGetLastError(), "batch launch");
}

int bst_batch_launch(bst_batch* b, uint32_t grid, uint32_t tiles_per_grab, int use_graph, void* stream) {
    if (!b) return set_error(BST_EINVAL, "NULL batch");
    hipStream_t st = (hipStream_t)stream;
    if (grid == 0) grid = g_tune[BST_TUNE_BATCH_GRID] > 0 ? (uint32_t)g_tune[BST_TUNE_BATCH_GRID] : (uint32_t)props().cus * 8;
    if (tiles_per_grab == 0) tiles_per_grab = g_tune[BST_TUNE_BATCH_GRAB] > 0 ? (uint32_t)g_tune[BST_TUNE_BATCH_GRAB] : 4;
    if (!b->uploaded) {
        char* ws = (char*)b->ws;
        int rc = hip_check(hipMemcpyAsync(ws, &b->hdr, sizeof(b->hdr), hipMemcpyHostToDevice, st), "batch upload");
        if (!rc && !b->items.empty())
            rc = hip_check(hipMemcpyAsync(ws + 256, b->items.data(), b->items.size() * sizeof(BatchItem),
                                          hipMemcpyHostToDevice, st), "batch upload");
        if (!rc) rc = hip_check(hipStreamSynchronize(st), "batch upload sync");
        if (rc) return rc;
        b->uploaded = true;
    }
    if (!use_graph) return batch_enqueue(b, grid, tiles_per_grab, st);
    if (!b->exec || b->graph_grid != grid || b->graph_grab != tiles_per_grab) {
        if (b->exec) hipGraphExecDestroy(b->exec);
        if (b->graph) hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        hipStream_t cap;
        int rc = hip_check(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "capture stream");
        if (rc) return rc;
        rc = hip_check(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
        if (!rc) {
            int rc2 = batch_enqueue(b, grid, tiles_per_grab, cap);
            rc = hip_check(hipStreamEndCapture(cap, &b->graph), "end capture");
            if (!rc) rc = rc2;
        }
        if (!rc) rc = hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiate");
        hipStreamDestroy(cap);
        if (rc) return rc;
        b->graph_grid = grid;
        b->graph_grab = tiles_per_grab;
    }
    return hip_check(hipGraphLaunch(b->exec, st), "graph launch");
}

void bst_batch_free(bst_batch* b) {
    if (!b) return;
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    delete b;
}

}  // extern "C"
