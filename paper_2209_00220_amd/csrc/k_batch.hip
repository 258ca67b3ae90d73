// Batched scans: many predicates over many columns in one persistent launch.
#include <algorithm>
#include <deque>
#include <mutex>
#include <vector>

#include "batch_kernel.h"

using namespace bst;
using namespace bst::dev;

namespace bst {
namespace dev {

// Items of one group share a kernel variant (layout, operator or width, incoming
// mask or not); tile0 counts tiles within the group.
constexpr int kBatchGroupsMax = 2 * (16 + 32);   // (16 slice kinds + 32 widths) x with/without incoming mask
constexpr uint64_t kBatchHeaderBytes = 64;          // per group: BatchHeader, then the grab counter at +32

// Zero the groups' grab counters (a fill kernel, so the launch sequence can be
// captured in a graph).
__global__ void k_reset_counters(char* __restrict__ ws, int n_groups) {
    const int g = threadIdx.x;
    if (g < n_groups) *reinterpret_cast<unsigned long long*>(ws + g * kBatchHeaderBytes + 32) = 0;
}


// Kernel of a group: kind (see batch_kind) and whether its items have an incoming mask.
static BatchKernel batch_kernel(uint32_t kind, bool has_in) {
    if (kind < 16) {
        const bool dense = kind & 1;
        const int mi = (kind >> 1) & 3;
        if (kind & 8) return batch_short_kernel(mi, dense, has_in);
        // a '<', '>' or '=' literal that is not one byte is longer (SHORT = 0); a
        // BETWEEN may have one short bound, decided per item (SHORT = -1)
#define BST_K(MODE, SH)                                                                                    \
    return dense ? (has_in ? k_batch_slices<MODE, SH, true, true> : k_batch_slices<MODE, SH, true, false>) \
                 : (has_in ? k_batch_slices<MODE, SH, false, true> : k_batch_slices<MODE, SH, false, false>)
        switch (mi) {
            case 0: BST_K(kModeLT, 0);
            case 1: BST_K(kModeGT, 0);
            case 2: BST_K(kModeEQ, 0);
            default: BST_K(kModeBetween, -1);
        }
#undef BST_K
    }
    return batch_packed_kernel(kind - 16, has_in);
}

}  // namespace dev
}  // namespace bst

// Pinned staging for batch uploads, one ring per process, allocated on first
// use and kept until the process ends.  A launch copies its header and work
// list into the ring and enqueues a true asynchronous copy from there, so the
// host never waits for the stream and can prepare the next batch while the
// device runs this one.  A region is reused only after the event recorded
// behind its copy has completed.
namespace {

constexpr size_t kRingBytes = 8u << 20;
constexpr size_t kRingAlign = 256;

struct UploadRing {
    std::mutex mu;
    char* host = nullptr;
    bool failed = false;
    size_t head = 0;
    struct Span {
        size_t begin, end;
        hipEvent_t ev;
    };
    std::deque<Span> live;   // regions whose copies may still be in flight, in ring order
    std::vector<hipEvent_t> spare;
};

UploadRing& ring() {
    static UploadRing* r = new UploadRing;   // never destroyed: its memory lives until exit
    return *r;
}

// Copy `len` bytes from `src` to device address `dst` on `st` through the ring.
// Returns BST_EHIP (with the message set) on a HIP error; a batch larger than
// the ring, or a ring that could not be allocated, goes through a synchronous
// copy instead.
int ring_upload(void* dst, const void* src, size_t len, hipStream_t st) {
    UploadRing& r = ring();
    std::lock_guard<std::mutex> lock(r.mu);
    if (!r.host && !r.failed) {
        if (hipHostMalloc((void**)&r.host, kRingBytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            r.host = nullptr;
            r.failed = true;
        }
    }
    const size_t need = (len + kRingAlign - 1) / kRingAlign * kRingAlign;
    if (!r.host || need > kRingBytes) {
        int rc = hip_check(hipMemcpyAsync(dst, src, len, hipMemcpyHostToDevice, st), "batch upload");
        if (!rc) rc = hip_check(hipStreamSynchronize(st), "batch upload sync");
        return rc;
    }
    size_t b = r.head;
    if (b + need > kRingBytes) b = 0;
    const size_t e = b + need;
    // retire finished regions, and wait for any that the new region overlaps
    while (!r.live.empty()) {
        UploadRing::Span& o = r.live.front();
        const bool overlaps = o.begin < e && b < o.end;
        if (!overlaps && hipEventQuery(o.ev) != hipSuccess) break;
        if (overlaps) {
            int rc = hip_check(hipEventSynchronize(o.ev), "batch upload wait");
            if (rc) return rc;
        }
        r.spare.push_back(o.ev);
        r.live.pop_front();
    }
    for (const UploadRing::Span& o : r.live)   // a younger region still in the way
        if (o.begin < e && b < o.end) {
            int rc = hip_check(hipEventSynchronize(o.ev), "batch upload wait");
            if (rc) return rc;
        }
    hipEvent_t ev;
    if (!r.spare.empty()) {
        ev = r.spare.back();
        r.spare.pop_back();
    } else {
        int rc = hip_check(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "batch upload event");
        if (rc) return rc;
    }
    memcpy(r.host + b, src, len);
    int rc = hip_check(hipMemcpyAsync(dst, r.host + b, len, hipMemcpyHostToDevice, st), "batch upload");
    if (!rc) rc = hip_check(hipEventRecord(ev, st), "batch upload event");
    if (rc) {
        // the copy may be queued: keep the region reserved until the device is idle
        (void)hipDeviceSynchronize();
        r.spare.push_back(ev);
        return rc;
    }
    r.live.push_back({b, e, ev});
    r.head = e;
    return BST_OK;
}

// Streams on which a batch's groups run side by side, per device: the caller's
// stream plus up to kBatchStreamsMax - 1 helpers (default priority, created
// on first use and kept until the process ends), with the events that fork
// the helpers off the caller's stream and join them back.  Under graph
// capture the fork and join become edges of the graph, so the groups are
// parallel branches of it.
constexpr int kBatchStreamsMax = 4;
constexpr int kMaxDevices = 64;

struct ForkSet {
    hipStream_t helper[kBatchStreamsMax - 1] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kBatchStreamsMax - 1] = {};
    bool ready = false;
    std::mutex use;   // held from the fork to the join: one batch on the helpers at a time
};

int fork_set(ForkSet** out) {
    static std::mutex mu;
    static ForkSet sets[kMaxDevices];
    int dev = 0;
    int rc = hip_check(hipGetDevice(&dev), "batch streams");
    if (rc) return rc;
    if (dev < 0 || dev >= kMaxDevices) return set_error(BST_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(mu);
    ForkSet& f = sets[dev];
    if (!f.ready) {
        rc = hip_check(hipEventCreateWithFlags(&f.fork, hipEventDisableTiming), "batch fork event");
        for (int i = 0; !rc && i < kBatchStreamsMax - 1; ++i) {
            rc = hip_check(hipStreamCreateWithFlags(&f.helper[i], hipStreamNonBlocking), "batch helper stream");
            if (!rc) rc = hip_check(hipEventCreateWithFlags(&f.join[i], hipEventDisableTiming), "batch join event");
        }
        if (rc) return rc;   // a partly built set is completed on the next call
        f.ready = true;
    }
    *out = &f;
    return BST_OK;
}

}  // namespace

struct BatchGroup {
    uint32_t kind;
    bool has_in;
    uint32_t first, count;   // items [first, first + count) of the sorted item list
    uint64_t tiles;
};

struct bst_batch {
    std::vector<BatchItem> items;        // sorted by group
    std::vector<BatchGroup> groups;
    std::vector<BatchItem> solo;         // items launched as single-column scans
    std::vector<std::pair<uint64_t*, std::pair<const uint64_t*, int>>> fills;   // (out, (in, all)) for ALL/NONE items
    std::vector<uint64_t> fill_rows;
    void* ws = nullptr;
    bool uploaded = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint32_t graph_grid = 0, graph_grab = 0;
    int64_t graph_streams = 0;
    hipStream_t graph_stream = nullptr;
    // fork and join events of the captured graph: its own, made before its
    // capture and destroyed after it, never shared with eager launches or other
    // graphs
    std::vector<hipEvent_t> graph_events;
};

// Streams a batch's launches are spread over: the tuned count, at most one per
// unit of work (group launch or solo item).
static int batch_streams(const bst_batch* b) {
    const uint64_t n_units = b->groups.size() + b->solo.size();
    return (int)std::max<uint64_t>(
        1, std::min<uint64_t>(n_units, (uint64_t)std::max<int64_t>(
                                           1, std::min<int64_t>(g_tune[BST_TUNE_BATCH_STREAMS], kBatchStreamsMax))));
}

static void destroy_graph(bst_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    for (hipEvent_t e : b->graph_events) (void)hipEventDestroy(e);
    b->graph_events.clear();
}

extern "C" {

// ---- batch ---------------------------------------------------------------
uint64_t bst_batch_workspace_bytes(int n_items) {
    if (n_items < 0) return 0;
    return (uint64_t)kBatchGroupsMax * kBatchHeaderBytes + (uint64_t)n_items * sizeof(BatchItem);
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
        choose_gather(&it.lit, (int)g_tune[BST_TUNE_GATHER_ROWS]);
        it.pl = packed_literal(*col->host, lit);
        it.in_mask = in;
        it.out = outs[i];
        it.tile0 = tiles;
        it.kind = batch_kind(col, lit);
        if ((int64_t)col->dev.ntiles >= g_tune[BST_TUNE_BATCH_SOLO_TILES]) {
            b->solo.push_back(it);
            continue;
        }
        tiles += col->dev.ntiles;
        b->items.push_back(it);
    }
    // group the items by kernel variant, keeping their order within a group
    std::vector<BatchItem> sorted;
    sorted.reserve(b->items.size());
    std::vector<bool> used(b->items.size(), false);
    for (size_t i = 0; i < b->items.size(); ++i) {
        if (used[i]) continue;
        BatchGroup g{b->items[i].kind, b->items[i].in_mask != nullptr, (uint32_t)sorted.size(), 0, 0};
        for (size_t j = i; j < b->items.size(); ++j) {
            if (used[j] || b->items[j].kind != g.kind || (b->items[j].in_mask != nullptr) != g.has_in) continue;
            used[j] = true;
            BatchItem it = b->items[j];
            it.tile0 = g.tiles;
            g.tiles += it.c.ntiles;
            sorted.push_back(it);
            ++g.count;
        }
        if (!batch_kernel(g.kind, g.has_in)) {
            delete b;
            return set_error(BST_EINVAL, "no batch kernel for this column");
        }
        b->groups.push_back(g);
    }
    b->items.swap(sorted);
    (void)tiles;
    *out = b;
    return BST_OK;
}

// Enqueue the batch on `st`.  events: the fork event and ns - 1 join events to
// use (a graph capture brings its own), or nullptr for the device's shared set.
static int batch_enqueue(bst_batch* b, uint32_t grid, uint32_t grab, hipStream_t st, const hipEvent_t* events) {
    char* ws = (char*)b->ws;
    const BatchItem* items = (const BatchItem*)(ws + (uint64_t)kBatchGroupsMax * kBatchHeaderBytes);
    for (size_t i = 0; i < b->fills.size(); ++i) {
        int rc = enqueue_fill(b->fills[i].first, b->fills[i].second.first, b->fill_rows[i], b->fills[i].second.second, st);
        if (rc) return rc;
    }
    // units of work: the groups' persistent launches, then the solo items
    const size_t n_units = b->groups.size() + b->solo.size();
    if (n_units == 0) return hip_check(hipGetLastError(), "batch launch");
    if (!b->groups.empty())
        hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(128), 0, st, ws, (int)b->groups.size());
    // Units go to the least loaded of `ns` streams, largest first: a group that
    // cannot fill the chip, and the tail of each launch, overlap with other
    // units instead of idling the device.
    const int ns = batch_streams(b);
    ForkSet* fs = nullptr;
    hipStream_t lanes[kBatchStreamsMax] = {st};
    hipEvent_t fork = nullptr, join[kBatchStreamsMax - 1] = {};
    std::unique_lock<std::mutex> hold;   // the device's helper streams, until they are joined back
    if (ns > 1) {
        int rc = fork_set(&fs);
        if (rc) return rc;
        hold = std::unique_lock<std::mutex>(fs->use);
        fork = events ? events[0] : fs->fork;
        for (int i = 1; i < ns; ++i) join[i - 1] = events ? events[i] : fs->join[i - 1];
        rc = hip_check(hipEventRecord(fork, st), "batch fork");
        for (int i = 1; !rc && i < ns; ++i) {
            lanes[i] = fs->helper[i - 1];
            rc = hip_check(hipStreamWaitEvent(lanes[i], fork, 0), "batch fork");
        }
        if (rc) return rc;
    }
    auto unit_tiles = [&](size_t u) {
        return u < b->groups.size() ? b->groups[u].tiles : b->solo[u - b->groups.size()].c.ntiles;
    };
    std::vector<uint32_t> order(n_units);
    for (size_t u = 0; u < n_units; ++u) order[u] = (uint32_t)u;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return unit_tiles(x) > unit_tiles(y); });
    uint64_t load[kBatchStreamsMax] = {};
    int rc = BST_OK;
    for (uint32_t u : order) {
        int lane = 0;
        for (int i = 1; i < ns; ++i)
            if (load[i] < load[lane]) lane = i;
        load[lane] += unit_tiles(u);
        const hipStream_t gs = lanes[lane];
        if (u >= b->groups.size()) {
            // a large item: the single-column kernel with its own launch shape
            const BatchItem& it = b->solo[u - b->groups.size()];
            const int r = it.c.layout == BST_BITPACKED ? launch_packed(it.c, it.pl, it.in_mask, it.out, nullptr, gs)
                                                       : launch_slices(it.c, it.lit, it.in_mask, it.out, nullptr, gs);
            if (!rc) rc = r;
            continue;
        }
        const uint32_t g = u;
        const BatchGroup& gr = b->groups[g];
        char* h = ws + g * kBatchHeaderBytes;
        // no more waves than the group has tiles
        const uint32_t grid_g = (uint32_t)std::max<uint64_t>(
            1, std::min<uint64_t>(grid, (gr.tiles + kWavesPerBlock - 1) / kWavesPerBlock));
        const uint64_t waves = (uint64_t)grid_g * kWavesPerBlock;
        // A small group spreads over all its waves, one take each.  A large one
        // takes at least `grab` tiles at a time and no more than about four
        // takes per wave: every take is an atomic on the group's one counter.
        // Round robin passes 0.
        uint64_t take;
        if (grab == BST_BATCH_ROUND_ROBIN)
            take = 0;
        else if (gr.tiles <= (uint64_t)grab * waves)
            take = std::max<uint64_t>(1, (gr.tiles + waves - 1) / waves);
        else
            take = std::max<uint64_t>(grab, (gr.tiles + 4 * waves - 1) / (4 * waves));
        if (take) take = std::min<uint64_t>(take, 1u << 20);
        hipLaunchKernelGGL(batch_kernel(gr.kind, gr.has_in), dim3(grid_g), dim3(kBlock), 0, gs,
                           (const BatchHeader*)h, items + gr.first, (unsigned long long*)(h + 32), (uint32_t)take);
    }
    {
        const int r = hip_check(hipGetLastError(), "batch launch");
        if (!rc) rc = r;
    }
    for (int i = 1; i < ns; ++i) {   // join every helper back, also after an error
        int r2 = hip_check(hipEventRecord(join[i - 1], lanes[i]), "batch join");
        if (!r2) r2 = hip_check(hipStreamWaitEvent(st, join[i - 1], 0), "batch join");
        if (!rc) rc = r2;
    }
    return rc;
}

int bst_batch_launch(bst_batch* b, uint32_t grid, uint32_t tiles_per_grab, int use_graph, void* stream) {
    if (!b) return set_error(BST_EINVAL, "NULL batch");
    hipStream_t st = (hipStream_t)stream;
    if (grid == 0) grid = g_tune[BST_TUNE_BATCH_GRID] > 0 ? (uint32_t)g_tune[BST_TUNE_BATCH_GRID] : (uint32_t)props().cus * 8;
    if (tiles_per_grab == 0) tiles_per_grab = g_tune[BST_TUNE_BATCH_GRAB] > 0 ? (uint32_t)g_tune[BST_TUNE_BATCH_GRAB] : 16;
    if (!b->uploaded) {
        // header block and work list as one image, one copy
        const size_t head = (size_t)kBatchGroupsMax * kBatchHeaderBytes;
        std::vector<char> img(head + b->items.size() * sizeof(BatchItem), 0);
        for (size_t g = 0; g < b->groups.size(); ++g) {
            BatchHeader h{b->groups[g].tiles, b->groups[g].count, 0};
            memcpy(img.data() + g * kBatchHeaderBytes, &h, sizeof(h));
        }
        if (!b->items.empty()) memcpy(img.data() + head, b->items.data(), b->items.size() * sizeof(BatchItem));
        int rc = ring_upload(b->ws, img.data(), img.size(), st);
        if (rc) return rc;
        b->uploaded = true;
    }
    if (!use_graph) return batch_enqueue(b, grid, tiles_per_grab, st, nullptr);
    if (!b->exec || b->graph_grid != grid || b->graph_grab != tiles_per_grab ||
        b->graph_streams != g_tune[BST_TUNE_BATCH_STREAMS]) {
        destroy_graph(b);
        // the graph's own fork and join events, made before the capture starts
        const int ns = batch_streams(b);
        for (int i = 0; ns > 1 && i < ns; ++i) {
            hipEvent_t e;
            int rc = hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "graph event");
            if (rc) return rc;
            b->graph_events.push_back(e);
        }
        hipStream_t cap;
        int rc = hip_check(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "capture stream");
        if (rc) return rc;
        rc = hip_check(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
        if (!rc) {
            int rc2 = batch_enqueue(b, grid, tiles_per_grab, cap, b->graph_events.empty() ? nullptr : b->graph_events.data());
            rc = hip_check(hipStreamEndCapture(cap, &b->graph), "end capture");
            if (!rc) rc = rc2;
        }
        if (!rc) rc = hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiate");
        (void)hipStreamDestroy(cap);
        if (rc) return rc;
        b->graph_grid = grid;
        b->graph_grab = tiles_per_grab;
        b->graph_streams = g_tune[BST_TUNE_BATCH_STREAMS];
    }
    return hip_check(hipGraphLaunch(b->exec, st), "graph launch");
}

void bst_batch_free(bst_batch* b) {
    if (!b) return;
    destroy_graph(b);
    delete b;
}

}  // extern "C"
