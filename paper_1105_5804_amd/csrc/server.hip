// server.hip -- served connected-component labeling (C ABI in include/swccl.h).
//
// Requests (binary images or bond arrays in host memory) are labeled on the
// GPU as they arrive.  Each admitted request takes one block of a caller-owned
// device arena, sized by its footprint (input, labels, optional roots and
// sizes, labeling workspace), so small and large requests share the memory
// without fixed-size slots; a request that does not fit waits in the caller's
// queue until completed requests are released.  Requests are spread over the
// caller's streams, so the copy of one request overlaps the labeling of
// others.
//
// Continuous batching: a request of at most batch_px pixels (and a few tiles)
// joins the open batch, whose images are copied on the batch's stream; a
// flush (explicit, or by the next poll) labels the whole batch with one launch
// per phase, so many small images share the fixed cost of a launch sequence.
// Larger requests are labeled on their own at once.  Completion is tracked by
// one event per launch sequence (a batch's requests share it), taken from a
// pool and returned when its last request is released.
//
// The server allocates no device memory and is not thread-safe: one host
// thread drives it.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <iterator>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/swccl.h"
#include "internal.hpp"

namespace {

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// Byte layout of one request inside its arena block.
struct ReqLayout {
    size_t in, labels, roots, sizes, ncl, ws, ws_bytes, total;
};

ReqLayout req_layout(int32_t W, int32_t H, int32_t mode, bool sizes)
{
    ReqLayout L{};
    const size_t N = static_cast<size_t>(W) * static_cast<size_t>(H);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += align_up(bytes);
        return at;
    };
    L.in = take(N);
    L.labels = take(N * 4);
    if (sizes) {
        L.roots = take(N * 4);
        L.sizes = take(N * 4);
    }
    L.ncl = take(4);
    L.ws_bytes = ccl_workspace_bytes(W, H, mode);
    L.ws = take(L.ws_bytes);
    L.total = off;
    return L;
}

struct Request {
    bool busy = false;     // admitted and not yet released
    bool reported = false; // returned by a poll
    uint64_t tag = 0;
    int32_t W = 0, H = 0;
    size_t off = 0;        // block in the arena
    ReqLayout L{};
    int ev = -1;           // completion event in the pool; -1 while in the open batch
};

// Batches: at most this many requests and tiles, each request at most
// BATCH_REQ_TILES tiles.  Each stream has a ring of TABLE_RING batch tables
// (device, in front of the arena) with pinned host copies, so a flush does
// not wait for the stream's earlier batches.
constexpr int32_t BATCH_MAX_REQS = 256;
constexpr int64_t BATCH_MAX_TILES = 8192;
constexpr int64_t BATCH_REQ_TILES = 128;
constexpr int TABLE_RING = 4;

}  // namespace

struct ccl_server {
    ccl_server_params p;
    char *arena;
    size_t arena_bytes;
    std::map<size_t, size_t> free_blocks;  // offset -> bytes, coalesced
    std::vector<Request> req;
    std::vector<hipStream_t> streams;
    int next_stream;
    // completion events (one per launch sequence) and their request counts
    std::vector<hipEvent_t> ev;
    std::vector<int32_t> ev_refs;
    // the open batch: its stream, requests and tiles so far
    int open_stream = -1;
    std::vector<int32_t> open_slots;
    int64_t open_tiles = 0;
    // per stream and ring slot: a batch table (device, arena front), its pinned
    // host copy, and the event of the batch that last used the slot
    size_t table_bytes = 0;
    char *pinned = nullptr;
    std::vector<int> ring_next;
    std::vector<int> slot_ev;  // [stream * TABLE_RING + slot]
    std::vector<int> last_ev;  // per stream: event of its last launch sequence, or -1
};

namespace {

// First fit; returns false when no free block is large enough.  Throws
// std::bad_alloc (with the free list unchanged) if the remainder's node cannot
// be allocated.
bool arena_take(ccl_server *s, size_t bytes, size_t *off)
{
    for (auto it = s->free_blocks.begin(); it != s->free_blocks.end(); ++it) {
        if (it->second < bytes) continue;
        const size_t at = it->first, rest = it->second - bytes;
        if (rest) s->free_blocks.emplace(at + bytes, rest);  // the only step that can throw
        s->free_blocks.erase(it);
        *off = at;
        return true;
    }
    return false;
}

// Returns a block to the free list, merging it with its neighbours.  Throws
// std::bad_alloc (with the free list unchanged) if its node cannot be allocated.
void arena_give(ccl_server *s, size_t off, size_t bytes)
{
    auto it = s->free_blocks.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != s->free_blocks.end() && it->first + it->second == next->first) {
        it->second += next->second;
        s->free_blocks.erase(next);
    }
    if (it != s->free_blocks.begin()) {
        auto prev = std::prev(it);
        if (prev->first + prev->second == it->first) {
            prev->second += it->second;
            s->free_blocks.erase(it);
        }
    }
}

bool valid_params(const ccl_server_params *p)
{
    return p && p->mode >= CCL_BONDS_PERIODIC && p->mode <= CCL_SITES_OPEN && p->max_inflight >= 1 &&
           p->max_inflight <= 4096 && p->n_streams >= 1 && p->n_streams <= 64 && (p->sizes == 0 || p->sizes == 1) &&
           p->batch_px >= 0;
}

// A free event of the pool, or -1.
int take_event(ccl_server *s)
{
    for (size_t i = 0; i < s->ev.size(); ++i)
        if (s->ev_refs[i] == 0) return static_cast<int>(i);
    return -1;
}

void drop_ref(ccl_server *s, int e)
{
    if (e >= 0 && s->ev_refs[static_cast<size_t>(e)] > 0) --s->ev_refs[static_cast<size_t>(e)];
}

// The stream for new work: the first one, from the round-robin position on,
// whose last launch sequence has completed and which does not hold the open
// batch, else the next round-robin one other than the open batch's (a
// single request must not delay the batch's labeling).
int pick_stream(ccl_server *s)
{
    const int n = s->p.n_streams;
    int chosen = -1;
    for (int k = 0; k < n && chosen < 0; ++k) {
        const int si = (s->next_stream + k) % n;
        if (si == s->open_stream && n > 1) continue;
        const int e = s->last_ev[static_cast<size_t>(si)];
        if (e < 0 || hipEventQuery(s->ev[static_cast<size_t>(e)]) == hipSuccess) chosen = si;
    }
    if (chosen < 0) {
        chosen = s->next_stream;
        if (chosen == s->open_stream && n > 1) chosen = (chosen + 1) % n;
    }
    s->next_stream = (chosen + 1) % n;
    return chosen;
}

bool batchable(const ccl_server *s, int32_t W, int32_t H)
{
    return s->p.batch_px > 0 && static_cast<int64_t>(W) * H <= s->p.batch_px &&
           swccl_internal::request_tiles(W, H) <= BATCH_REQ_TILES;
}

size_t table_index(int stream, int slot) { return static_cast<size_t>(stream) * TABLE_RING + static_cast<size_t>(slot); }

// Label the open batch (one launch per phase on its stream); its requests
// then share one completion event.
sw_status flush_open(ccl_server *s)
{
    if (s->open_slots.empty()) return SW_OK;
    const int si = s->open_stream;
    hipStream_t st = s->streams[static_cast<size_t>(si)];
    // the next table slot of this stream; its last batch (TABLE_RING flushes
    // ago on this stream) has normally long passed, else wait for it
    const int slot = s->ring_next[static_cast<size_t>(si)];
    const size_t ti = table_index(si, slot);
    const int prev = s->slot_ev[ti];
    if (prev >= 0 && hipEventSynchronize(s->ev[static_cast<size_t>(prev)]) != hipSuccess) return SW_ERR_DEVICE;
    const int e = take_event(s);
    if (e < 0) return SW_ERR_STATE;  // cannot happen: one event per request at most
    std::vector<swccl_internal::LabelRequest> lr;
    try {
        lr.reserve(s->open_slots.size());
    } catch (const std::bad_alloc &) {
        return SW_ERR_HOST_MEMORY;
    }
    for (const int32_t k : s->open_slots) {
        const Request &r = s->req[static_cast<size_t>(k)];
        char *base = s->arena + r.off;
        swccl_internal::LabelRequest q{};
        q.in = reinterpret_cast<const uint8_t *>(base + r.L.in);
        q.W = r.W;
        q.H = r.H;
        q.labels = reinterpret_cast<int32_t *>(base + r.L.labels);
        q.roots = s->p.sizes ? reinterpret_cast<int32_t *>(base + r.L.roots) : nullptr;
        q.sizes = s->p.sizes ? reinterpret_cast<int32_t *>(base + r.L.sizes) : nullptr;
        q.n_clusters = reinterpret_cast<int32_t *>(base + r.L.ncl);
        q.ws = base + r.L.ws;
        lr.push_back(q);
    }
    sw_status status = swccl_internal::label_batch(lr.data(), static_cast<int32_t>(lr.size()), s->p.mode,
                                                   s->p.sizes != 0, s->arena + ti * s->table_bytes,
                                                   s->pinned + ti * s->table_bytes, s->table_bytes, st);
    if (status == SW_OK && hipEventRecord(s->ev[static_cast<size_t>(e)], st) != hipSuccess) status = SW_ERR_DEVICE;
    if (status != SW_OK) return status;  // the batch stays open: the flush can be retried
    s->ev_refs[static_cast<size_t>(e)] = static_cast<int32_t>(s->open_slots.size());
    for (const int32_t k : s->open_slots) s->req[static_cast<size_t>(k)].ev = e;
    s->slot_ev[ti] = e;
    s->last_ev[static_cast<size_t>(si)] = e;
    s->ring_next[static_cast<size_t>(si)] = (slot + 1) % TABLE_RING;
    s->open_slots.clear();
    s->open_tiles = 0;
    s->open_stream = -1;
    return SW_OK;
}

}  // namespace

extern "C" {

size_t ccl_server_footprint(int32_t W, int32_t H, const ccl_server_params *p)
{
    if (!valid_params(p) || ccl_workspace_bytes(W, H, p->mode) == 0) return 0;
    return req_layout(W, H, p->mode, p->sizes != 0).total;
}

sw_status ccl_server_create(ccl_server **out, const ccl_server_params *p, void *arena, size_t arena_bytes,
                            void *const *streams)
{
    if (!out || !valid_params(p) || !streams) return SW_ERR_ARG;
    if (!arena || arena_bytes < ALIGN || reinterpret_cast<uintptr_t>(arena) % ALIGN) return SW_ERR_WORKSPACE;
    // with batching, the front of the arena holds the batch tables
    const size_t tb = p->batch_px > 0 ? align_up(swccl_internal::batch_table_bytes(BATCH_MAX_REQS, BATCH_MAX_TILES)) : 0;
    const size_t ntables = static_cast<size_t>(p->n_streams) * TABLE_RING;
    const size_t usable = arena_bytes / ALIGN * ALIGN;
    if (tb * ntables + ALIGN > usable) return SW_ERR_WORKSPACE;
    ccl_server *s = new (std::nothrow) ccl_server();
    if (!s) return SW_ERR_HOST_MEMORY;
    s->p = *p;
    s->arena = static_cast<char *>(arena);
    s->arena_bytes = usable;
    s->next_stream = 0;
    s->table_bytes = tb;
    const size_t first = tb * ntables;
    if (tb && hipHostMalloc(reinterpret_cast<void **>(&s->pinned), tb * ntables, hipHostMallocDefault) != hipSuccess) {
        delete s;
        return SW_ERR_HOST_MEMORY;
    }
    try {
        s->free_blocks[first] = s->arena_bytes - first;
        for (int32_t i = 0; i < p->n_streams; ++i) s->streams.push_back(static_cast<hipStream_t>(streams[i]));
        s->req.resize(static_cast<size_t>(p->max_inflight));
        s->ev.resize(static_cast<size_t>(p->max_inflight), nullptr);
        s->ev_refs.assign(static_cast<size_t>(p->max_inflight), 0);
        s->ring_next.assign(static_cast<size_t>(p->n_streams), 0);
        s->last_ev.assign(static_cast<size_t>(p->n_streams), -1);
        s->slot_ev.assign(ntables, -1);
        s->open_slots.reserve(BATCH_MAX_REQS);
    } catch (const std::bad_alloc &) {
        if (s->pinned) (void)hipHostFree(s->pinned);
        delete s;
        return SW_ERR_HOST_MEMORY;
    }
    for (auto &e : s->ev) {
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            for (auto &f : s->ev)
                if (f) (void)hipEventDestroy(f);
            if (s->pinned) (void)hipHostFree(s->pinned);
            delete s;
            return SW_ERR_DEVICE;
        }
    }
    *out = s;
    return SW_OK;
}

sw_status ccl_server_submit(ccl_server *s, const uint8_t *image, int32_t W, int32_t H, size_t pitch, uint64_t tag,
                            int32_t *slot)
{
    if (!s || !image || !slot || pitch < static_cast<size_t>(W > 0 ? W : 0)) return SW_ERR_ARG;
    if (ccl_workspace_bytes(W, H, s->p.mode) == 0) return SW_ERR_SIZE;
    const ReqLayout L = req_layout(W, H, s->p.mode, s->p.sizes != 0);
    if (L.total > s->arena_bytes - s->table_bytes * s->streams.size() * TABLE_RING) return SW_ERR_SIZE;  // never fits
    int32_t k = -1;
    for (size_t i = 0; i < s->req.size(); ++i)
        if (!s->req[i].busy) {
            k = static_cast<int32_t>(i);
            break;
        }
    size_t off = 0;
    try {
        if (k < 0 || !arena_take(s, L.total, &off)) return SW_ERR_STATE;  // wait for a release
    } catch (const std::bad_alloc &) {
        return SW_ERR_HOST_MEMORY;
    }
    Request &r = s->req[static_cast<size_t>(k)];
    const bool batch = batchable(s, W, H);
    const int64_t ntiles = swccl_internal::request_tiles(W, H);
    if (batch && !s->open_slots.empty() &&
        (static_cast<int32_t>(s->open_slots.size()) >= BATCH_MAX_REQS || s->open_tiles + ntiles > BATCH_MAX_TILES)) {
        const sw_status fs = flush_open(s);  // the open batch is full: label it first
        if (fs != SW_OK) {
            try {
                arena_give(s, off, L.total);
            } catch (const std::bad_alloc &) {
            }
            return fs;
        }
    }
    int ev = -1;
    if (!batch && (ev = take_event(s)) < 0) {
        try {
            arena_give(s, off, L.total);
        } catch (const std::bad_alloc &) {
        }
        return SW_ERR_STATE;  // cannot happen: one event per request at most
    }
    // the open batch's stream for a batched request (its copies precede the
    // batch's labeling), else a stream that is idle if one is
    const int si = (batch && s->open_stream >= 0) ? s->open_stream : pick_stream(s);
    hipStream_t st = s->streams[static_cast<size_t>(si)];
    char *base = s->arena + off;
    uint8_t *in = reinterpret_cast<uint8_t *>(base + L.in);
    int32_t *labels = reinterpret_cast<int32_t *>(base + L.labels);
    int32_t *roots = s->p.sizes ? reinterpret_cast<int32_t *>(base + L.roots) : nullptr;
    int32_t *sizes = s->p.sizes ? reinterpret_cast<int32_t *>(base + L.sizes) : nullptr;
    int32_t *ncl = reinterpret_cast<int32_t *>(base + L.ncl);
    sw_status status = SW_OK;
    // A batched (small) contiguous image in pinned memory is pulled by a kernel
    // in the compute queue, so it does not wait behind large copies on the copy
    // engines; other images go as one linear copy (much faster than a 2D
    // copy) or as a 2D copy.
    const void *src_dev = nullptr;
    if (batch && pitch == static_cast<size_t>(W)) {
        hipPointerAttribute_t attr{};
        if (hipPointerGetAttributes(&attr, image) == hipSuccess && attr.type == hipMemoryTypeHost)
            src_dev = attr.devicePointer;
        else
            (void)hipGetLastError();  // pageable memory: no device address, not an error here
    }
    hipError_t ce = hipSuccess;
    if (src_dev)
        status = swccl_internal::pull(in, src_dev, static_cast<int64_t>(W) * H, st);
    else if (pitch == static_cast<size_t>(W))
        ce = hipMemcpyAsync(in, image, static_cast<size_t>(W) * static_cast<size_t>(H), hipMemcpyHostToDevice, st);
    else
        ce = hipMemcpy2DAsync(in, static_cast<size_t>(W), image, pitch, static_cast<size_t>(W), static_cast<size_t>(H),
                              hipMemcpyHostToDevice, st);
    if (ce != hipSuccess) status = SW_ERR_DEVICE;
    if (status == SW_OK && !batch) {
        status = ccl_label(in, W, H, s->p.mode, labels, roots, sizes, ncl, base + L.ws, L.ws_bytes, st);
        if (status == SW_OK && hipEventRecord(s->ev[static_cast<size_t>(ev)], st) != hipSuccess)
            status = SW_ERR_DEVICE;
        if (status == SW_OK) s->last_ev[static_cast<size_t>(si)] = ev;
    }
    if (status != SW_OK) {
        // nothing of this request may still run when its block is reused
        (void)hipStreamSynchronize(st);
        try {
            arena_give(s, off, L.total);
        } catch (const std::bad_alloc &) {
            // the block stays out of the free list: lost capacity, not a leak of device memory
        }
        return status;
    }
    r.busy = true;
    r.reported = false;
    r.tag = tag;
    r.W = W;
    r.H = H;
    r.off = off;
    r.L = L;
    r.ev = ev;
    if (batch) {
        s->open_stream = si;
        s->open_slots.push_back(k);  // capacity reserved at creation
        s->open_tiles += ntiles;
    } else {
        s->ev_refs[static_cast<size_t>(ev)] = 1;
    }
    *slot = k;
    return SW_OK;
}

sw_status ccl_server_flush(ccl_server *s)
{
    if (!s) return SW_ERR_ARG;
    return flush_open(s);
}

sw_status ccl_server_poll(ccl_server *s, int32_t *slots, uint64_t *tags, int32_t max, int32_t *n)
{
    if (!s || !n || max < 0 || (max > 0 && (!slots || !tags))) return SW_ERR_ARG;
    *n = 0;
    if (const sw_status fs = flush_open(s)) return fs;
    int32_t m = 0;
    for (size_t i = 0; i < s->req.size() && m < max; ++i) {
        Request &r = s->req[i];
        if (!r.busy || r.reported || r.ev < 0) continue;
        const hipError_t e = hipEventQuery(s->ev[static_cast<size_t>(r.ev)]);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) {
            *n = m;  // the pairs already written are still returned
            return SW_ERR_DEVICE;
        }
        r.reported = true;
        slots[m] = static_cast<int32_t>(i);
        tags[m] = r.tag;
        ++m;
    }
    *n = m;
    return SW_OK;
}

sw_status ccl_server_result(ccl_server *s, int32_t slot, int32_t **labels, int32_t **roots, int32_t **sizes,
                            int32_t **n_clusters)
{
    if (!s || slot < 0 || slot >= static_cast<int32_t>(s->req.size())) return SW_ERR_ARG;
    const Request &r = s->req[static_cast<size_t>(slot)];
    if (!r.busy) return SW_ERR_STATE;
    char *base = s->arena + r.off;
    if (labels) *labels = reinterpret_cast<int32_t *>(base + r.L.labels);
    if (roots) *roots = s->p.sizes ? reinterpret_cast<int32_t *>(base + r.L.roots) : nullptr;
    if (sizes) *sizes = s->p.sizes ? reinterpret_cast<int32_t *>(base + r.L.sizes) : nullptr;
    if (n_clusters) *n_clusters = reinterpret_cast<int32_t *>(base + r.L.ncl);
    return SW_OK;
}

sw_status ccl_server_release(ccl_server *s, int32_t slot)
{
    if (!s || slot < 0 || slot >= static_cast<int32_t>(s->req.size())) return SW_ERR_ARG;
    Request &r = s->req[static_cast<size_t>(slot)];
    if (!r.busy) return SW_ERR_STATE;
    if (r.ev < 0)
        if (const sw_status fs = flush_open(s)) return fs;  // still in the open batch
    // a block is reused only after its request has finished on the device
    if (hipEventSynchronize(s->ev[static_cast<size_t>(r.ev)]) != hipSuccess) return SW_ERR_DEVICE;
    try {
        arena_give(s, r.off, r.L.total);
    } catch (const std::bad_alloc &) {
        return SW_ERR_HOST_MEMORY;  // still admitted: the release can be retried
    }
    drop_ref(s, r.ev);
    r.busy = false;
    r.reported = false;
    r.ev = -1;
    return SW_OK;
}

sw_status ccl_server_destroy(ccl_server *s)
{
    if (!s) return SW_ERR_ARG;
    // the open batch's copies may still run: wait for every stream
    for (auto st : s->streams) (void)hipStreamSynchronize(st);
    for (auto &e : s->ev) {
        (void)hipEventSynchronize(e);
        (void)hipEventDestroy(e);
    }
    if (s->pinned) (void)hipHostFree(s->pinned);
    delete s;
    return SW_OK;
}

}  // extern "C"
