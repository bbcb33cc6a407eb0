// server.hip -- served connected-component labeling (C ABI in include/swccl.h).
//
// Requests (binary images or bond arrays in host memory) are labeled on the
// GPU as they arrive.  Each admitted request takes one block of a caller-owned
// device arena, sized by its footprint (input, labels, optional roots and
// sizes, labeling workspace), so small and large requests share the memory
// without fixed-size slots; a request that does not fit waits in the caller's
// queue until completed requests are released.  Requests are spread over the
// caller's streams, so the copy of one request overlaps the labeling of
// others.  Completion is tracked with one event per admitted request.
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
    hipEvent_t done{};
};

}  // namespace

struct ccl_server {
    ccl_server_params p;
    char *arena;
    size_t arena_bytes;
    std::map<size_t, size_t> free_blocks;  // offset -> bytes, coalesced
    std::vector<Request> req;
    std::vector<hipStream_t> streams;
    int next_stream;
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
           p->max_inflight <= 4096 && p->n_streams >= 1 && p->n_streams <= 64 && (p->sizes == 0 || p->sizes == 1);
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
    ccl_server *s = new (std::nothrow) ccl_server();
    if (!s) return SW_ERR_HOST_MEMORY;
    s->p = *p;
    s->arena = static_cast<char *>(arena);
    s->arena_bytes = arena_bytes / ALIGN * ALIGN;
    s->next_stream = 0;
    try {
        s->free_blocks[0] = s->arena_bytes;
        for (int32_t i = 0; i < p->n_streams; ++i) s->streams.push_back(static_cast<hipStream_t>(streams[i]));
        s->req.resize(static_cast<size_t>(p->max_inflight));
    } catch (const std::bad_alloc &) {
        delete s;
        return SW_ERR_HOST_MEMORY;
    }
    for (auto &r : s->req) {
        if (hipEventCreateWithFlags(&r.done, hipEventDisableTiming) != hipSuccess) {
            for (auto &q : s->req)
                if (q.done) (void)hipEventDestroy(q.done);
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
    if (L.total > s->arena_bytes) return SW_ERR_SIZE;  // can never be admitted
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
    hipStream_t st = s->streams[static_cast<size_t>(s->next_stream)];
    s->next_stream = (s->next_stream + 1) % s->p.n_streams;
    char *base = s->arena + off;
    uint8_t *in = reinterpret_cast<uint8_t *>(base + L.in);
    int32_t *labels = reinterpret_cast<int32_t *>(base + L.labels);
    int32_t *roots = s->p.sizes ? reinterpret_cast<int32_t *>(base + L.roots) : nullptr;
    int32_t *sizes = s->p.sizes ? reinterpret_cast<int32_t *>(base + L.sizes) : nullptr;
    int32_t *ncl = reinterpret_cast<int32_t *>(base + L.ncl);
    sw_status status = SW_OK;
    // a contiguous image goes as one linear copy (much faster than a 2D copy)
    const hipError_t ce =
        pitch == static_cast<size_t>(W)
            ? hipMemcpyAsync(in, image, static_cast<size_t>(W) * static_cast<size_t>(H), hipMemcpyHostToDevice, st)
            : hipMemcpy2DAsync(in, static_cast<size_t>(W), image, pitch, static_cast<size_t>(W),
                               static_cast<size_t>(H), hipMemcpyHostToDevice, st);
    if (ce != hipSuccess) status = SW_ERR_DEVICE;
    if (status == SW_OK)
        status = ccl_label(in, W, H, s->p.mode, labels, roots, sizes, ncl, base + L.ws, L.ws_bytes, st);
    if (status == SW_OK && hipEventRecord(r.done, st) != hipSuccess) status = SW_ERR_DEVICE;
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
    *slot = k;
    return SW_OK;
}

sw_status ccl_server_poll(ccl_server *s, int32_t *slots, uint64_t *tags, int32_t max, int32_t *n)
{
    if (!s || !n || max < 0 || (max > 0 && (!slots || !tags))) return SW_ERR_ARG;
    int32_t m = 0;
    for (size_t i = 0; i < s->req.size() && m < max; ++i) {
        Request &r = s->req[i];
        if (!r.busy || r.reported) continue;
        const hipError_t e = hipEventQuery(r.done);
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
    // a block is reused only after its request has finished on the device
    if (hipEventSynchronize(r.done) != hipSuccess) return SW_ERR_DEVICE;
    try {
        arena_give(s, r.off, r.L.total);
    } catch (const std::bad_alloc &) {
        return SW_ERR_HOST_MEMORY;  // still admitted: the release can be retried
    }
    r.busy = false;
    r.reported = false;
    return SW_OK;
}

sw_status ccl_server_destroy(ccl_server *s)
{
    if (!s) return SW_ERR_ARG;
    for (auto &r : s->req) {
        if (r.busy) (void)hipEventSynchronize(r.done);
        (void)hipEventDestroy(r.done);
    }
    delete s;
    return SW_OK;
}

}  // extern "C"
