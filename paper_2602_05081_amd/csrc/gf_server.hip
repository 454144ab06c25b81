// Serving executor: resident scenes, render requests admitted by memory and
// rendered in shared device batches (continuous batching).
//
// Memory: the server owns one device pool of `mem_budget` bytes, carved by a
// first-fit allocator; an admitted request holds width*height*32 bytes of
// camera rays there until its last tile completes.  No device allocation
// happens while serving; the tracking workspace of one batch is allocated
// with the server.
// Scheduling: requests wait in FIFO order until their rays fit the pool; an
// admitted request's rays are generated on the device right away.  Each step
// assembles one batch of up to `max_tiles` tiles of `tile_rays` rays from the
// admitted requests, shortest remaining work first (rays left x samples,
// multiple scattering weighted 3x), and launches it as a single kernel; up to
// two batches are in flight, each followed by an event.  A request finishes
// when the events of all its tiles have completed.
// The API is single-threaded: all calls on one server come from one thread.
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <vector>

#include "gf_internal.hpp"

gf_status gf_camera_launch(const gf_camera* cam, float* rays, hipStream_t sm);
gf_status gf_check_camera(const gf_camera* cam, const char* who);
gf_status gf_check_render_desc(const gf_render_desc* d, const char* who);
gf_status gf_serve_fill_req(const gf_request* q, const float* rays, void* out_desc);
size_t gf_serve_req_size();
size_t gf_serve_tile_size();
gf_status gf_serve_launch(const void* dreqs, const void* dtiles, int ntiles, int tile_rays, float* ws, hipStream_t sm);
size_t gf_serve_workspace_bytes(int max_tiles, int tile_rays);

namespace {

const size_t kAlign = 256;
const int kSlots = 2;  // batches in flight

struct Req {
    uint64_t id;
    gf_request q;
    int n;
    size_t bytes, off;
    int next_ray;   // first ray not yet put in a batch
    int rays_done;  // rays whose batch completed
};

struct Batch {
    hipEvent_t ev;
    int slot;
    std::vector<std::pair<uint64_t, int>> work;  // (request id, rays)
};

struct FreeBlock {
    size_t off, size;
};

}  // namespace

struct gf_server_s {
    size_t budget, held;
    int tile_rays, max_tiles;
    hipStream_t stream;
    char* pool;
    float* ws;  // tracking workspace of one batch (batches run in stream order)
    std::vector<FreeBlock> freel;  // sorted by offset, coalesced
    std::deque<Req*> queue;
    std::vector<Req*> active;
    std::map<uint64_t, Req*> byid;
    std::deque<uint64_t> done;
    std::deque<Batch> inflight;
    bool slot_busy[kSlots];
    char* hreq[kSlots];
    char* htile[kSlots];
    char* dreq[kSlots];
    char* dtile[kSlots];
    hipEvent_t events[kSlots];
    uint64_t next_id;
};

static bool pool_alloc(gf_server_s* S, size_t bytes, size_t* off) {
    for (size_t i = 0; i < S->freel.size(); ++i) {
        FreeBlock& b = S->freel[i];
        if (b.size >= bytes) {
            *off = b.off;
            b.off += bytes;
            b.size -= bytes;
            if (b.size == 0) S->freel.erase(S->freel.begin() + i);
            S->held += bytes;
            return true;
        }
    }
    return false;
}

static void pool_free(gf_server_s* S, size_t off, size_t bytes) {
    auto it = std::lower_bound(S->freel.begin(), S->freel.end(), off,
                               [](const FreeBlock& b, size_t o) { return b.off < o; });
    it = S->freel.insert(it, FreeBlock{off, bytes});
    size_t i = it - S->freel.begin();
    if (i + 1 < S->freel.size() && S->freel[i].off + S->freel[i].size == S->freel[i + 1].off) {
        S->freel[i].size += S->freel[i + 1].size;
        S->freel.erase(S->freel.begin() + i + 1);
    }
    if (i > 0 && S->freel[i - 1].off + S->freel[i - 1].size == S->freel[i].off) {
        S->freel[i - 1].size += S->freel[i].size;
        S->freel.erase(S->freel.begin() + i);
    }
    S->held -= bytes;
}

static size_t req_bytes(const gf_request* q) {
    size_t b = (size_t)q->camera.width * q->camera.height * 8 * sizeof(float);
    return (b + kAlign - 1) / kAlign * kAlign;
}

extern "C" gf_status gf_server_create(size_t mem_budget, int tile_rays, int max_tiles, void* stream,
                                      gf_server* out) {
    if (!out) return gf_fail(GF_EINVAL, "gf_server_create: out is NULL");
    *out = nullptr;
    if (mem_budget < kAlign || tile_rays < 64 || tile_rays > (1 << 20) || max_tiles < 1 || max_tiles > 65536)
        return gf_fail(GF_EINVAL, "gf_server_create: budget >= 256 B, 64 <= tile_rays <= 2^20, 1 <= max_tiles <= 65536");
    gf_server_s* S = new gf_server_s();
    S->budget = mem_budget / kAlign * kAlign;
    S->held = 0;
    S->tile_rays = tile_rays;
    S->max_tiles = max_tiles;
    S->stream = (hipStream_t)stream;
    S->next_id = 1;
    S->pool = nullptr;
    S->ws = nullptr;
    for (int k = 0; k < kSlots; ++k) {
        S->slot_busy[k] = false;
        S->hreq[k] = S->htile[k] = S->dreq[k] = S->dtile[k] = nullptr;
        S->events[k] = nullptr;
    }
    auto fail = [&](hipError_t e, const char* what) {
        gf_server_destroy(S);
        return gf_hip_check(e, what);
    };
    hipError_t e = hipMalloc((void**)&S->pool, S->budget);
    if (e != hipSuccess) return fail(e, "hipMalloc(pool)");
    S->freel.push_back(FreeBlock{0, S->budget});
    e = hipMalloc((void**)&S->ws, gf_serve_workspace_bytes(max_tiles, tile_rays));
    if (e != hipSuccess) return fail(e, "hipMalloc(workspace)");
    for (int k = 0; k < kSlots; ++k) {
        if ((e = hipHostMalloc((void**)&S->hreq[k], gf_serve_req_size() * max_tiles)) != hipSuccess)
            return fail(e, "hipHostMalloc");
        if ((e = hipHostMalloc((void**)&S->htile[k], gf_serve_tile_size() * max_tiles)) != hipSuccess)
            return fail(e, "hipHostMalloc");
        if ((e = hipMalloc((void**)&S->dreq[k], gf_serve_req_size() * max_tiles)) != hipSuccess)
            return fail(e, "hipMalloc");
        if ((e = hipMalloc((void**)&S->dtile[k], gf_serve_tile_size() * max_tiles)) != hipSuccess)
            return fail(e, "hipMalloc");
        if ((e = hipEventCreateWithFlags(&S->events[k], hipEventDisableTiming)) != hipSuccess)
            return fail(e, "hipEventCreate");
    }
    *out = S;
    return GF_OK;
}

extern "C" gf_status gf_server_destroy(gf_server S) {
    if (!S) return gf_fail(GF_EINVAL, "gf_server_destroy: NULL server");
    if (S->stream || S->pool) (void)hipStreamSynchronize(S->stream);
    for (int k = 0; k < kSlots; ++k) {
        if (S->hreq[k]) (void)hipHostFree(S->hreq[k]);
        if (S->htile[k]) (void)hipHostFree(S->htile[k]);
        if (S->dreq[k]) (void)hipFree(S->dreq[k]);
        if (S->dtile[k]) (void)hipFree(S->dtile[k]);
        if (S->events[k]) (void)hipEventDestroy(S->events[k]);
    }
    if (S->pool) (void)hipFree(S->pool);
    if (S->ws) (void)hipFree(S->ws);
    for (auto& kv : S->byid) delete kv.second;
    delete S;
    return GF_OK;
}

extern "C" gf_status gf_server_submit(gf_server S, const gf_request* q, uint64_t* id) {
    if (!S || !q || !id) return gf_fail(GF_EINVAL, "gf_server_submit: NULL argument");
    if (!q->scene || !q->out) return gf_fail(GF_EINVAL, "gf_server_submit: request without scene or output");
    gf_status st = gf_check_camera(&q->camera, "gf_server_submit");
    if (st == GF_OK) st = gf_check_render_desc(&q->render, "gf_server_submit");
    if (st != GF_OK) return st;
    if (q->scene->depth > 64) return gf_fail(GF_EINVAL, "gf_server_submit: scene LBVH deeper than 64");
    size_t bytes = req_bytes(q);
    if (bytes > S->budget) return gf_fail(GF_EINVAL, "gf_server_submit: request needs %zu bytes, budget %zu", bytes,
                                          S->budget);
    Req* r = new Req();
    r->id = S->next_id++;
    r->q = *q;
    r->n = q->camera.width * q->camera.height;
    r->bytes = bytes;
    r->off = 0;
    r->next_ray = 0;
    r->rays_done = 0;
    S->queue.push_back(r);
    S->byid[r->id] = r;
    *id = r->id;
    return GF_OK;
}

static gf_status retire(gf_server_s* S, bool wait) {
    while (!S->inflight.empty()) {
        Batch& b = S->inflight.front();
        hipError_t e = wait ? hipEventSynchronize(b.ev) : hipEventQuery(b.ev);
        if (e == hipErrorNotReady) return GF_OK;
        if (e != hipSuccess) return gf_hip_check(e, "batch event");
        for (auto& w : b.work) {
            Req* r = S->byid[w.first];
            r->rays_done += w.second;
            if (r->rays_done == r->n) {
                pool_free(S, r->off, r->bytes);
                S->active.erase(std::find(S->active.begin(), S->active.end(), r));
                S->done.push_back(r->id);
                S->byid.erase(r->id);
                delete r;
            }
        }
        S->slot_busy[b.slot] = false;
        S->inflight.pop_front();
        wait = false;  // block for at most one batch
    }
    return GF_OK;
}

static gf_status admit(gf_server_s* S) {
    while (!S->queue.empty()) {
        Req* r = S->queue.front();
        size_t off;
        if (!pool_alloc(S, r->bytes, &off)) break;
        r->off = off;
        gf_status st = gf_camera_launch(&r->q.camera, (float*)(S->pool + off), S->stream);
        if (st != GF_OK) return st;
        S->active.push_back(r);
        S->queue.pop_front();
    }
    return GF_OK;
}

static gf_status launch_batch(gf_server_s* S) {
    int slot = -1;
    for (int k = 0; k < kSlots; ++k)
        if (!S->slot_busy[k]) slot = k;
    if (slot < 0) return GF_OK;
    std::vector<Req*> open;
    for (Req* r : S->active)
        if (r->next_ray < r->n) open.push_back(r);
    if (open.empty()) return GF_OK;
    // shortest remaining work first (rays left x samples, multiple scattering
    // weighted 3x), arrival order among equals: a small request that arrives
    // behind a large one finishes in the next batch instead of after it
    auto work = [](const Req* r) {
        return (double)(r->n - r->next_ray) * r->q.render.spp * (r->q.render.multiple ? 3.0 : 1.0);
    };
    std::stable_sort(open.begin(), open.end(), [&](const Req* a, const Req* b) { return work(a) < work(b); });
    char* hreq = S->hreq[slot];
    char* htile = S->htile[slot];
    std::map<uint64_t, int> local;
    Batch b;
    b.slot = slot;
    b.ev = S->events[slot];
    int ntiles = 0, nreq = 0;
    std::map<uint64_t, int> rays_in;
    for (Req* r : open) {
        while (ntiles < S->max_tiles && r->next_ray < r->n) {
            auto it = local.find(r->id);
            int li;
            if (it == local.end()) {
                li = nreq++;
                local[r->id] = li;
                gf_serve_fill_req(&r->q, (const float*)(S->pool + r->off), hreq + li * gf_serve_req_size());
            } else {
                li = it->second;
            }
            int cnt = std::min(S->tile_rays, r->n - r->next_ray);
            int tile[4] = {li, r->next_ray, cnt, 0};
            memcpy(htile + ntiles * gf_serve_tile_size(), tile, sizeof(tile));
            r->next_ray += cnt;
            rays_in[r->id] += cnt;
            ++ntiles;
        }
    }
    for (auto& kv : rays_in) b.work.push_back(kv);
    GF_HIP(hipMemcpyAsync(S->dreq[slot], hreq, gf_serve_req_size() * nreq, hipMemcpyHostToDevice, S->stream));
    GF_HIP(hipMemcpyAsync(S->dtile[slot], htile, gf_serve_tile_size() * ntiles, hipMemcpyHostToDevice, S->stream));
    gf_status st = gf_serve_launch(S->dreq[slot], S->dtile[slot], ntiles, S->tile_rays, S->ws, S->stream);
    if (st != GF_OK) return st;
    GF_HIP(hipEventRecord(b.ev, S->stream));
    S->slot_busy[slot] = true;
    S->inflight.push_back(b);
    return GF_OK;
}

extern "C" gf_status gf_server_step(gf_server S, int wait) {
    if (!S) return gf_fail(GF_EINVAL, "gf_server_step: NULL server");
    gf_status st = retire(S, false);
    if (st != GF_OK) return st;
    st = admit(S);
    if (st != GF_OK) return st;
    st = launch_batch(S);
    if (st != GF_OK) return st;
    if (wait && !S->inflight.empty()) {
        st = retire(S, true);
        if (st != GF_OK) return st;
        st = admit(S);
    }
    return st;
}

extern "C" gf_status gf_server_poll(gf_server S, uint64_t* ids, int max, int* n_done) {
    if (!S || !n_done || (max > 0 && !ids)) return gf_fail(GF_EINVAL, "gf_server_poll: NULL argument");
    int k = 0;
    while (k < max && !S->done.empty()) {
        ids[k++] = S->done.front();
        S->done.pop_front();
    }
    *n_done = k;
    return GF_OK;
}

extern "C" gf_status gf_server_stats(gf_server S, int* queued, int* in_flight, size_t* bytes_held) {
    if (!S) return gf_fail(GF_EINVAL, "gf_server_stats: NULL server");
    if (queued) *queued = (int)S->queue.size();
    if (in_flight) *in_flight = (int)S->active.size();
    if (bytes_held) *bytes_held = S->held;
    return GF_OK;
}
