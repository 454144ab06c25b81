// Serving executor: resident scenes, render requests admitted by memory and
// rendered in shared device batches (continuous batching).
//
// Memory: the server owns one device pool of `mem_budget` bytes, carved by a
// first-fit allocator; an admitted request holds width*height*32 bytes of
// camera rays and width*height*spp*4 bytes of per-sample radiance there
// until its last tile completes.  No device allocation
// happens while serving; the tracking workspaces of the two batch slots are
// allocated with the server.
// Scheduling: requests wait in FIFO order until their rays fit the pool; an
// admitted request's rays are generated on the device right away (on the
// caller's stream).  Each step assembles one batch of up to `max_tiles`
// tiles of `tile_rays` rays from the admitted requests, shortest remaining
// work first (rays left x samples, multiple scattering weighted 3x), and
// launches it as a single kernel whose work units are single samples of 64
// rays (a chunk's samples on different waves), followed by the per-ray
// means of the batch's tiles.  Two batch slots, each with its own
// stream (default priority), workspace and event, let a batch start while
// the previous one drains its last chunks; each slot stream first waits for
// the ray generation queued before its launch.  A request finishes when the
// events of all its tiles have completed.
// The API is single-threaded: all calls on one server come from one thread.
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <vector>

#include "gf_internal.hpp"
#include "gf_sched.hpp"

gf_status gf_serve_fill_req(const gf_request* q, const float* rays, float* part, void* out_desc);
size_t gf_serve_req_size();
size_t gf_serve_tile_size();
int gf_serve_tile_threads();
gf_status gf_serve_launch(const void* dreqs, const void* dtiles, int ntiles, int nunits, int tile_rays,
                          int max_tiles, float* ws, hipStream_t sm);
size_t gf_serve_workspace_bytes(int max_tiles, int tile_rays);

namespace {

using gfs::kAlign;
const int kSlots = 2;  // batches in flight

struct Req : gfs::SchedReq {
    gf_request q;
};

struct Batch {
    hipEvent_t ev;
    int slot;
    std::vector<std::pair<uint64_t, int>> work;  // (request id, rays)
};

}  // namespace

struct gf_server_s {
    gfs::Pool mem;  // offsets into `pool`
    int tile_rays, max_tiles;
    hipStream_t stream;  // the caller's: ray generation
    char* pool;
    float* ws[kSlots];           // tracking workspace of each batch slot
    hipStream_t sstream[kSlots];  // each slot's stream
    hipEvent_t rays_ready;        // ray generation done (waited on by the slots)
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

extern "C" gf_status gf_server_create(size_t mem_budget, int tile_rays, int max_tiles, void* stream,
                                      gf_server* out) {
    if (!out) return gf_fail(GF_EINVAL, "gf_server_create: out is NULL");
    *out = nullptr;
    if (mem_budget < kAlign || tile_rays < 64 || tile_rays > (1 << 20) || max_tiles < 1 || max_tiles > 65536)
        return gf_fail(GF_EINVAL, "gf_server_create: budget >= 256 B, 64 <= tile_rays <= 2^20, 1 <= max_tiles <= 65536");
    gf_server_s* S = new gf_server_s();
    S->mem.reset(mem_budget / kAlign * kAlign);
    S->tile_rays = tile_rays;
    S->max_tiles = max_tiles;
    S->stream = (hipStream_t)stream;
    S->next_id = 1;
    S->pool = nullptr;
    S->rays_ready = nullptr;
    for (int k = 0; k < kSlots; ++k) {
        S->slot_busy[k] = false;
        S->hreq[k] = S->htile[k] = S->dreq[k] = S->dtile[k] = nullptr;
        S->events[k] = nullptr;
        S->ws[k] = nullptr;
        S->sstream[k] = nullptr;
    }
    auto fail = [&](hipError_t e, const char* what) {
        gf_server_destroy(S);
        return gf_hip_check(e, what);
    };
    hipError_t e = hipMalloc((void**)&S->pool, S->mem.budget);
    if (e != hipSuccess) return fail(e, "hipMalloc(pool)");
    if ((e = hipEventCreateWithFlags(&S->rays_ready, hipEventDisableTiming)) != hipSuccess)
        return fail(e, "hipEventCreate");
    for (int k = 0; k < kSlots; ++k) {
        if ((e = hipMalloc((void**)&S->ws[k], gf_serve_workspace_bytes(max_tiles, tile_rays))) != hipSuccess)
            return fail(e, "hipMalloc(workspace)");
        if ((e = hipStreamCreateWithFlags(&S->sstream[k], hipStreamNonBlocking)) != hipSuccess)
            return fail(e, "hipStreamCreate");
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
        if (S->sstream[k]) {
            (void)hipStreamSynchronize(S->sstream[k]);
            (void)hipStreamDestroy(S->sstream[k]);
        }
        if (S->ws[k]) (void)hipFree(S->ws[k]);
        if (S->hreq[k]) (void)hipHostFree(S->hreq[k]);
        if (S->htile[k]) (void)hipHostFree(S->htile[k]);
        if (S->dreq[k]) (void)hipFree(S->dreq[k]);
        if (S->dtile[k]) (void)hipFree(S->dtile[k]);
        if (S->events[k]) (void)hipEventDestroy(S->events[k]);
    }
    if (S->pool) (void)hipFree(S->pool);
    if (S->rays_ready) (void)hipEventDestroy(S->rays_ready);
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
    if (q->render.free_flight != 0 || q->render.transmittance != 0)
        return gf_fail(GF_EINVAL, "gf_server_submit: the server batches delta-tracked renders with ratio-tracked "
                                  "transmittance only (free_flight 0, transmittance 0)");
    if (q->scene->depth > 64) return gf_fail(GF_EINVAL, "gf_server_submit: scene LBVH deeper than 64");
    const int64_t chunks = (int64_t)S->max_tiles * ((S->tile_rays + gf_serve_tile_threads() - 1) / gf_serve_tile_threads());
    if (chunks * q->render.spp > (int64_t)INT32_MAX / 2)
        return gf_fail(GF_EINVAL, "gf_server_submit: %d samples per ray exceed what a batch of %d tiles can index",
                       q->render.spp, S->max_tiles);
    size_t bytes = gfs::request_bytes(q->camera.width, q->camera.height, q->render.spp);
    if (bytes > S->mem.budget)
        return gf_fail(GF_EINVAL, "gf_server_submit: request needs %zu bytes, budget %zu", bytes, S->mem.budget);
    Req* r = new Req();
    r->id = S->next_id++;
    r->q = *q;
    r->n = q->camera.width * q->camera.height;
    r->spp = q->render.spp;
    r->multiple = q->render.multiple != 0;
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
                S->mem.release(r->off, r->bytes);
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
        if (!S->mem.alloc(r->bytes, &off)) break;
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
    std::vector<gfs::SchedReq*> act(S->active.begin(), S->active.end());
    std::vector<gfs::TileRef> plan = gfs::plan_batch(act, S->tile_rays, S->max_tiles);
    if (plan.empty()) return GF_OK;
    char* hreq = S->hreq[slot];
    char* htile = S->htile[slot];
    std::map<uint64_t, int> local;
    Batch b;
    b.slot = slot;
    b.ev = S->events[slot];
    int ntiles = 0, nreq = 0;
    int64_t nunits = 0;
    std::map<uint64_t, int> rays_in;
    for (const gfs::TileRef& t : plan) {
        const Req* r = static_cast<const Req*>(t.r);
        auto it = local.find(r->id);
        int li;
        if (it == local.end()) {
            li = nreq++;
            local[r->id] = li;
            gf_serve_fill_req(&r->q, (const float*)(S->pool + r->off),
                              (float*)(S->pool + r->off + gfs::request_ray_bytes(r->q.camera.width, r->q.camera.height)),
                              hreq + li * gf_serve_req_size());
        } else {
            li = it->second;
        }
        int tile[4] = {li, t.first, t.count, (int)nunits};
        nunits += (int64_t)((t.count + gf_serve_tile_threads() - 1) / gf_serve_tile_threads()) * r->spp;
        memcpy(htile + ntiles * gf_serve_tile_size(), tile, sizeof(tile));
        rays_in[r->id] += t.count;
        ++ntiles;
    }
    for (auto& kv : rays_in) b.work.push_back(kv);
    hipStream_t sm = S->sstream[slot];
    GF_HIP(hipEventRecord(S->rays_ready, S->stream));
    GF_HIP(hipStreamWaitEvent(sm, S->rays_ready, 0));
    GF_HIP(hipMemcpyAsync(S->dreq[slot], hreq, gf_serve_req_size() * nreq, hipMemcpyHostToDevice, sm));
    GF_HIP(hipMemcpyAsync(S->dtile[slot], htile, gf_serve_tile_size() * ntiles, hipMemcpyHostToDevice, sm));
    gf_status st = gf_serve_launch(S->dreq[slot], S->dtile[slot], ntiles, (int)nunits, S->tile_rays, S->max_tiles,
                                   S->ws[slot], sm);
    if (st != GF_OK) return st;
    GF_HIP(hipEventRecord(b.ev, sm));
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
    if (bytes_held) *bytes_held = S->mem.held;
    return GF_OK;
}

// The executor's policy on a virtual clock, with no device work: requests
// arrive at arrival_s[i]; each step retires the batches whose end has
// passed, admits queued requests in arrival order while their rays fit the
// pool, and launches a batch while fewer than two are in flight.  A batch
// runs after the previous one ends and takes sum(rays x spp x (3 if
// multiple)) / work_per_s seconds.
extern "C" gf_status gf_server_simulate(size_t mem_budget, int tile_rays, int max_tiles, int64_t n,
                                        const int32_t* width, const int32_t* height, const int32_t* spp,
                                        const int32_t* multiple, const double* arrival_s, double work_per_s,
                                        double* admit_s, double* done_s, size_t* max_held) {
    if (n < 0 || (n > 0 && (!width || !height || !spp || !multiple || !arrival_s || !admit_s || !done_s)))
        return gf_fail(GF_EINVAL, "gf_server_simulate: NULL argument");
    if (mem_budget < kAlign || tile_rays < 64 || tile_rays > (1 << 20) || max_tiles < 1 || max_tiles > 65536 ||
        !(work_per_s > 0.0))
        return gf_fail(GF_EINVAL, "gf_server_simulate: budget >= 256 B, 64 <= tile_rays <= 2^20, "
                                  "1 <= max_tiles <= 65536, work_per_s > 0");
    gfs::Pool mem;
    mem.reset(mem_budget / kAlign * kAlign);
    std::vector<gfs::SchedReq> reqs((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        if (width[i] < 1 || height[i] < 1 || spp[i] < 1 || (int64_t)width[i] * height[i] > (1 << 28))
            return gf_fail(GF_EINVAL, "gf_server_simulate: request %lld has an invalid size", (long long)i);
        if (i > 0 && arrival_s[i] < arrival_s[i - 1])
            return gf_fail(GF_EINVAL, "gf_server_simulate: arrivals must be sorted");
        gfs::SchedReq& r = reqs[(size_t)i];
        r.id = (uint64_t)i;
        r.n = width[i] * height[i];
        r.spp = spp[i];
        r.multiple = multiple[i] != 0;
        r.bytes = gfs::request_bytes(width[i], height[i], spp[i]);
        r.off = 0;
        r.next_ray = r.rays_done = 0;
        if (r.bytes > mem.budget)
            return gf_fail(GF_EINVAL, "gf_server_simulate: request %lld needs %zu bytes, budget %zu", (long long)i,
                           r.bytes, mem.budget);
        admit_s[i] = done_s[i] = -1.0;
    }
    struct VBatch {
        double end;
        std::vector<std::pair<gfs::SchedReq*, int>> work;
    };
    std::deque<gfs::SchedReq*> queue;
    std::vector<gfs::SchedReq*> active;
    std::deque<VBatch> inflight;
    double now = 0.0, last_end = 0.0;
    int64_t next = 0, finished = 0;
    size_t peak = 0;
    while (finished < n) {
        while (next < n && arrival_s[next] <= now) queue.push_back(&reqs[(size_t)next++]);
        while (!inflight.empty() && inflight.front().end <= now) {
            for (auto& w : inflight.front().work) {
                gfs::SchedReq* r = w.first;
                r->rays_done += w.second;
                if (r->rays_done == r->n) {
                    mem.release(r->off, r->bytes);
                    active.erase(std::find(active.begin(), active.end(), r));
                    done_s[r->id] = inflight.front().end;
                    ++finished;
                }
            }
            inflight.pop_front();
        }
        while (!queue.empty()) {
            size_t off;
            if (!mem.alloc(queue.front()->bytes, &off)) break;
            queue.front()->off = off;
            admit_s[queue.front()->id] = now;
            active.push_back(queue.front());
            queue.pop_front();
        }
        peak = std::max(peak, mem.held);
        while ((int)inflight.size() < kSlots) {
            std::vector<gfs::TileRef> plan = gfs::plan_batch(active, tile_rays, max_tiles);
            if (plan.empty()) break;
            VBatch b;
            double work = 0.0;
            std::map<gfs::SchedReq*, int> rays_in;
            for (const gfs::TileRef& t : plan) {
                work += (double)t.count * t.r->spp * (t.r->multiple ? 3.0 : 1.0);
                rays_in[t.r] += t.count;
            }
            for (auto& kv : rays_in) b.work.push_back(kv);
            b.end = std::max(now, last_end) + work / work_per_s;
            last_end = b.end;
            inflight.push_back(b);
        }
        if (finished == n) break;
        double t_next = INFINITY;
        if (next < n) t_next = arrival_s[next];
        if (!inflight.empty()) t_next = std::min(t_next, inflight.front().end);
        if (!(t_next < INFINITY)) return gf_fail(GF_ESTATE, "gf_server_simulate: no event left");
        now = std::max(now, t_next);
    }
    if (max_held) *max_held = peak;
    return GF_OK;
}
