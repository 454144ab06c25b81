// Host-side policy of the serving executor, free of device calls so that the
// executor and its virtual-clock simulation share one implementation:
// * a first-fit pool allocator with coalescing free list (offsets into one
//   device block of `budget` bytes, 256 B aligned);
// * batch planning: the open requests (admitted, rays left to schedule) in
//   order of least remaining work first (rays left x samples, multiple
//   scattering weighted 3x; arrival order among equals), cut into tiles of at
//   most `tile_rays` rays, at most `max_tiles` tiles per batch.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

namespace gfs {

const size_t kAlign = 256;

struct FreeBlock {
    size_t off, size;
};

struct Pool {
    size_t budget = 0, held = 0;
    std::vector<FreeBlock> freel;  // sorted by offset, coalesced

    void reset(size_t bytes) {
        budget = bytes;
        held = 0;
        freel.assign(1, FreeBlock{0, bytes});
    }
    bool alloc(size_t bytes, size_t* off) {
        for (size_t i = 0; i < freel.size(); ++i) {
            FreeBlock& b = freel[i];
            if (b.size >= bytes) {
                *off = b.off;
                b.off += bytes;
                b.size -= bytes;
                if (b.size == 0) freel.erase(freel.begin() + i);
                held += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto it = std::lower_bound(freel.begin(), freel.end(), off,
                                   [](const FreeBlock& b, size_t o) { return b.off < o; });
        it = freel.insert(it, FreeBlock{off, bytes});
        size_t i = it - freel.begin();
        if (i + 1 < freel.size() && freel[i].off + freel[i].size == freel[i + 1].off) {
            freel[i].size += freel[i + 1].size;
            freel.erase(freel.begin() + i + 1);
        }
        if (i > 0 && freel[i - 1].off + freel[i - 1].size == freel[i].off) {
            freel[i - 1].size += freel[i].size;
            freel.erase(freel.begin() + i);
        }
        held -= bytes;
    }
};

static inline size_t align_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// pool bytes of a request: its camera rays (8 float32 per pixel), then one
// float32 radiance per pixel and sample
static inline size_t request_ray_bytes(int64_t width, int64_t height) {
    return align_up((size_t)(width * height) * 8 * sizeof(float));
}
static inline size_t request_bytes(int64_t width, int64_t height, int64_t spp) {
    return request_ray_bytes(width, height) + align_up((size_t)(width * height * spp) * sizeof(float));
}

struct SchedReq {
    uint64_t id;
    int n;          // rays
    int spp;
    bool multiple;
    size_t bytes, off;
    int next_ray;   // first ray not yet put in a batch
    int rays_done;  // rays whose batch completed
};

struct TileRef {
    SchedReq* r;
    int first, count;
};

static inline double remaining_work(const SchedReq* r) {
    return (double)(r->n - r->next_ray) * r->spp * (r->multiple ? 3.0 : 1.0);
}

// Tiles of the next batch (empty when no admitted request has rays left);
// advances each request's next_ray.  `active` is in admission order.
static inline std::vector<TileRef> plan_batch(const std::vector<SchedReq*>& active, int tile_rays, int max_tiles) {
    std::vector<SchedReq*> open;
    for (SchedReq* r : active)
        if (r->next_ray < r->n) open.push_back(r);
    std::stable_sort(open.begin(), open.end(),
                     [](const SchedReq* a, const SchedReq* b) { return remaining_work(a) < remaining_work(b); });
    std::vector<TileRef> tiles;
    for (SchedReq* r : open) {
        while ((int)tiles.size() < max_tiles && r->next_ray < r->n) {
            int cnt = std::min(tile_rays, r->n - r->next_ray);
            tiles.push_back(TileRef{r, r->next_ray, cnt});
            r->next_ray += cnt;
        }
    }
    return tiles;
}

}  // namespace gfs
