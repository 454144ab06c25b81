// Allocation-free camera render (gf_render_noalloc): the same kernels as
// gf_render with the workspace in a file-scope device array.
#include <mutex>

#include "gf_internal.hpp"

// ---------------------------------------------------------------------------
// Camera render without allocation (gf_render_noalloc).  Its workspace is a
// file-scope device array: the camera rays of at most NOALLOC_MAX_PIXELS
// pixels, then the tracking slices of NOALLOC_WAVES resident waves (the
// render's waves loop over the image's chunks, so fewer resident waves than
// chunks only costs time), then NOALLOC_PART_FLOATS floats of per-sample
// storage (a render whose samples need more keeps each chunk's samples in
// one work unit: slower on images with a few very dense tiles, the same
// bits).  Each device holds its own copy for the life of
// the process; host code reaches it through the address hipGetSymbolAddress
// returns on that device, kept per device.  Calls that overlap on one device
// share the array and race.
// ---------------------------------------------------------------------------
#define NOALLOC_MAX_PIXELS (1 << 20)
#define NOALLOC_WAVES 1024
#define NOALLOC_RAY_FLOATS ((size_t)NOALLOC_MAX_PIXELS * 8)
#define NOALLOC_TRACK_FLOATS ((size_t)GF_TRACK_HEAD_FLOATS + (size_t)NOALLOC_WAVES * GF_TRACK_WAVE_FLOATS)
#define NOALLOC_PART_FLOATS ((size_t)8 << 20)
#define NOALLOC_FLOATS (NOALLOC_RAY_FLOATS + NOALLOC_TRACK_FLOATS + NOALLOC_PART_FLOATS)

static __device__ __align__(256) float scratch[NOALLOC_FLOATS];

#define NOALLOC_DEVICES 64
static float* g_scratch_ptr[NOALLOC_DEVICES];
static std::mutex g_scratch_mu;

static gf_status scratch_address(float** out) {
    int dev = 0;
    GF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_DEVICES) return gf_fail(GF_EDEVICE, "gf_render_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        float* p = nullptr;
        hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return gf_hip_check(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GF_OK;
}

extern "C" gf_status gf_render_noalloc(gf_scene s, const gf_camera* cam, const gf_render_desc* d, float* radiance,
                                       float* primary_T, void* stream) {
    gf_status st = gf_check_camera(cam, "gf_render_noalloc");
    if (st == GF_OK) st = gf_check_render_desc(d, "gf_render_noalloc");
    if (st != GF_OK) return st;
    if (!s || !radiance) return gf_fail(GF_EINVAL, "gf_render_noalloc: NULL argument");
    const int64_t n = (int64_t)cam->width * cam->height;
    if (n > NOALLOC_MAX_PIXELS)
        return gf_fail(GF_EINVAL, "gf_render_noalloc: %lld pixels exceed its fixed workspace of %d pixels", (long long)n,
                       NOALLOC_MAX_PIXELS);
    st = gf_check_track_depth(s, "gf_render_noalloc");
    if (st != GF_OK) return st;
    float* base = nullptr;
    st = scratch_address(&base);
    if (st != GF_OK) return st;
    hipStream_t sm = (hipStream_t)stream;
    const int tile_w = cam->width % 8 == 0 ? cam->width : 0;
    st = gf_camera_launch(cam, base, sm);
    if (st != GF_OK) return st;
    return gf_render_launch_in(s, base, n, tile_w, d, base + NOALLOC_RAY_FLOATS, NOALLOC_WAVES,
                               base + NOALLOC_RAY_FLOATS + NOALLOC_TRACK_FLOATS, NOALLOC_PART_FLOATS, radiance,
                               primary_T, sm);
}
