// Internal definitions of the Gabor-field HIP library (gfx950).
//
// Device data layout of a resident scene (all in HBM, Morton order):
//   prims  : n x 64 B records (4 x float4), read wave-uniformly through the
//            scalar cache by the packet traversal:
//            [mu.x mu.y mu.z phi] [A00 A01 A02 A11] [A12 A22 f.x f.y]
//            [f.z amp r^2 (orig | cell << 28)]  with A = Sigma^-1 (float32),
//            amp = rho alpha / (4 pi s0 s1 s2), r the primitive's truncation
//            radius (the scene's, or less under adaptive clamping), cell =
//            3 level + bin, orig = caller index (< 2^28).
//   nodes  : (n-1) x 64 B traversal records of the internal LBVH nodes, each
//            holding both child boxes so one scalar load tests both children:
//            [lbox lo/hi] [rbox lo/hi] [lchild rchild cells pad]; a child id
//            c >= 0 is an internal node, c < 0 is the leaf (Morton index) ~c.
//   cnodes : the same records with every subtree of at most GF_LEAF_MAX
//            primitives collapsed into a leaf range: c < 0 is the Morton
//            range first = ~c & 0x0FFFFFFF, count = (~c >> 28) + 1 (the
//            subtree's primitives are contiguous in Morton order).
//   A64    : n x 64 B, Sigma^-1 (6) and the squared truncation radius in
//            binary64 (one pad) for the chord geometry of the
//            optical-depth and adjoint kernels (float32 rounding of an
//            anisotropic Sigma^-1 moves h^2 by ~1e-5 relative).
//   grid   : G^3 voxels x 12 cells of float32 majorants over the root box.
//   canon  : the canonical LBVH arrays (keys, perm, left, right, parent,
//            aabb, cellor) kept for export and refit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gaborfields.h"

#define GF_NCELLS 12
#define GF_STACK 128
#define GF_LEAF_MAX 4
#define GF_A64 8  // binary64 words per primitive in SceneView::A64

// last word of a primitive record: caller index in the low 28 bits, cell above
static __device__ __forceinline__ int rec_orig(float w) { return __float_as_int(w) & 0x0FFFFFFF; }
static __device__ __forceinline__ int rec_cell(float w) { return (int)((unsigned)__float_as_int(w) >> 28); }
static __device__ __forceinline__ float rec_word(int orig, int cell) {
    return __int_as_float((int)((unsigned)orig | ((unsigned)cell << 28)));
}

// Leaf range of a collapsed child id c < 0.
static __device__ __forceinline__ void leaf_range(int c, int* first, int* count) {
    unsigned v = ~(unsigned)c;
    *first = (int)(v & 0x0FFFFFFFu);
    *count = (int)(v >> 28) + 1;
}

struct TNode {
    float lbox[6];
    float rbox[6];
    int lchild, rchild;
    uint32_t cells;  // low 16 bits: left subtree cells, high 16 bits: right
    int pad;
};
static_assert(sizeof(TNode) == 64, "traversal node must be 64 bytes");

// Scene as seen by kernels (passed by value).
struct SceneView {
    const float4* __restrict__ prims;
    const TNode* __restrict__ nodes;
    const TNode* __restrict__ cnodes;  // the same tree with small subtrees collapsed into leaf ranges
    int croot;                         // root as a leaf range (< 0) when the whole scene is one, else 0
    const float* __restrict__ grid;
    const float4* __restrict__ aux;
    const double* __restrict__ A64;  // GF_A64 per primitive: a00 a01 a02 a11 a12 a22, r^2, pad
    int n;
    float r, r2;
    int G;
    float glo[3], ghi[3], ginv[3];  // grid box and voxels per unit length
    float med[GF_NCELLS];           // per-cell median |k_W|
};

struct MaskView {
    uint32_t cells;                          // 12 used bits
    const uint32_t* __restrict__ prim_bits;  // caller order, may be null
    float lod_k;                             // continuous-LOD cutoff (0: off)
    float lod2;                              // its square
};

struct gf_scene_s {
    int device;
    int64_t n;
    float rho, r, clamp_eps;
    int G;
    int depth;  // largest number of internal nodes on a root-to-leaf path
    double fmax2;
    float lo[3], hi[3];
    uint64_t nonempty;
    int64_t cell_count[GF_NCELLS];
    float med[GF_NCELLS];
    // device memory
    float4* prims;
    double* A64;  // Sigma^-1 in binary64 (Morton order), 6 per primitive
    float4* aux;  // adjoint data, 3 x float4 per primitive (Morton
                  // order): [q w x y z (caller's)] [|q| s0 s1 s2] [alpha, rho/(4 pi s0 s1 s2), 0, 0]
    TNode* nodes;
    TNode* cnodes;
    float* grid;
    uint64_t* keys;
    int32_t* perm;
    int32_t* left;
    int32_t* right;
    int32_t* parent;
    float* aabb;
    uint64_t* cellor;
    size_t bytes;
};

// ---------------------------------------------------------------------------
// error reporting
// ---------------------------------------------------------------------------
gf_status gf_fail(gf_status st, const char* fmt, ...);
gf_status gf_hip_check(hipError_t e, const char* what);
#define GF_HIP(call)                                               \
    do {                                                           \
        hipError_t _e = (call);                                    \
        if (_e != hipSuccess) return gf_hip_check(_e, #call);      \
    } while (0)

// Weideman coefficients live in constant memory of every translation unit
// that evaluates w(z); gf_ensure_weideman() uploads them once per device.
gf_status gf_ensure_weideman_tau();
gf_status gf_ensure_weideman_grad();

SceneView gf_scene_view(const gf_scene_s* s);
unsigned gf_packet_blocks(int64_t n, int tile_w);
gf_status gf_check_rays(int64_t n, int tile_w, const char* who);
MaskView gf_mask_view(const gf_mask& m);
gf_status gf_check_mask(const gf_mask& m, const char* who);
// Rejects (GF_EINVAL) rays with a NaN/Inf origin, direction or tmin, a NaN
// tmax, |v| = 0 or tmin > tmax: one check kernel on `sm`, whose verdict the
// call waits for, before any compute kernel is launched.
gf_status gf_validate_rays(const float* rays, int64_t n, hipStream_t sm, const char* who);

// Zeroes `words` 32-bit words with a fill kernel on `sm` (a kernel rather
// than a memset node, so the call can sit in a captured HIP graph).
gf_status gf_zero_words(void* p, size_t words, hipStream_t sm);

// Tracking workspace of the render kernels: a head of GF_TRACK_HEAD_FLOATS
// floats (the launch's chunk counter), then GF_TRACK_WAVE_FLOATS floats per
// resident wave.
#define GF_TRACK_HEAD_FLOATS 64
#define GF_TRACK_WAVE_FLOATS (256 * 64)

// host helpers of the render and serving code (gf_track.hip)
gf_status gf_check_track_depth(const gf_scene_s* s, const char* who);
// render of n rays with the tracking workspace ws (head + ws_waves slices;
// the launch uses at most that many waves) and a per-sample buffer part of
// part_cap floats (used when it holds gf_render_part_floats); outputs as
// gf_render
size_t gf_render_part_floats(const gf_render_desc* d, int64_t n, int tile_w);
gf_status gf_render_launch_in(gf_scene s, const float* rays, int64_t n, int image_width, const gf_render_desc* d,
                              float* ws, int64_t ws_waves, float* part, size_t part_cap, float* radiance,
                              float* primary_T, hipStream_t sm);
gf_status gf_camera_launch(const gf_camera* cam, float* rays, hipStream_t sm);
gf_status gf_check_camera(const gf_camera* cam, const char* who);
gf_status gf_check_render_desc(const gf_render_desc* d, const char* who);
gf_status gf_ensure_weideman_track();

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
#define GF_PI 3.14159265358979323846
#define GF_INV_2PI 0.15915494309189533577

static __device__ __forceinline__ int lane_id() { return __lane_id(); }

static __device__ __forceinline__ uint64_t lanemask_lt() {
    int l = __lane_id();
    return l ? (~0ull >> (64 - l)) : 0ull;
}

static __device__ __forceinline__ int uniform_int(int x) { return __builtin_amdgcn_readfirstlane(x); }


// sin / cos of 2 pi x for |x| <= 0.5
static __device__ __forceinline__ void sincos2pi(float x, float* s, float* c) { sincospif(2.0f * x, s, c); }

// sin and cos of 2 pi c for a phase c in cycles (binary64), each with a
// small relative error also near its zeros: c is reduced to the nearest
// quarter cycle q / 4 in binary64, the remainder x (|x| <= 1/8) becomes
// float32 with full relative precision, and q mod 4 turns sin / cos of
// 2 pi x into those of 2 pi c.
static __device__ __forceinline__ void sincos_cycles(double c, float* s, float* co) {
    const double q = rint(4.0 * c);
    const float x = (float)(c - 0.25 * q);
    float sx, cx;
    sincospif(2.0f * x, &sx, &cx);
    switch ((int)((long long)q & 3)) {
        case 0: *s = sx; *co = cx; break;
        case 1: *s = cx; *co = -sx; break;
        case 2: *s = -sx; *co = -cx; break;
        default: *s = -cx; *co = sx; break;
    }
}

// Philox4x32-10 (Salmon et al., SC 2011): 10 rounds of two 32x32->64
// multiplications with Weyl-sequence key bumps.
static __device__ __forceinline__ uint4 philox4x32(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// uniform in (0, 1) from 32 random bits: ((x >> 8) + 0.5) 2^-24
static __device__ __forceinline__ float unit_float(uint32_t x) { return ((float)(x >> 8) + 0.5f) * (1.0f / 16777216.0f); }

// Counter-based stream: key = seed, counter = (a, b, block, tag).
struct Rng {
    uint32_t k0, k1, a, b, tag, blk;
    uint4 buf;
    int used;
    __device__ void init(uint64_t seed, uint32_t a_, uint32_t b_, uint32_t tag_) {
        k0 = (uint32_t)seed;
        k1 = (uint32_t)(seed >> 32);
        a = a_;
        b = b_;
        tag = tag_;
        blk = 0;
        used = 4;
    }
    // next 32 random bits of the stream
    __device__ uint32_t bits() {
        if (used == 4) {
            buf = philox4x32(make_uint4(a, b, blk, tag), k0, k1);
            ++blk;
            used = 0;
        }
        uint32_t x = used == 0 ? buf.x : used == 1 ? buf.y : used == 2 ? buf.z : buf.w;
        ++used;
        return x;
    }
    // uniform in (0, 1): ((x >> 8) + 0.5) 2^-24
    __device__ float u() { return unit_float(bits()); }
};

static __device__ __forceinline__ bool mask_keep(const MaskView& m, int cell, int orig) {
    if (!((m.cells >> cell) & 1u)) return false;
    if (m.prim_bits && !((m.prim_bits[orig >> 5] >> (orig & 31)) & 1u)) return false;
    return true;
}

// Robust slab test of a ray against a box (conservative: the far distance is
// inflated by a few ulps so that rounding never rejects a grazing chord).
static __device__ __forceinline__ bool slab_hit(const float* b, float ox, float oy, float oz, float ix, float iy,
                                                float iz, float tmin, float tmax) {
    float t0x = (b[0] - ox) * ix, t1x = (b[3] - ox) * ix;
    float t0y = (b[1] - oy) * iy, t1y = (b[4] - oy) * iy;
    float t0z = (b[2] - oz) * iz, t1z = (b[5] - oz) * iz;
    float tn = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), tmin));
    float tf = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
    return tn <= tf + fabsf(tf) * 1e-6f + 1e-30f;
}

static __device__ __forceinline__ bool box_contains(const float* b, float x, float y, float z) {
    return x >= b[0] && x <= b[3] && y >= b[1] && y <= b[4] && z >= b[2] && z <= b[5];
}

// Majorant of |kappa| in the voxel holding grid index (ix, iy, iz) for a set of
// per-cell weights.
static __device__ __forceinline__ float voxel_majorant(const SceneView& S, int vox, const float* cw) {
    const float* g = S.grid + (size_t)vox * GF_NCELLS;
    float acc = 0.0f;
#pragma unroll
    for (int c = 0; c < GF_NCELLS; ++c) acc += cw[c] * g[c];
    return acc;
}
