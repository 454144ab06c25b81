// Scene construction for the Gabor-field library (gfx950): validation,
// derived per-primitive constants, Morton keys, stable LSD radix sort, Karras
// radix tree, bottom-up box refit, traversal records and majorant grid.
//
// The Morton quantisation and the leaf boxes follow a bit-exact
// specification (written in include/gaborfields.h at gf_scene_create) and are
// evaluated without floating-point contraction.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "gf_internal.hpp"

// ---------------------------------------------------------------------------
// error state
// ---------------------------------------------------------------------------
static thread_local char g_err[512] = "";

gf_status gf_fail(gf_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

gf_status gf_hip_check(hipError_t e, const char* what) {
    return gf_fail(e == hipErrorOutOfMemory ? GF_ENOMEM : GF_EDEVICE, "%s failed: %s", what, hipGetErrorString(e));
}

extern "C" const char* gf_last_error(void) { return g_err; }

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
static __device__ __forceinline__ uint64_t spread21(uint64_t x) {
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// |f|^2 in the fixed order (fx^2 + fy^2) + fz^2, binary64, no contraction
static __device__ __forceinline__ double fnorm2(const float* p) {
#pragma clang fp contract(off)
    double fx = p[10], fy = p[11], fz = p[12];
    return (fx * fx + fy * fy) + fz * fz;
}

static __device__ __forceinline__ int cell_of(const float* p, double fmax2) {
#pragma clang fp contract(off)
    double f2 = fnorm2(p);
    int lev = (f2 <= fmax2 / 64.0) ? 0 : (f2 <= fmax2 / 16.0) ? 1 : (f2 <= fmax2 / 4.0) ? 2 : 3;
    double a = (double)p[10] * (double)p[10], b = (double)p[11] * (double)p[11], c = (double)p[12] * (double)p[12];
    int bin = 0;
    double best = a;
    if (b > best) { bin = 1; best = b; }
    if (c > best) bin = 2;
    return lev * 3 + bin;
}

// rotation of the normalised quaternion, binary64, no contraction
static __device__ __forceinline__ void rotation64(const float* p, double R[3][3], double qh[4]) {
#pragma clang fp contract(off)
    double w = p[3], x = p[4], y = p[5], z = p[6];
    double qn = sqrt(((w * w + x * x) + y * y) + z * z);
    w = w / qn;
    x = x / qn;
    y = y / qn;
    z = z / qn;
    qh[0] = w; qh[1] = x; qh[2] = y; qh[3] = z;
    R[0][0] = 1.0 - 2.0 * (y * y + z * z);
    R[0][1] = 2.0 * (x * y - w * z);
    R[0][2] = 2.0 * (x * z + w * y);
    R[1][0] = 2.0 * (x * y + w * z);
    R[1][1] = 1.0 - 2.0 * (x * x + z * z);
    R[1][2] = 2.0 * (y * z - w * x);
    R[2][0] = 2.0 * (x * z - w * y);
    R[2][1] = 2.0 * (y * z + w * x);
    R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

// ---------------------------------------------------------------------------
// 1. validation and bounds
// ---------------------------------------------------------------------------
struct BoundsPartial {
    float lo[3], hi[3];
    double f2max;
    int bad;
    int pad;
};

__global__ __launch_bounds__(256) void k_bounds_partial(const float* __restrict__ params, int n,
                                                        BoundsPartial* __restrict__ out) {
    __shared__ BoundsPartial sh[256];
    BoundsPartial b;
    for (int a = 0; a < 3; ++a) { b.lo[a] = INFINITY; b.hi[a] = -INFINITY; }
    b.f2max = 0.0;
    b.bad = 0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const float* p = params + (size_t)i * 15;
        int bad = 0;
        for (int k = 0; k < 15; ++k) bad |= !isfinite(p[k]);
        bad |= !(p[7] > 0.0f) || !(p[8] > 0.0f) || !(p[9] > 0.0f);
        bad |= (p[3] == 0.0f && p[4] == 0.0f && p[5] == 0.0f && p[6] == 0.0f);
        b.bad |= bad;
        for (int a = 0; a < 3; ++a) {
            b.lo[a] = fminf(b.lo[a], p[a]);
            b.hi[a] = fmaxf(b.hi[a], p[a]);
        }
        double f2 = fnorm2(p);
        b.f2max = f2 > b.f2max ? f2 : b.f2max;
    }
    sh[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            BoundsPartial& x = sh[threadIdx.x];
            const BoundsPartial& y = sh[threadIdx.x + s];
            for (int a = 0; a < 3; ++a) {
                x.lo[a] = fminf(x.lo[a], y.lo[a]);
                x.hi[a] = fmaxf(x.hi[a], y.hi[a]);
            }
            x.f2max = y.f2max > x.f2max ? y.f2max : x.f2max;
            x.bad |= y.bad;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_bounds_final(BoundsPartial* __restrict__ parts, int m) {
    __shared__ BoundsPartial sh[256];
    BoundsPartial b;
    for (int a = 0; a < 3; ++a) { b.lo[a] = INFINITY; b.hi[a] = -INFINITY; }
    b.f2max = 0.0;
    b.bad = 0;
    for (int i = threadIdx.x; i < m; i += 256) {
        const BoundsPartial& y = parts[i];
        for (int a = 0; a < 3; ++a) {
            b.lo[a] = fminf(b.lo[a], y.lo[a]);
            b.hi[a] = fmaxf(b.hi[a], y.hi[a]);
        }
        b.f2max = y.f2max > b.f2max ? y.f2max : b.f2max;
        b.bad |= y.bad;
    }
    sh[threadIdx.x] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            BoundsPartial& x = sh[threadIdx.x];
            const BoundsPartial& y = sh[threadIdx.x + s];
            for (int a = 0; a < 3; ++a) {
                x.lo[a] = fminf(x.lo[a], y.lo[a]);
                x.hi[a] = fmaxf(x.hi[a], y.hi[a]);
            }
            x.f2max = y.f2max > x.f2max ? y.f2max : x.f2max;
            x.bad |= y.bad;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) parts[0] = sh[0];
}

// ---------------------------------------------------------------------------
// 2. Morton keys (caller order)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_morton(const float* __restrict__ params, int n,
                                                const BoundsPartial* __restrict__ bnd, uint64_t* __restrict__ keys,
                                                uint32_t* __restrict__ vals) {
#pragma clang fp contract(off)
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float* p = params + (size_t)i * 15;
    uint64_t q[3];
    for (int a = 0; a < 3; ++a) {
        double lo = bnd->lo[a], hi = bnd->hi[a];
        if (hi == lo) {
            q[a] = 0;
            continue;
        }
        double scale = 2097152.0 / (hi - lo);
        double t = floor(((double)p[a] - lo) * scale);
        q[a] = t >= 2097151.0 ? 2097151ull : (uint64_t)t;
    }
    keys[i] = (spread21(q[0]) << 2) | (spread21(q[1]) << 1) | spread21(q[2]);
    vals[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// 3. stable LSD radix sort of (u64 key, u32 value), 4-bit digits
//    tile = 256 threads x 8 items; per tile digit counts -> column-major
//    exclusive scan -> stable scatter (in-tile ranks from wave ballots)
// ---------------------------------------------------------------------------
#define RS_THREADS 256
#define RS_ITEMS 8
#define RS_TILE (RS_THREADS * RS_ITEMS)
#define RS_DIGITS 16

__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint64_t* __restrict__ keys, int n, int shift,
                                                        uint32_t* __restrict__ hist, int ntiles) {
    __shared__ uint32_t cnt[RS_DIGITS];
    if (threadIdx.x < RS_DIGITS) cnt[threadIdx.x] = 0;
    __syncthreads();
    int base = blockIdx.x * RS_TILE;
    for (int k = 0; k < RS_ITEMS; ++k) {
        int i = base + k * RS_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 15], 1u);
    }
    __syncthreads();
    if (threadIdx.x < RS_DIGITS) hist[threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// exclusive scan of m values in one block of 1024 threads
__global__ __launch_bounds__(1024) void k_scan_excl(uint32_t* __restrict__ a, int m) {
    __shared__ uint32_t part[1024];
    int per = (m + 1023) / 1024;
    int b = threadIdx.x * per, e = min(m, b + per);
    uint32_t s = 0;
    for (int i = b; i < e; ++i) s += a[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - s;
    for (int i = b; i < e; ++i) {
        uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
}

__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
                                                           uint32_t* __restrict__ vout, int n, int shift,
                                                           const uint32_t* __restrict__ hist, int ntiles) {
    __shared__ uint32_t run[RS_DIGITS];
    __shared__ uint32_t wcnt[RS_THREADS / 64][RS_DIGITS];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (threadIdx.x < RS_DIGITS) run[threadIdx.x] = hist[threadIdx.x * ntiles + blockIdx.x];
    __syncthreads();
    int base = blockIdx.x * RS_TILE;
    for (int k = 0; k < RS_ITEMS; ++k) {
        int i = base + k * RS_THREADS + threadIdx.x;
        bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0;
        uint32_t val = valid ? vin[i] : 0;
        int d = valid ? (int)((key >> shift) & 15) : -1;
        uint32_t myrank = 0;
        for (int dd = 0; dd < RS_DIGITS; ++dd) {
            uint64_t m = __ballot(d == dd);
            if (d == dd) myrank = __popcll(m & lanemask_lt());
            if (lane == 0) wcnt[wave][dd] = __popcll(m);
        }
        __syncthreads();
        if (valid) {
            uint32_t off = run[d];
            for (int w = 0; w < wave; ++w) off += wcnt[w][d];
            off += myrank;
            kout[off] = key;
            vout[off] = val;
        }
        __syncthreads();
        if (threadIdx.x < RS_DIGITS) {
            uint32_t t = 0;
            for (int w = 0; w < RS_THREADS / 64; ++w) t += wcnt[w][threadIdx.x];
            run[threadIdx.x] += t;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// 4. Karras radix tree (HPG 2012) over the sorted keys
// ---------------------------------------------------------------------------
static __device__ __forceinline__ int kdelta(const uint64_t* __restrict__ k, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    uint64_t a = k[i], b = k[j];
    if (a != b) return __clzll((long long)(a ^ b));
    uint32_t x = (uint32_t)i ^ (uint32_t)j;
    return 64 + (x ? __clz((int)x) : 32);
}

__global__ __launch_bounds__(256) void k_karras(const uint64_t* __restrict__ keys, int n, int32_t* __restrict__ left,
                                                int32_t* __restrict__ right, int32_t* __restrict__ parent,
                                                int2* __restrict__ range) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n - 1) return;
    int d = (kdelta(keys, n, i, i + 1) - kdelta(keys, n, i, i - 1)) > 0 ? 1 : -1;
    int dmin = kdelta(keys, n, i, i - d);
    int lmax = 2;
    while (kdelta(keys, n, i, i + lmax * d) > dmin) lmax *= 2;
    int l = 0;
    for (int t = lmax / 2; t >= 1; t /= 2)
        if (kdelta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = kdelta(keys, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (kdelta(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int g = i + s * d + (d < 0 ? -1 : 0);
    int first = min(i, j), last = max(i, j);
    int L0 = n - 1;
    int lc = (first == g) ? L0 + g : g;
    int rc = (last == g + 1) ? L0 + g + 1 : g + 1;
    left[i] = lc;
    right[i] = rc;
    parent[lc] = i;
    parent[rc] = i;
    range[i] = make_int2(first, last);
}

// ---------------------------------------------------------------------------
// 5. Morton-ordered primitive records and leaf boxes
// ---------------------------------------------------------------------------
// Adaptive clamping (Sec. 4.4): the truncation radius of a primitive whose
// kernel magnitude rho |alpha| (2 pi)^-3/2 / (s0 s1 s2) exp(-E^2/2), taken on
// the ray of largest chord measure (times s_max / sqrt(2 pi) for the
// integral across it), drops below eps at Mahalanobis radius E:
// E^2 = 2 ln(rho |alpha| s_max / (2 pi s0 s1 s2 eps)); the radius is
// min(r, E), 0 when E^2 <= 0.  The paper's own extent drops alpha and the
// Jacobian and subtracts |k_W|^2, which no ray perpendicular to k_W
// attains, so it is no bound; the carrier is left out here.  eps = 0: r.
static __device__ double clamp_radius(const float* p, double r, double rho, double eps) {
#pragma clang fp contract(off)
    if (!(eps > 0.0)) return r;
    double s0 = p[7], s1 = p[8], s2 = p[9];
    double smax = fmax(s0, fmax(s1, s2));
    double arg = rho * fabs((double)p[14]) * smax / (2.0 * GF_PI * s0 * s1 * s2 * eps);
    if (!(arg > 1.0)) return 0.0;
    double E = sqrt(2.0 * log(arg));
    return E < r ? E : r;
}

__global__ __launch_bounds__(256) void k_leaves(const float* __restrict__ params, int n, float r, float rho,
                                                float clamp_eps,
                                                const BoundsPartial* __restrict__ bnd, const uint32_t* __restrict__ perm,
                                                float4* __restrict__ prims, float* __restrict__ aabb,
                                                uint64_t* __restrict__ cellor, float* __restrict__ kw,
                                                float4* __restrict__ aux, double* __restrict__ A64) {
    int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    int i = (int)perm[j];
    const float* p = params + (size_t)i * 15;
    double R[3][3], qh[4];
    rotation64(p, R, qh);
    double s[3] = {p[7], p[8], p[9]};
    float* bx = aabb + (size_t)(n - 1 + j) * 6;
    const double rr = clamp_radius(p, (double)r, (double)rho, (double)clamp_eps);
    {
#pragma clang fp contract(off)
        for (int a = 0; a < 3; ++a) {
            double t0 = R[a][0] * s[0], t1 = R[a][1] * s[1], t2 = R[a][2] * s[2];
            double e = rr * sqrt((t0 * t0 + t1 * t1) + t2 * t2);
            bx[a] = __double2float_rd((double)p[a] - e);
            bx[3 + a] = __double2float_ru((double)p[a] + e);
        }
    }
    int cell = cell_of(p, bnd->f2max);
    cellor[n - 1 + j] = 1ull << cell;
    double A[6];
    int idx = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = a; b < 3; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += R[a][k] * R[b][k] / (s[k] * s[k]);
            A[idx++] = acc;
        }
    for (int k = 0; k < 6; ++k) A64[(size_t)j * GF_A64 + k] = A[k];
    A64[(size_t)j * GF_A64 + 6] = rr * rr;
    A64[(size_t)j * GF_A64 + 7] = 0.0;
    double amp = (double)rho * (double)p[14] / (4.0 * GF_PI * s[0] * s[1] * s[2]);
    float4* rec = prims + (size_t)j * 4;
    rec[0] = make_float4(p[0], p[1], p[2], p[13]);
    rec[1] = make_float4((float)A[0], (float)A[1], (float)A[2], (float)A[3]);
    rec[2] = make_float4((float)A[4], (float)A[5], p[10], p[11]);
    rec[3] = make_float4(p[12], (float)amp, (float)(rr * rr), rec_word(i, cell));
    double qn = sqrt(((double)p[3] * p[3] + (double)p[4] * p[4]) + (double)p[5] * p[5] + (double)p[6] * p[6]);
    float4* ax = aux + (size_t)j * 3;
    ax[0] = make_float4(p[3], p[4], p[5], p[6]);
    ax[1] = make_float4((float)qn, p[7], p[8], p[9]);
    ax[2] = make_float4(p[14], (float)((double)rho / (4.0 * GF_PI * s[0] * s[1] * s[2])), 0.0f, 0.0f);
    // |k_W| = |S R^T omega| for the per-cell medians
    double kk = 0.0;
    for (int k = 0; k < 3; ++k) {
        double rt = 2.0 * GF_PI * (R[0][k] * p[10] + R[1][k] * p[11] + R[2][k] * p[12]);
        kk += (s[k] * rt) * (s[k] * rt);
    }
    kw[j] = (float)sqrt(kk);
}

// ---------------------------------------------------------------------------
// 6. bottom-up refit: the second child to arrive at a node unions both boxes
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_refit(int n, const int32_t* __restrict__ left,
                                               const int32_t* __restrict__ right, const int32_t* __restrict__ parent,
                                               float* aabb, uint64_t* cellor, int* __restrict__ visits) {
    int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    int node = parent[n - 1 + j];
    while (node >= 0) {
        __threadfence();
        if (atomicAdd(&visits[node], 1) == 0) return;
        __threadfence();
        int a = left[node], b = right[node];
        float* bx = aabb + (size_t)node * 6;
        for (int k = 0; k < 3; ++k) {
            float la = __hip_atomic_load(&aabb[(size_t)a * 6 + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            float lb = __hip_atomic_load(&aabb[(size_t)b * 6 + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            float ha = __hip_atomic_load(&aabb[(size_t)a * 6 + 3 + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            float hb = __hip_atomic_load(&aabb[(size_t)b * 6 + 3 + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            bx[k] = fminf(la, lb);
            bx[3 + k] = fmaxf(ha, hb);
        }
        uint64_t ca = __hip_atomic_load(&cellor[a], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint64_t cb = __hip_atomic_load(&cellor[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        cellor[node] = ca | cb;
        node = parent[node];
    }
}

// depth of every leaf (internal nodes on its root path), max-reduced
__global__ __launch_bounds__(256) void k_depth(int n, const int32_t* __restrict__ parent, int* __restrict__ depth) {
    int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    int d = 0;
    for (int node = parent[n - 1 + j]; node >= 0; node = parent[node]) ++d;
    atomicMax(depth, d);
}

// ---------------------------------------------------------------------------
// 7. traversal records
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_tnodes(int n, const int32_t* __restrict__ left,
                                                const int32_t* __restrict__ right, const float* __restrict__ aabb,
                                                const uint64_t* __restrict__ cellor, TNode* __restrict__ nodes) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n - 1) return;
    int a = left[i], b = right[i];
    TNode t;
    for (int k = 0; k < 6; ++k) {
        t.lbox[k] = aabb[(size_t)a * 6 + k];
        t.rbox[k] = aabb[(size_t)b * 6 + k];
    }
    int L0 = n - 1;
    t.lchild = a >= L0 ? ~(a - L0) : a;
    t.rchild = b >= L0 ? ~(b - L0) : b;
    t.cells = (uint32_t)(cellor[a] & 0xffffu) | ((uint32_t)(cellor[b] & 0xffffu) << 16);
    t.pad = 0;
    nodes[i] = t;
}

// Traversal records with every subtree of at most GF_LEAF_MAX primitives
// collapsed into a Morton leaf range (fewer dependent node steps for the
// per-lane traversals; the subtree's box and cell mask stay those of its
// root).
__global__ __launch_bounds__(256) void k_tnodes_collapsed(int n, const int32_t* __restrict__ left,
                                                          const int32_t* __restrict__ right,
                                                          const int2* __restrict__ range,
                                                          const TNode* __restrict__ nodes,
                                                          TNode* __restrict__ cnodes) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n - 1) return;
    const int L0 = n - 1;
    auto enc = [&](int a) -> int {
        if (a >= L0) return ~(a - L0);
        int2 r = range[a];
        int cnt = r.y - r.x + 1;
        if (cnt <= GF_LEAF_MAX) return ~(int)((unsigned)r.x | ((unsigned)(cnt - 1) << 28));
        return a;
    };
    TNode t = nodes[i];
    t.lchild = enc(left[i]);
    t.rchild = enc(right[i]);
    cnodes[i] = t;
}

// ---------------------------------------------------------------------------
// 8. majorant grid: per voxel and cell, sum over primitives whose leaf box
//    meets the voxel of rho |alpha| c exp(-m / 2), with m a lower bound of the
//    Mahalanobis form over the voxel: the larger of |d|^2 / s_max^2 and
//    max_a d_a^2 / Sigma_aa (d = distance from mu to the voxel per axis; the
//    level set {M <= m} lies inside |x_a - mu_a| <= sqrt(m Sigma_aa)).  Sums are
//    exact fixed-point integers (order independent), rounded up.
// ---------------------------------------------------------------------------
#define GRID_FIX 1048576.0  // 2^20

__global__ __launch_bounds__(256) void k_grid_splat(const float* __restrict__ params, int n, float rho, int G,
                                                    float3 glo, float3 gh, const uint32_t* __restrict__ perm,
                                                    const float4* __restrict__ prims,
                                                    const float* __restrict__ aabb,
                                                    unsigned long long* __restrict__ acc) {
    int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    const float* p = params + (size_t)perm[j] * 15;
    int cell = rec_cell(prims[(size_t)j * 4 + 3].w);
    float smax = fmaxf(p[7], fmaxf(p[8], p[9]));
    double c = (double)rho * fabs((double)p[14]) / (pow(2.0 * GF_PI, 1.5) * (double)p[7] * p[8] * p[9]);
    double R[3][3], qh[4];
    rotation64(p, R, qh);
    float isd2[3];
    for (int a = 0; a < 3; ++a) {
        double t0 = R[a][0] * p[7], t1 = R[a][1] * p[8], t2 = R[a][2] * p[9];
        isd2[a] = (float)(1.0 / (t0 * t0 + t1 * t1 + t2 * t2));
    }
    const float* bx = aabb + (size_t)(n - 1 + j) * 6;
    int i0[3], i1[3];
    float lo[3] = {glo.x, glo.y, glo.z}, h[3] = {gh.x, gh.y, gh.z};
    for (int a = 0; a < 3; ++a) {
        i0[a] = max(0, min(G - 1, (int)floorf((bx[a] - lo[a]) / h[a])));
        i1[a] = max(0, min(G - 1, (int)floorf((bx[3 + a] - lo[a]) / h[a])));
    }
    float inv2 = 1.0f / (smax * smax);
    for (int z = i0[2]; z <= i1[2]; ++z) {
        float vz0 = lo[2] + z * h[2], dz = fmaxf(0.0f, fmaxf(vz0 - p[2], p[2] - (vz0 + h[2])));
        for (int y = i0[1]; y <= i1[1]; ++y) {
            float vy0 = lo[1] + y * h[1], dy = fmaxf(0.0f, fmaxf(vy0 - p[1], p[1] - (vy0 + h[1])));
            for (int x = i0[0]; x <= i1[0]; ++x) {
                float vx0 = lo[0] + x * h[0], dx = fmaxf(0.0f, fmaxf(vx0 - p[0], p[0] - (vx0 + h[0])));
                float m1 = (dx * dx + dy * dy + dz * dz) * inv2;
                float m2 = fmaxf(fmaxf(dx * dx * isd2[0], dy * dy * isd2[1]), dz * dz * isd2[2]);
                // shrink slightly so float32 rounding never over-estimates the bound
                float m = fmaxf(m1, m2) * 0.999f;
                double v = c * exp(-0.5 * (double)m);
                unsigned long long q = (unsigned long long)ceil(v * GRID_FIX);
                if (q) atomicAdd(&acc[((size_t)(z * G + y) * G + x) * GF_NCELLS + cell], q);
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_grid_final(const unsigned long long* __restrict__ acc, size_t m,
                                                    float* __restrict__ grid) {
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    unsigned long long q = acc[i];
    grid[i] = q ? __double2float_ru((double)q / GRID_FIX) : 0.0f;
}

// ---------------------------------------------------------------------------
// masks
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_cells_morton(const float4* __restrict__ prims, int n,
                                                      int32_t* __restrict__ out) {
    int j = blockIdx.x * 256 + threadIdx.x;
    if (j < n) out[j] = rec_cell(prims[(size_t)j * 4 + 3].w);
}

__global__ __launch_bounds__(256) void k_cells_export(const float4* __restrict__ prims, int n,
                                                      int32_t* __restrict__ out) {
    int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    float4 r = prims[(size_t)j * 4 + 3];
    out[rec_orig(r.w)] = rec_cell(r.w);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static gf_status scene_free(gf_scene_s* s) {
    if (!s) return GF_OK;
    void* ptrs[] = {s->prims,  s->aux,  s->A64,   s->nodes,  s->cnodes, s->grid, s->keys,
                    s->perm,   s->left, s->right, s->parent, s->aabb,   s->cellor};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    delete s;
    return GF_OK;
}

template <class T>
static gf_status dalloc(T** p, size_t count, size_t* total) {
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc((void**)p, bytes);
    if (e != hipSuccess) return gf_hip_check(e, "hipMalloc");
    *total += bytes;
    return GF_OK;
}

#define GF_TRY(x)                        \
    do {                                 \
        gf_status _s = (x);              \
        if (_s != GF_OK) {               \
            scene_free(s);               \
            return _s;                   \
        }                                \
    } while (0)
#define GF_HTRY(x) GF_TRY(((x) == hipSuccess) ? GF_OK : gf_hip_check(hipGetLastError(), #x))

static unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

extern "C" gf_status gf_scene_create(const float* params, int64_t n, const gf_scene_desc* desc, void* stream,
                                     gf_scene* out) {
    if (!out) return gf_fail(GF_EINVAL, "gf_scene_create: out is NULL");
    *out = nullptr;
    if (!params || !desc) return gf_fail(GF_EINVAL, "gf_scene_create: params/desc is NULL");
    if (n < 1 || n > (int64_t)(1 << 28)) return gf_fail(GF_EINVAL, "gf_scene_create: n=%lld out of range", (long long)n);
    if (!(desc->rho > 0.0f) || !isfinite(desc->rho)) return gf_fail(GF_EINVAL, "gf_scene_create: rho must be > 0");
    float r = desc->trunc_r == 0.0f ? 3.0f : desc->trunc_r;
    if (!(r > 0.0f) || !isfinite(r)) return gf_fail(GF_EINVAL, "gf_scene_create: trunc_r must be > 0");
    if (!(desc->clamp_eps >= 0.0f) || !isfinite(desc->clamp_eps))
        return gf_fail(GF_EINVAL, "gf_scene_create: clamp_eps must be finite and >= 0");
    int G = desc->majorant_grid;
    if (G < 0 || G > 512) return gf_fail(GF_EINVAL, "gf_scene_create: majorant_grid must be in [0, 512]");
    gf_status st = gf_ensure_weideman_tau();
    if (st != GF_OK) return st;
    st = gf_ensure_weideman_grad();
    if (st != GF_OK) return st;
    hipStream_t sm = (hipStream_t)stream;
    int ni = (int)n;

    gf_scene_s* s = new gf_scene_s();
    memset(s, 0, sizeof(*s));
    GF_HTRY(hipGetDevice(&s->device));
    s->n = n;
    s->rho = desc->rho;
    s->r = r;
    s->clamp_eps = desc->clamp_eps;
    s->G = G;
    size_t total = 0;
    GF_TRY(dalloc(&s->prims, (size_t)n * 4, &total));
    GF_TRY(dalloc(&s->aux, (size_t)n * 3, &total));
    GF_TRY(dalloc(&s->A64, (size_t)n * GF_A64, &total));
    GF_TRY(dalloc(&s->nodes, (size_t)std::max<int64_t>(n - 1, 1), &total));
    GF_TRY(dalloc(&s->cnodes, (size_t)std::max<int64_t>(n - 1, 1), &total));
    GF_TRY(dalloc(&s->grid, (size_t)G * G * G * GF_NCELLS, &total));
    GF_TRY(dalloc(&s->keys, (size_t)n, &total));
    GF_TRY(dalloc(&s->perm, (size_t)n, &total));
    GF_TRY(dalloc(&s->left, (size_t)std::max<int64_t>(n - 1, 1), &total));
    GF_TRY(dalloc(&s->right, (size_t)std::max<int64_t>(n - 1, 1), &total));
    GF_TRY(dalloc(&s->parent, (size_t)(2 * n - 1), &total));
    GF_TRY(dalloc(&s->aabb, (size_t)(2 * n - 1) * 6, &total));
    GF_TRY(dalloc(&s->cellor, (size_t)(2 * n - 1), &total));
    s->bytes = total;

    // scratch (freed before return)
    size_t scratch_bytes = 0;
    const int nparts = (int)std::min<int64_t>(1024, nblk(n));
    BoundsPartial* parts = nullptr;
    uint64_t* k2 = nullptr;
    uint32_t *v1 = nullptr, *v2 = nullptr, *hist = nullptr;
    int* visits = nullptr;
    float* kw = nullptr;
    unsigned long long* gacc = nullptr;
    int2* ranges = nullptr;
    const int ntiles = (int)((n + RS_TILE - 1) / RS_TILE);
    auto cleanup = [&]() {
        void* q[] = {parts, k2, v1, v2, hist, visits, kw, gacc, ranges};
        for (void* x : q)
            if (x) (void)hipFree(x);
    };
#define GF_STRY(x)                       \
    do {                                 \
        gf_status _s = (x);              \
        if (_s != GF_OK) {               \
            cleanup();                   \
            scene_free(s);               \
            return _s;                   \
        }                                \
    } while (0)
    GF_STRY(dalloc(&parts, nparts, &scratch_bytes));
    GF_STRY(dalloc(&k2, n, &scratch_bytes));
    GF_STRY(dalloc(&v1, n, &scratch_bytes));
    GF_STRY(dalloc(&v2, n, &scratch_bytes));
    GF_STRY(dalloc(&hist, (size_t)ntiles * RS_DIGITS, &scratch_bytes));
    GF_STRY(dalloc(&visits, std::max<int64_t>(n - 1, 1), &scratch_bytes));
    GF_STRY(dalloc(&kw, n, &scratch_bytes));
    if (G > 0) GF_STRY(dalloc(&gacc, (size_t)G * G * G * GF_NCELLS, &scratch_bytes));
    GF_STRY(dalloc(&ranges, std::max<int64_t>(n - 1, 1), &scratch_bytes));

    // 1. validation, bounds, |f| max
    k_bounds_partial<<<nparts, 256, 0, sm>>>(params, ni, parts);
    k_bounds_final<<<1, 256, 0, sm>>>(parts, nparts);
    BoundsPartial hb;
    GF_STRY(hipMemcpyAsync(&hb, parts, sizeof(hb), hipMemcpyDeviceToHost, sm) == hipSuccess
                ? GF_OK : gf_hip_check(hipGetLastError(), "bounds copy"));
    GF_STRY(hipStreamSynchronize(sm) == hipSuccess ? GF_OK : gf_hip_check(hipGetLastError(), "sync"));
    if (hb.bad) {
        cleanup();
        scene_free(s);
        return gf_fail(GF_EINVAL, "gf_scene_create: a record has NaN/Inf, a scale <= 0 or a zero quaternion");
    }
    s->fmax2 = hb.f2max;
    for (int a = 0; a < 3; ++a) {
        s->lo[a] = hb.lo[a];
        s->hi[a] = hb.hi[a];
    }
    // 2-3. keys and stable sort
    k_morton<<<nblk(n), 256, 0, sm>>>(params, ni, parts, s->keys, v1);
    uint64_t *ka = s->keys, *kb = k2;
    uint32_t *va = v1, *vb = v2;
    for (int shift = 0; shift < 64; shift += 4) {
        k_rs_hist<<<ntiles, RS_THREADS, 0, sm>>>(ka, ni, shift, hist, ntiles);
        k_scan_excl<<<1, 1024, 0, sm>>>(hist, ntiles * RS_DIGITS);
        k_rs_scatter<<<ntiles, RS_THREADS, 0, sm>>>(ka, va, kb, vb, ni, shift, hist, ntiles);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    // 16 passes: result back in s->keys / v1
    GF_STRY(hipMemcpyAsync(s->perm, va, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, sm) == hipSuccess
                ? GF_OK : gf_hip_check(hipGetLastError(), "perm copy"));
    // 4. hierarchy
    GF_STRY(hipMemsetAsync(s->parent, 0xff, sizeof(int32_t) * (2 * n - 1), sm) == hipSuccess
                ? GF_OK : gf_hip_check(hipGetLastError(), "memset"));
    if (n > 1) k_karras<<<nblk(n - 1), 256, 0, sm>>>(s->keys, ni, s->left, s->right, s->parent, ranges);
    // 5. records and leaves
    k_leaves<<<nblk(n), 256, 0, sm>>>(params, ni, r, s->rho, s->clamp_eps, parts, (const uint32_t*)s->perm, s->prims, s->aabb,
                                      s->cellor, kw, s->aux, s->A64);
    // 6-7. refit and traversal records
    if (n > 1) {
        GF_STRY(hipMemsetAsync(visits, 0, sizeof(int) * (n - 1), sm) == hipSuccess
                    ? GF_OK : gf_hip_check(hipGetLastError(), "memset"));
        k_refit<<<nblk(n), 256, 0, sm>>>(ni, s->left, s->right, s->parent, s->aabb, s->cellor, visits);
        k_tnodes<<<nblk(n - 1), 256, 0, sm>>>(ni, s->left, s->right, s->aabb, s->cellor, s->nodes);
        k_tnodes_collapsed<<<nblk(n - 1), 256, 0, sm>>>(ni, s->left, s->right, ranges, s->nodes, s->cnodes);
        GF_STRY(hipMemsetAsync(visits, 0, sizeof(int), sm) == hipSuccess
                    ? GF_OK : gf_hip_check(hipGetLastError(), "memset"));
        k_depth<<<nblk(n), 256, 0, sm>>>(ni, s->parent, visits);
    }
    GF_STRY(hipGetLastError() == hipSuccess ? GF_OK : gf_hip_check(hipGetLastError(), "build kernels"));
    // root box, per-cell statistics
    float root[6];
    int hdepth = 0;
    if (n > 1)
        GF_STRY(hipMemcpyAsync(&hdepth, visits, sizeof(int), hipMemcpyDeviceToHost, sm) == hipSuccess
                    ? GF_OK : gf_hip_check(hipGetLastError(), "depth copy"));
    std::vector<float> hkw(n);
    std::vector<int32_t> hcell(n);
    GF_STRY(hipMemcpyAsync(root, s->aabb, sizeof(root), hipMemcpyDeviceToHost, sm) == hipSuccess
                ? GF_OK : gf_hip_check(hipGetLastError(), "root copy"));
    GF_STRY(hipMemcpyAsync(hkw.data(), kw, sizeof(float) * n, hipMemcpyDeviceToHost, sm) == hipSuccess
                ? GF_OK : gf_hip_check(hipGetLastError(), "kw copy"));
    k_cells_morton<<<nblk(n), 256, 0, sm>>>(s->prims, ni, (int32_t*)v2);
    GF_STRY(hipMemcpyAsync(hcell.data(), v2, sizeof(int32_t) * n, hipMemcpyDeviceToHost, sm) == hipSuccess
                ? GF_OK : gf_hip_check(hipGetLastError(), "cell copy"));
    GF_STRY(hipStreamSynchronize(sm) == hipSuccess ? GF_OK : gf_hip_check(hipGetLastError(), "sync"));
    s->depth = hdepth;
    {
        std::vector<std::vector<float>> per(GF_NCELLS);
        for (int64_t j = 0; j < n; ++j) {
            int c = hcell[j];
            per[c].push_back(hkw[j]);
        }
        s->nonempty = 0;
        for (int c = 0; c < GF_NCELLS; ++c) {
            s->cell_count[c] = (int64_t)per[c].size();
            if (per[c].empty()) {
                s->med[c] = 0.0f;
                continue;
            }
            s->nonempty |= 1ull << c;
            size_t m = (per[c].size() - 1) / 2;
            std::nth_element(per[c].begin(), per[c].begin() + m, per[c].end());
            s->med[c] = per[c][m];
        }
    }
    // 8. scene box; majorant grid over it (optional)
    for (int a = 0; a < 3; ++a) {
        s->lo[a] = root[a];
        s->hi[a] = root[3 + a];
        if (!(s->hi[a] > s->lo[a])) s->hi[a] = s->lo[a] + 1e-6f;
    }
    if (G == 0) {
        GF_STRY(hipStreamSynchronize(sm) == hipSuccess ? GF_OK : gf_hip_check(hipGetLastError(), "sync"));
        cleanup();
        *out = s;
        return GF_OK;
    }
    float3 glo = make_float3(s->lo[0], s->lo[1], s->lo[2]);
    float3 gh = make_float3((s->hi[0] - s->lo[0]) / G, (s->hi[1] - s->lo[1]) / G, (s->hi[2] - s->lo[2]) / G);
    size_t gm = (size_t)G * G * G * GF_NCELLS;
    GF_STRY(hipMemsetAsync(gacc, 0, gm * sizeof(unsigned long long), sm) == hipSuccess
                ? GF_OK : gf_hip_check(hipGetLastError(), "memset"));
    k_grid_splat<<<nblk(n), 256, 0, sm>>>(params, ni, s->rho, G, glo, gh, (const uint32_t*)s->perm, s->prims,
                                          s->aabb, gacc);
    k_grid_final<<<nblk((int64_t)gm), 256, 0, sm>>>(gacc, gm, s->grid);
    GF_STRY(hipStreamSynchronize(sm) == hipSuccess ? GF_OK : gf_hip_check(hipGetLastError(), "sync"));
    GF_STRY(hipGetLastError() == hipSuccess ? GF_OK : gf_hip_check(hipGetLastError(), "grid kernels"));
    cleanup();
    *out = s;
    return GF_OK;
}

extern "C" gf_status gf_scene_destroy(gf_scene scene) {
    if (!scene) return gf_fail(GF_EINVAL, "gf_scene_destroy: NULL scene");
    return scene_free(scene);
}

extern "C" gf_status gf_scene_info(gf_scene s, gf_scene_info_t* info) {
    if (!s || !info) return gf_fail(GF_EINVAL, "gf_scene_info: NULL argument");
    memset(info, 0, sizeof(*info));
    info->n = s->n;
    info->rho = s->rho;
    info->trunc_r = s->r;
    info->clamp_eps = s->clamp_eps;
    info->fmax = sqrt(s->fmax2);
    info->nonempty_cells = s->nonempty;
    for (int c = 0; c < GF_NCELLS; ++c) {
        info->cell_count[c] = s->cell_count[c];
        info->cell_median_kw[c] = s->med[c];
    }
    info->grid_res = s->G;
    for (int a = 0; a < 3; ++a) {
        info->bounds_lo[a] = s->lo[a];
        info->bounds_hi[a] = s->hi[a];
    }
    info->device_bytes = s->bytes;
    return GF_OK;
}

extern "C" gf_status gf_scene_export_lbvh(gf_scene s, uint64_t* keys, int32_t* perm, int32_t* left, int32_t* right,
                                          int32_t* parent, float* aabb, uint64_t* cellor, void* stream) {
    if (!s) return gf_fail(GF_EINVAL, "gf_scene_export_lbvh: NULL scene");
    hipStream_t sm = (hipStream_t)stream;
    size_t n = (size_t)s->n;
    if (keys) GF_HIP(hipMemcpyAsync(keys, s->keys, n * 8, hipMemcpyDeviceToDevice, sm));
    if (perm) GF_HIP(hipMemcpyAsync(perm, s->perm, n * 4, hipMemcpyDeviceToDevice, sm));
    if (left && n > 1) GF_HIP(hipMemcpyAsync(left, s->left, (n - 1) * 4, hipMemcpyDeviceToDevice, sm));
    if (right && n > 1) GF_HIP(hipMemcpyAsync(right, s->right, (n - 1) * 4, hipMemcpyDeviceToDevice, sm));
    if (parent) GF_HIP(hipMemcpyAsync(parent, s->parent, (2 * n - 1) * 4, hipMemcpyDeviceToDevice, sm));
    if (aabb) GF_HIP(hipMemcpyAsync(aabb, s->aabb, (2 * n - 1) * 24, hipMemcpyDeviceToDevice, sm));
    if (cellor) GF_HIP(hipMemcpyAsync(cellor, s->cellor, (2 * n - 1) * 8, hipMemcpyDeviceToDevice, sm));
    return GF_OK;
}

extern "C" gf_status gf_scene_cells(gf_scene s, int32_t* cells, void* stream) {
    if (!s || !cells) return gf_fail(GF_EINVAL, "gf_scene_cells: NULL argument");
    k_cells_export<<<nblk(s->n), 256, 0, (hipStream_t)stream>>>(s->prims, (int)s->n, cells);
    GF_HIP(hipGetLastError());
    return GF_OK;
}

extern "C" uint64_t gf_mask_lod_cells(int lod) {
    if (lod < 0) lod = 0;
    if (lod > 3) lod = 3;
    uint64_t m = 0;
    for (int l = 0; l < 4 - lod; ++l) m |= 7ull << (3 * l);
    return m;
}

// Cone test on the float32 frequency kept in every Morton-ordered record;
// the bit of the primitive's caller index is set.
__global__ __launch_bounds__(256) void k_cone_rec(const float4* __restrict__ prims, int n, double ax, double ay,
                                                  double az, double c2, uint32_t* __restrict__ bits) {
    int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    float4 r2 = prims[(size_t)j * 4 + 2], r3 = prims[(size_t)j * 4 + 3];
    double fx = r2.z, fy = r2.w, fz = r3.x;
    double fa = fx * ax + fy * ay + fz * az;
    double f2;
    {
#pragma clang fp contract(off)
        f2 = (fx * fx + fy * fy) + fz * fz;
    }
    int orig = rec_orig(r3.w);
    if (fa * fa <= c2 * f2) atomicOr(&bits[orig >> 5], 1u << (orig & 31));
}

extern "C" gf_status gf_mask_cone(gf_scene s, const float axis[3], float half_angle, uint32_t* prim_bits,
                                  void* stream) {
    if (!s || !axis || !prim_bits) return gf_fail(GF_EINVAL, "gf_mask_cone: NULL argument");
    double an = sqrt((double)axis[0] * axis[0] + (double)axis[1] * axis[1] + (double)axis[2] * axis[2]);
    if (!(an > 0.0) || !isfinite(an) || !isfinite(half_angle))
        return gf_fail(GF_EINVAL, "gf_mask_cone: invalid axis or angle");
    hipStream_t sm = (hipStream_t)stream;
    gf_status st = gf_zero_words(prim_bits, (size_t)((s->n + 31) / 32), sm);
    if (st != GF_OK) return st;
    double c = cos((double)half_angle);
    k_cone_rec<<<nblk(s->n), 256, 0, sm>>>(s->prims, (int)s->n, axis[0] / an, axis[1] / an, axis[2] / an, c * c,
                                           prim_bits);
    GF_HIP(hipGetLastError());
    return GF_OK;
}

SceneView gf_scene_view(const gf_scene_s* s) {
    SceneView v;
    v.prims = s->prims;
    v.nodes = s->nodes;
    v.cnodes = s->cnodes;
    v.croot = s->n <= GF_LEAF_MAX ? ~(int)((unsigned)(s->n - 1) << 28) : 0;
    v.grid = s->grid;
    v.aux = s->aux;
    v.A64 = s->A64;
    v.n = (int)s->n;
    v.r = s->r;
    v.r2 = s->r * s->r;
    v.G = s->G;
    for (int a = 0; a < 3; ++a) {
        v.glo[a] = s->lo[a];
        v.ghi[a] = s->hi[a];
        v.ginv[a] = (float)s->G / (s->hi[a] - s->lo[a]);
    }
    for (int c = 0; c < GF_NCELLS; ++c) v.med[c] = s->med[c];
    return v;
}

__global__ __launch_bounds__(256) void k_zero_words(uint32_t* __restrict__ p, size_t words) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (size_t)gridDim.x * 256) p[i] = 0u;
}

gf_status gf_zero_words(void* p, size_t words, hipStream_t sm) {
    if (words == 0) return GF_OK;
    size_t blocks = (words + 255) / 256;
    k_zero_words<<<(unsigned)(blocks < 4096 ? blocks : 4096), 256, 0, sm>>>((uint32_t*)p, words);
    GF_HIP(hipGetLastError());
    return GF_OK;
}

gf_status gf_check_mask(const gf_mask& m, const char* who) {
    if (!(m.lod_k >= 0.0f) || !isfinite(m.lod_k)) return gf_fail(GF_EINVAL, "%s: mask lod_k must be finite and >= 0", who);
    return GF_OK;
}

MaskView gf_mask_view(const gf_mask& m) {
    MaskView v;
    v.cells = (uint32_t)(m.cells & 0xfffu);
    v.prim_bits = m.prim_bits;
    v.lod_k = m.lod_k > 0.0f ? m.lod_k : 0.0f;
    v.lod2 = v.lod_k * v.lod_k;
    return v;
}
