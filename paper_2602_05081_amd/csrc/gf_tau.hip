// Deterministic optical depth and transmittance (Sec. 3, Eqs. 2-3; Sec. 4.4).
//
// Packet traversal: one wave64 carries 64 rays (an 8x8 pixel tile when the
// rays form an image) through the LBVH together.  The node index, the
// stack (in LDS) and the primitive index at a leaf are wave-uniform, so node
// and primitive records come in through the scalar cache once per wave and
// are shared by all 64 rays; each lane tests its own ray against both child
// boxes and the wave descends where any lane hits (ballot).  A subtree whose
// cell mask misses the query mask is skipped before its boxes are tested
// (visibility masks of Sec. 4.6, implementation details).  Per-ray sums are
// binary64; the summation order is the depth-first leaf order, independent of
// which other rays share the wave.
#include <math.h>
#include <string.h>

#include <atomic>

#include "gf_hit.hpp"

__constant__ float c_weid[WEID_N];
__constant__ float c_weidL;
__constant__ double c_weid64[WEID64_N];
__constant__ double c_weidL64;

// Weideman's coefficients: f(t) = exp(-t^2)(L^2 + t^2) sampled at
// t = L tan(theta/2), theta = k pi / M, then the real part of the DFT of the
// (fftshift-ed) samples; a[p] holds the coefficient of Z^(N-1-p).
static void weideman(int N, double* a, double* Lout) {
    const int M = 2 * N, M2 = 2 * M;
    const double Ld = sqrt(N / sqrt(2.0));
    double f[256];
    f[0] = 0.0;
    for (int k = -M + 1; k <= M - 1; ++k) {
        double th = k * GF_PI / M;
        double t = Ld * tan(0.5 * th);
        f[k + M] = exp(-t * t) * (Ld * Ld + t * t);
    }
    double y[256];
    for (int i = 0; i < M2; ++i) y[i] = f[(i + M2 / 2) % M2];
    double A[256];
    for (int m = 0; m < M2; ++m) {
        double re = 0.0;
        for (int j = 0; j < M2; ++j) re += y[j] * cos(2.0 * GF_PI * (double)(((long)j * m) % M2) / M2);
        A[m] = re / M2;
    }
    for (int p = 0; p < N; ++p) a[p] = A[N - p];
    *Lout = Ld;
}

void gf_weideman_coeffs(float* a, float* L) {
    double ad[WEID_N], Ld;
    weideman(WEID_N, ad, &Ld);
    for (int p = 0; p < WEID_N; ++p) a[p] = (float)ad[p];
    *L = (float)Ld;
}

void gf_weideman_coeffs64(double* a, double* L) { weideman(WEID64_N, a, L); }

static bool g_weid_ready[64];

gf_status gf_ensure_weideman_tau() {
    int dev = 0;
    GF_HIP(hipGetDevice(&dev));
    if (dev >= 0 && dev < 64 && g_weid_ready[dev]) return GF_OK;
    float a[WEID_N], L;
    gf_weideman_coeffs(a, &L);
    GF_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_weid), a, sizeof(a)));
    GF_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_weidL), &L, sizeof(L)));
    double a64[WEID64_N], L64;
    gf_weideman_coeffs64(a64, &L64);
    GF_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_weid64), a64, sizeof(a64)));
    GF_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_weidL64), &L64, sizeof(L64)));
    if (dev >= 0 && dev < 64) g_weid_ready[dev] = true;
    return GF_OK;
}

template <bool COUNT>
__global__ __launch_bounds__(256) void k_tau(SceneView S, MaskView M, const float* __restrict__ rays, int n,
                                             int tile_w, float* __restrict__ tau, float* __restrict__ T,
                                             int* __restrict__ cnodes, int* __restrict__ chits) {
    __shared__ int stk[PK_WAVES][GF_STACK];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int idx = packet_ray(blockIdx.x * PK_WAVES + w, lane, n, tile_w);
    const bool valid = idx >= 0;
    RayD R = valid ? load_ray(rays, idx) : RayD{0, 0, 0, 0, 0, 1, 1.0f, 0.0f};
    double acc = 0.0;
    int nn = 0, nh = 0;
    packet_traverse(S, M, valid, R, stk[w], nn, [&](int j, bool active) {
        PrimF P = load_prim(S.prims, j);
        if (M.prim_bits && !((M.prim_bits[P.orig >> 5] >> (P.orig & 31)) & 1u)) return;
        if (!active) return;
        HitGeom H;
        if (!hit_geom(P, R, S.A64 + (size_t)j * GF_A64, H)) return;
        if (!lod_keep64(P, R, H, M.lod_k)) return;
        if (COUNT) ++nh;
        else acc += (double)hit_value(P, H, c_weid, c_weidL, c_weid64, c_weidL64);
    });
    if (valid) {
        if (COUNT) {
            if (cnodes) cnodes[idx] = nn;
            if (chits) chits[idx] = nh;
        } else {
            tau[idx] = (float)acc;
            if (T) T[idx] = (float)exp(-acc);
        }
    }
}

unsigned gf_packet_blocks(int64_t n, int tile_w) {
    int64_t waves;
    if (tile_w <= 0) waves = (n + 63) / 64;
    else waves = (int64_t)(tile_w / 8) * ((n / tile_w + 7) / 8);
    return (unsigned)((waves + PK_WAVES - 1) / PK_WAVES);
}

gf_status gf_check_rays(int64_t n, int tile_w, const char* who) {
    if (n < 0 || n > (int64_t)INT32_MAX / 8) return gf_fail(GF_EINVAL, "%s: ray count out of range", who);
    if (tile_w < 0) return gf_fail(GF_EINVAL, "%s: image_width < 0", who);
    if (tile_w > 0 && (tile_w % 8 != 0 || n % tile_w != 0))
        return gf_fail(GF_EINVAL, "%s: image_width must be a multiple of 8 dividing n", who);
    return GF_OK;
}

// ---------------------------------------------------------------------------
// Validation of caller rays.  One slot of g_bad_ray per call (taken round
// robin, so concurrent calls on different streams do not share one)
// receives the smallest index of an invalid ray; the host waits for it.
// ---------------------------------------------------------------------------
#define RAY_CHECK_SLOTS 64
static __device__ unsigned g_bad_ray[RAY_CHECK_SLOTS];

__global__ __launch_bounds__(256) void k_check_rays(const float* __restrict__ rays, int n, unsigned* __restrict__ bad) {
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float* r = rays + (size_t)i * 8;
    bool ok = true;
    for (int a = 0; a < 7; ++a) ok = ok && isfinite(r[a]);
    ok = ok && !isnan(r[7]) && r[6] <= r[7];
    ok = ok && (r[3] != 0.0f || r[4] != 0.0f || r[5] != 0.0f);
    if (!ok) atomicMin(bad, (unsigned)i);
}

__global__ void k_set_word(unsigned* p, unsigned v) { *p = v; }

gf_status gf_validate_rays(const float* rays, int64_t n, hipStream_t sm, const char* who) {
    static std::atomic<unsigned> next_slot{0};
    if (n <= 0) return GF_OK;
    unsigned* slots = nullptr;
    GF_HIP(hipGetSymbolAddress((void**)&slots, HIP_SYMBOL(g_bad_ray)));
    unsigned* bad = slots + (next_slot.fetch_add(1) % RAY_CHECK_SLOTS);
    k_set_word<<<1, 1, 0, sm>>>(bad, 0xFFFFFFFFu);
    k_check_rays<<<(unsigned)((n + 255) / 256), 256, 0, sm>>>(rays, (int)n, bad);
    GF_HIP(hipGetLastError());
    unsigned first = 0;
    GF_HIP(hipMemcpyAsync(&first, bad, sizeof(first), hipMemcpyDeviceToHost, sm));
    GF_HIP(hipStreamSynchronize(sm));
    if (first != 0xFFFFFFFFu)
        return gf_fail(GF_EINVAL, "%s: ray %u is invalid (NaN/Inf, |v| = 0 or tmin > tmax)", who, first);
    return GF_OK;
}

extern "C" gf_status gf_optical_depth(gf_scene s, const float* rays, int64_t n, int image_width, gf_mask mask,
                                      float* tau, float* T, void* stream) {
    if (!s || (!rays && n) || (!tau && n)) return gf_fail(GF_EINVAL, "gf_optical_depth: NULL argument");
    gf_status st = gf_check_rays(n, image_width, "gf_optical_depth");
    if (st == GF_OK) st = gf_check_mask(mask, "gf_optical_depth");
    if (st == GF_OK && n > 0) st = gf_validate_rays(rays, n, (hipStream_t)stream, "gf_optical_depth");
    if (st != GF_OK) return st;
    if (n == 0) return GF_OK;
    unsigned nb = gf_packet_blocks(n, image_width);
    k_tau<false><<<nb, 256, 0, (hipStream_t)stream>>>(gf_scene_view(s), gf_mask_view(mask), rays, (int)n,
                                                       image_width, tau, T, nullptr, nullptr);
    GF_HIP(hipGetLastError());
    return GF_OK;
}

extern "C" gf_status gf_optical_depth_counts(gf_scene s, const float* rays, int64_t n, int image_width,
                                             gf_mask mask, int32_t* nodes, int32_t* hits, void* stream) {
    if (!s || (!rays && n)) return gf_fail(GF_EINVAL, "gf_optical_depth_counts: NULL argument");
    gf_status st = gf_check_rays(n, image_width, "gf_optical_depth_counts");
    if (st == GF_OK) st = gf_check_mask(mask, "gf_optical_depth_counts");
    if (st == GF_OK && n > 0) st = gf_validate_rays(rays, n, (hipStream_t)stream, "gf_optical_depth_counts");
    if (st != GF_OK) return st;
    if (n == 0) return GF_OK;
    unsigned nb = gf_packet_blocks(n, image_width);
    k_tau<true><<<nb, 256, 0, (hipStream_t)stream>>>(gf_scene_view(s), gf_mask_view(mask), rays, (int)n, image_width,
                                                      nullptr, nullptr, nodes, hits);
    GF_HIP(hipGetLastError());
    return GF_OK;
}
