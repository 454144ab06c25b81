// Adjoint of the optical depth with respect to all 15 primitive parameters.
//
// Segment recomputation: the backward pass re-traverses the LBVH with the same
// wave packets as the forward pass and recomputes every hit; nothing from the
// forward pass is stored.  For one hit, with y(t) = x(t) - mu, A = Sigma^-1,
// G = rho alpha c exp(-M/2) cos psi, the complex moments
//   z_k = rho c/n exp(-h^2/2) e^{i theta} J_k,  J_k = int u^k exp(-u^2/2 + i Omega u) du
// give (tau_i = alpha Re z_0):
//   d/dalpha = Re z0,  d/dphi = -alpha Im z0,  d/domega = -alpha Im Z1,
//   d/dmu = alpha (A Re Z1 + omega Im z0),  d/dA = -alpha Re Z2 / 2,
//   d/ds_k (normalisation) = -tau_i / s_k,
// with Z1 = z0 y_c + z1 v / n and Z2 = z0 y_c y_c^T + z1 (y_c v^T + v y_c^T)/n
// + z2 v v^T / n^2; plus Leibniz terms where a segment end is a chord end
// (M = r^2): dt_e/dtheta = -(dM/dtheta)/(dM/dt).  J1, J2 follow from J0 by
// integration by parts (J1 = -[e] + i Omega J0, J2 = -[u e] + J0 + i Omega J1)
// or, on short segments, by Gauss-Legendre.  A -> (s, R(qhat)) -> q by the
// chain rule.  Each wave sums its lanes' contributions to the (wave-uniform)
// primitive before one float32 atomic add per parameter.
#include <math.h>

#include "gf_hit.hpp"

__constant__ float c_weid_g[WEID_N];
__constant__ float c_weidL_g;

static bool g_ready[64];

gf_status gf_ensure_weideman_grad() {
    int dev = 0;
    GF_HIP(hipGetDevice(&dev));
    if (dev >= 0 && dev < 64 && g_ready[dev]) return GF_OK;
    float a[WEID_N], L;
    gf_weideman_coeffs(a, &L);
    GF_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_weid_g), a, sizeof(a)));
    GF_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_weidL_g), &L, sizeof(L)));
    if (dev >= 0 && dev < 64) g_ready[dev] = true;
    return GF_OK;
}

struct Cf {
    float r, i;
};
static __device__ __forceinline__ Cf cmul(Cf a, Cf b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
static __device__ __forceinline__ Cf cadd(Cf a, Cf b) { return {a.r + b.r, a.i + b.i}; }
static __device__ __forceinline__ Cf csub(Cf a, Cf b) { return {a.r - b.r, a.i - b.i}; }
static __device__ __forceinline__ Cf cscale(Cf a, float s) { return {a.r * s, a.i * s}; }
static __device__ __forceinline__ Cf cexpi_cycles(double c) {
    float s, co;
    sincos_cycles(c, &s, &co);
    return {co, s};
}

// e^{i theta} E(u) (complex), E(u) = exp(-Omega^2/2) erf((u - i Omega)/sqrt 2)
static __device__ __forceinline__ Cf theta_E(float u, float Om, float eO, Cf eth, double thc, double omc) {
    const float is2 = 0.70710678118654752440f;
    float sg = u < 0.0f ? -1.0f : 1.0f;
    float2 w = wofz_weideman(sg * Om * is2, fabsf(u) * is2, c_weid_g, c_weidL_g);
    Cf ep = cexpi_cycles(thc + (double)u * omc);
    Cf t = cmul(ep, Cf{w.x, w.y});
    float eu = __expf(-0.5f * u * u);
    return cscale(csub(cscale(eth, eO), cscale(t, eu)), sg);
}

// moments e^{i theta} J_k, k = 0, 1, 2 over [ua, ub]
static __device__ __forceinline__ void moments(const HitGeom& H, float Om, Cf* m0, Cf* m1, Cf* m2) {
    float len = H.ub - H.ua;
    if (len < 1e-4f) {
        float um = 0.5f * (H.ua + H.ub);
        Cf e = cscale(cexpi_cycles(H.thc + (double)um * H.omc), len * __expf(-0.5f * um * um));
        *m0 = e;
        *m1 = cscale(e, um);
        *m2 = cscale(e, um * um);
        return;
    }
    float q = len * (1.0f + fabsf(Om) + fmaxf(fabsf(H.ua), fabsf(H.ub)));
    if (q < 4.0f) {
        const float xg[4] = {0.18343464249564980f, 0.52553240991632899f, 0.79666647741362674f, 0.96028985649753623f};
        const float wg[4] = {0.36268378337836198f, 0.31370664587788729f, 0.22238103445337447f, 0.10122853629037626f};
        float c = 0.5f * (H.ua + H.ub), h = 0.5f * len;
        Cf a0 = {0, 0}, a1 = {0, 0}, a2 = {0, 0};
        for (int k = 0; k < 4; ++k) {
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                float u = c + sgn * h * xg[k];
                Cf e = cscale(cexpi_cycles(H.thc + (double)u * H.omc), wg[k] * h * __expf(-0.5f * u * u));
                a0 = cadd(a0, e);
                a1 = cadd(a1, cscale(e, u));
                a2 = cadd(a2, cscale(e, u * u));
            }
        }
        *m0 = a0;
        *m1 = a1;
        *m2 = a2;
        return;
    }
    const float sqpi2 = 1.25331413731550025121f;  // sqrt(pi/2)
    float eO = __expf(-0.5f * Om * Om);
    Cf eth = cexpi_cycles(H.thc);
    Cf Pb = theta_E(H.ub, Om, eO, eth, H.thc, H.omc);
    Cf Pa = theta_E(H.ua, Om, eO, eth, H.thc, H.omc);
    Cf J0 = cscale(csub(Pb, Pa), sqpi2);
    Cf Qb = cscale(cexpi_cycles(H.thc + (double)H.ub * H.omc), __expf(-0.5f * H.ub * H.ub));
    Cf Qa = cscale(cexpi_cycles(H.thc + (double)H.ua * H.omc), __expf(-0.5f * H.ua * H.ua));
    Cf iO = {0.0f, Om};
    Cf J1 = cadd(cscale(csub(Qb, Qa), -1.0f), cmul(iO, J0));
    Cf J2 = cadd(cadd(cscale(csub(cscale(Qb, H.ub), cscale(Qa, H.ua)), -1.0f), J0), cmul(iO, J1));
    *m0 = J0;
    *m1 = J1;
    *m2 = J2;
}

// 15 gradient components of tau_i for one hit, scaled by gr
static __device__ void hit_grad(const PrimF& P, const float4* __restrict__ auxp, const HitGeom& H, const RayD& R,
                                float r2, float gr, float* out) {
    float4 x0 = auxp[0], x1 = auxp[1], x2 = auxp[2];
    float qn = x1.x, s[3] = {x1.y, x1.z, x1.w};
    float qw = x0.x / qn, qx = x0.y / qn, qy = x0.z / qn, qz = x0.w / qn;
    float alpha = x2.x, amp1 = x2.y;
    const float sq2pi = 0.79788456080286535588f;
    float n = (float)H.n, inv_n = (float)H.inv_n;
    float Om = (float)(2.0 * GF_PI * H.omc);
    float K = amp1 * sq2pi * inv_n * __expf(-0.5f * H.h2);  // rho c / n exp(-h^2/2)
    Cf m0, m1, m2;
    moments(H, Om, &m0, &m1, &m2);
    Cf z0 = cscale(m0, K), z1 = cscale(m1, K * inv_n), z2 = cscale(m2, K * inv_n * inv_n);
    float yc[3] = {(float)H.ycx, (float)H.ycy, (float)H.ycz};
    float v[3] = {(float)R.vx, (float)R.vy, (float)R.vz};
    float A[3][3] = {{P.a00, P.a01, P.a02}, {P.a01, P.a11, P.a12}, {P.a02, P.a12, P.a22}};
    float om[3] = {2.0f * (float)GF_PI * P.fx, 2.0f * (float)GF_PI * P.fy, 2.0f * (float)GF_PI * P.fz};
    float Z1r[3], Z1i[3];
    for (int a = 0; a < 3; ++a) {
        Z1r[a] = z0.r * yc[a] + z1.r * v[a];
        Z1i[a] = z0.i * yc[a] + z1.i * v[a];
    }
    float tau = alpha * z0.r;
    float gmu[3], gA[3][3];
    for (int a = 0; a < 3; ++a) {
        gmu[a] = alpha * (A[a][0] * Z1r[0] + A[a][1] * Z1r[1] + A[a][2] * Z1r[2] + om[a] * z0.i);
        for (int b = 0; b < 3; ++b)
            gA[a][b] = -0.5f * alpha *
                       (z0.r * yc[a] * yc[b] + z1.r * (yc[a] * v[b] + v[a] * yc[b]) + z2.r * v[a] * v[b]);
    }
    // Leibniz terms at chord ends
    float rr = sqrtf(r2);
    for (int side = 0; side < 2; ++side) {
        bool isend = side ? H.endb : H.enda;
        if (!isend || H.half < 1e-6f) continue;
        float sgn = side ? 1.0f : -1.0f;
        float ue = side ? H.half : -H.half;
        Cf ep = cexpi_cycles(H.thc + (double)ue * H.omc);
        float Ge = alpha * amp1 * sq2pi * __expf(-0.5f * rr * rr) * ep.r;
        float ye[3] = {yc[0] + ue * inv_n * v[0], yc[1] + ue * inv_n * v[1], yc[2] + ue * inv_n * v[2]};
        float De = ue * n;
        float cfac = sgn * Ge / De;
        for (int a = 0; a < 3; ++a) {
            gmu[a] += cfac * (A[a][0] * ye[0] + A[a][1] * ye[1] + A[a][2] * ye[2]);
            for (int b = 0; b < 3; ++b) gA[a][b] -= 0.5f * cfac * ye[a] * ye[b];
        }
    }
    // R(qhat), then A = sum_k r_k r_k^T / s_k^2 -> s, R
    float Rm[3][3] = {{1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
                      {2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)},
                      {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
    float gs[3], gR[3][3];
    for (int k = 0; k < 3; ++k) {
        float Ar[3];
        for (int a = 0; a < 3; ++a) Ar[a] = gA[a][0] * Rm[0][k] + gA[a][1] * Rm[1][k] + gA[a][2] * Rm[2][k];
        float rAr = Rm[0][k] * Ar[0] + Rm[1][k] * Ar[1] + Rm[2][k] * Ar[2];
        float is2 = 1.0f / (s[k] * s[k]);
        gs[k] = -2.0f * rAr * is2 / s[k] - tau / s[k];
        for (int a = 0; a < 3; ++a) gR[a][k] = 2.0f * Ar[a] * is2;
    }
    // dR/dqhat contracted with gR
    float gw = 2.0f * (-qz * gR[0][1] + qy * gR[0][2] + qz * gR[1][0] - qx * gR[1][2] - qy * gR[2][0] +
                       qx * gR[2][1]);
    float gx = 2.0f * (qy * gR[0][1] + qz * gR[0][2] + qy * gR[1][0] - 2.0f * qx * gR[1][1] - qw * gR[1][2] +
                       qz * gR[2][0] + qw * gR[2][1] - 2.0f * qx * gR[2][2]);
    float gy = 2.0f * (-2.0f * qy * gR[0][0] + qx * gR[0][1] + qw * gR[0][2] + qx * gR[1][0] + qz * gR[1][2] -
                       qw * gR[2][0] + qz * gR[2][1] - 2.0f * qy * gR[2][2]);
    float gz = 2.0f * (-2.0f * qz * gR[0][0] - qw * gR[0][1] + qx * gR[0][2] + qw * gR[1][0] -
                       2.0f * qz * gR[1][1] + qy * gR[1][2] + qx * gR[2][0] + qy * gR[2][1]);
    float dot = gw * qw + gx * qx + gy * qy + gz * qz;
    float iq = 1.0f / qn;
    out[0] += gr * gmu[0];
    out[1] += gr * gmu[1];
    out[2] += gr * gmu[2];
    out[3] += gr * (gw - qw * dot) * iq;
    out[4] += gr * (gx - qx * dot) * iq;
    out[5] += gr * (gy - qy * dot) * iq;
    out[6] += gr * (gz - qz * dot) * iq;
    out[7] += gr * gs[0];
    out[8] += gr * gs[1];
    out[9] += gr * gs[2];
    for (int a = 0; a < 3; ++a) out[10 + a] += gr * (-2.0f * (float)GF_PI * alpha * Z1i[a]);
    out[13] += gr * (-alpha * z0.i);
    out[14] += gr * z0.r;
}

static __device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__global__ __launch_bounds__(256) void k_tau_bwd(SceneView S, MaskView M, const float* __restrict__ rays, int n,
                                                 int tile_w, const float* __restrict__ dL_dtau,
                                                 const float* __restrict__ dL_dT, const float* __restrict__ T,
                                                 float* __restrict__ dparams) {
    __shared__ int stk[PK_WAVES][GF_STACK];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int idx = packet_ray(blockIdx.x * PK_WAVES + w, lane, n, tile_w);
    float gr = 0.0f;
    if (idx >= 0) {
        gr = dL_dtau[idx];
        if (dL_dT) gr -= dL_dT[idx] * T[idx];
    }
    const bool valid = idx >= 0 && gr != 0.0f;
    RayD R = valid ? load_ray(rays, idx) : RayD{0, 0, 0, 0, 0, 1, 1.0f, 0.0f};
    int nn = 0;
    packet_traverse(S, M, valid, R, stk[w], nn, [&](int j, bool active) {
        PrimF P = load_prim(S.prims, j);
        if (M.prim_bits && !((M.prim_bits[P.orig >> 5] >> (P.orig & 31)) & 1u)) return;
        float g[15];
#pragma unroll
        for (int k = 0; k < 15; ++k) g[k] = 0.0f;
        HitGeom H;
        bool hit = active && hit_geom(P, R, S.A64 + (size_t)j * GF_A64, H) && lod_keep64(P, R, H, M.lod_k);
        if (hit) hit_grad(P, S.aux + (size_t)j * 3, H, R, P.r2, gr, g);
        if (!__ballot(hit)) return;
        float* dst = dparams + (size_t)P.orig * 15;
#pragma unroll
        for (int k = 0; k < 15; ++k) {
            float t = wave_sum(g[k]);
            if (lane == 0 && t != 0.0f) atomicAdd(dst + k, t);
        }
    });
}

extern "C" gf_status gf_optical_depth_backward(gf_scene s, const float* rays, int64_t n, int image_width,
                                               gf_mask mask, const float* dL_dtau, const float* dL_dT,
                                               const float* T, float* dparams, void* stream) {
    if (!s || !dparams || (n && (!rays || !dL_dtau)))
        return gf_fail(GF_EINVAL, "gf_optical_depth_backward: NULL argument");
    if ((dL_dT == nullptr) != (T == nullptr))
        return gf_fail(GF_EINVAL, "gf_optical_depth_backward: dL_dT and T must be both given or both NULL");
    hipStream_t sm = (hipStream_t)stream;
    gf_status st = gf_check_rays(n, image_width, "gf_optical_depth_backward");
    if (st == GF_OK) st = gf_check_mask(mask, "gf_optical_depth_backward");
    if (st == GF_OK && n > 0) st = gf_validate_rays(rays, n, sm, "gf_optical_depth_backward");
    if (st == GF_OK) st = gf_zero_words(dparams, 15 * (size_t)s->n, sm);
    if (st != GF_OK || n == 0) return st;
    k_tau_bwd<<<gf_packet_blocks(n, image_width), 256, 0, sm>>>(gf_scene_view(s), gf_mask_view(mask), rays, (int)n,
                                                               image_width, dL_dtau, dL_dT, T, dparams);
    GF_HIP(hipGetLastError());
    return GF_OK;
}
