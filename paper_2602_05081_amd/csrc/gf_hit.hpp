// Per-hit geometry and the closed-form segment integral (device code).
//
// For primitive i and ray x(t) = o + t v:
//   A = Sigma^-1, tc = -(d.Av)/(v.Av) with d = o - mu (binary64), y_c = d + tc v,
//   n = sqrt(v.Av), h^2 = y_c.A y_c, whitened arc length u = n (t - tc), so the
//   Mahalanobis form is M = h^2 + u^2 and the carrier phase is
//   psi(u) = theta + Omega u, theta = 2 pi f.y_c + phi, Omega = 2 pi f.v / n.
// The chord {M < r^2} is u in [-sqrt(r^2 - h^2), +sqrt(r^2 - h^2)], clipped
// to [tmin, tmax].  With E(u) = exp(-Omega^2/2) erf((u - i Omega)/sqrt 2)
// the segment integral (Sec. 4.4, definite form; Appendix A) is
//   tau_i = amp / n * exp(-h^2/2) * Re{ e^{i theta} [E(u_b) - E(u_a)] },
//   amp = rho alpha / (4 pi s0 s1 s2),
// and erfc(z) = exp(-z^2) w(iz) gives the bounded form
//   Re{e^{i theta} E(u)} = sgn(u) [exp(-Omega^2/2) cos theta
//                          - exp(-u^2/2) Re{e^{i psi(u)} w((sgn(u) Omega + i|u|)/sqrt 2)}].
// Phases are carried in cycles in binary64 and reduced before the float32
// sin/cos; the geometry setup is binary64 (FP64 VALU runs at the float32 rate
// on CDNA when packed float32 math is off).  Segments shorter than 1e-4 in
// whitened units use the midpoint rule (Sec. 4.4, implementation details);
// other short segments use Gauss-Legendre (see hit_value).
#pragma once

#include "gf_internal.hpp"

#define WEID_N 16

// w(z) for Im z >= 0 by Weideman's rational approximation (SIAM J. Numer.
// Anal. 31, 1994): w(z) ~ 2 p(Z) / (L - iz)^2 + (1/sqrt pi) / (L - iz),
// Z = (L + iz)/(L - iz), p a degree-15 polynomial (coefficients in `a`,
// highest power first).
static __device__ __forceinline__ float2 wofz_weideman(float x, float y, const float* __restrict__ a, float L) {
    // iz = -y + i x;  D = L - iz = (L + y) - i x;  N = L + iz = (L - y) + i x
    float dr = L + y, di = -x;
    float nr = L - y, ni = x;
    float inv = 1.0f / (dr * dr + di * di);
    float ir = dr * inv, ii = -di * inv;  // 1/D
    float zr = nr * ir - ni * ii, zi = nr * ii + ni * ir;
    float pr = a[0], pi = 0.0f;
#pragma unroll
    for (int k = 1; k < WEID_N; ++k) {
        float tr = pr * zr - pi * zi + a[k];
        pi = pr * zi + pi * zr;
        pr = tr;
    }
    float i2r = ir * ir - ii * ii, i2i = 2.0f * ir * ii;  // 1/D^2
    const float isp = 0.56418958354775628695f;            // 1/sqrt(pi)
    float wr = 2.0f * (pr * i2r - pi * i2i) + isp * ir;
    float wi = 2.0f * (pr * i2i + pi * i2r) + isp * ii;
    return make_float2(wr, wi);
}

#define WEID64_N 32

// The same rational approximation in binary64 with N = 32 (coefficients `a`,
// highest power first); used only for ill-conditioned hits.
static __device__ __forceinline__ void wofz_weideman64(double x, double y, const double* __restrict__ a, double L,
                                                       double* wr, double* wi) {
    double dr = L + y, di = -x;
    double nr = L - y, ni = x;
    double inv = 1.0 / (dr * dr + di * di);
    double ir = dr * inv, ii = -di * inv;
    double zr = nr * ir - ni * ii, zi = nr * ii + ni * ir;
    double pr = a[0], pi = 0.0;
    for (int k = 1; k < WEID64_N; ++k) {
        double tr = pr * zr - pi * zi + a[k];
        pi = pr * zi + pi * zr;
        pr = tr;
    }
    double i2r = ir * ir - ii * ii, i2i = 2.0 * ir * ii;
    const double isp = 0.56418958354775628695;
    *wr = 2.0 * (pr * i2r - pi * i2i) + isp * ir;
    *wi = 2.0 * (pr * i2i + pi * i2r) + isp * ii;
}

struct PrimF {
    float mux, muy, muz, phi;
    float a00, a01, a02, a11, a12, a22;
    float fx, fy, fz, amp;
    float r2;  // square of the truncation radius
    int cell, orig;
};

static __device__ __forceinline__ PrimF load_prim(const float4* __restrict__ prims, int j) {
    float4 r0 = prims[(size_t)j * 4 + 0], r1 = prims[(size_t)j * 4 + 1];
    float4 r2 = prims[(size_t)j * 4 + 2], r3 = prims[(size_t)j * 4 + 3];
    PrimF p;
    p.mux = r0.x; p.muy = r0.y; p.muz = r0.z; p.phi = r0.w;
    p.a00 = r1.x; p.a01 = r1.y; p.a02 = r1.z; p.a11 = r1.w;
    p.a12 = r2.x; p.a22 = r2.y; p.fx = r2.z; p.fy = r2.w;
    p.fz = r3.x; p.amp = r3.y; p.r2 = r3.z; p.cell = rec_cell(r3.w); p.orig = rec_orig(r3.w);
    return p;
}

struct RayD {
    double ox, oy, oz, vx, vy, vz;
    float tmin, tmax;
};

// Geometry of one hit; returns false when the clipped chord is empty.
struct HitGeom {
    double tc, n, inv_n;
    double ycx, ycy, ycz;
    double thc;   // theta in cycles (phase at the closest point)
    double omc;   // Omega in cycles per whitened unit
    float h2, half, ua, ub;
    double h2d, halfd, uad, ubd;  // binary64 versions for ill-conditioned hits
    bool enda, endb;
};

// Geometry from A (a00 a01 a02 a11 a12 a22).  Returns 0 when the clipped
// chord is empty, 1 on a hit, 2 (float32 path only) when h^2 lies within
// [r^2 - 0.05, r^2 + 0.01) and must be redone with binary64 A.
static __device__ __forceinline__ int hit_geom_a(const PrimF& P, const RayD& R, double r2, const double* A,
                                                 bool h2_double, HitGeom& H) {
    double dx = R.ox - P.mux, dy = R.oy - P.muy, dz = R.oz - P.muz;
    double avx = A[0] * R.vx + A[1] * R.vy + A[2] * R.vz;
    double avy = A[1] * R.vx + A[3] * R.vy + A[4] * R.vz;
    double avz = A[2] * R.vx + A[4] * R.vy + A[5] * R.vz;
    double a = R.vx * avx + R.vy * avy + R.vz * avz;
    double beta = dx * avx + dy * avy + dz * avz;
    double inv_a = 1.0 / a;
    double tc = -beta * inv_a;
    double ycx = dx + tc * R.vx, ycy = dy + tc * R.vy, ycz = dz + tc * R.vz;
    double h2d;
    float h2;
    if (h2_double) {
        h2d = ycx * (A[0] * ycx + A[1] * ycy + A[2] * ycz) + ycy * (A[1] * ycx + A[3] * ycy + A[4] * ycz) +
              ycz * (A[2] * ycx + A[4] * ycy + A[5] * ycz);
        h2 = (float)h2d;
        if (!(h2d < (double)r2)) return 0;
    } else {
        float yx = (float)ycx, yy = (float)ycy, yz = (float)ycz;
        h2 = yx * (P.a00 * yx + P.a01 * yy + P.a02 * yz) + yy * (P.a01 * yx + P.a11 * yy + P.a12 * yz) +
             yz * (P.a02 * yx + P.a12 * yy + P.a22 * yz);
        if (!(h2 < r2 + 0.01f)) return 0;
        if (h2 > r2 - 0.05f) return 2;
        h2d = h2;
    }
    double n = sqrt(a);
    double inv_n = n * inv_a;
    double halfd = sqrt((double)r2 - h2d);
    float half = (float)halfd;
    double hn = halfd * inv_n;
    double tin = tc - hn, tout = tc + hn;
    double ta = fmax((double)R.tmin, tin), tb = fmin((double)R.tmax, tout);
    if (!(ta < tb)) return 0;
    H.enda = !((double)R.tmin > tin);
    H.endb = !((double)R.tmax < tout);
    H.uad = H.enda ? -halfd : n * (ta - tc);
    H.ubd = H.endb ? halfd : n * (tb - tc);
    H.ua = (float)H.uad;
    H.ub = (float)H.ubd;
    H.h2d = h2d;
    H.halfd = halfd;
    H.tc = tc;
    H.n = n;
    H.inv_n = inv_n;
    H.ycx = ycx;
    H.ycy = ycy;
    H.ycz = ycz;
    H.h2 = h2;
    H.half = half;
    H.thc = (double)P.fx * ycx + (double)P.fy * ycy + (double)P.fz * ycz + (double)P.phi * GF_INV_2PI;
    H.omc = ((double)P.fx * R.vx + (double)P.fy * R.vy + (double)P.fz * R.vz) * inv_n;
    return 1;
}

// Chord geometry of one hit from the binary64 record of primitive j
// (Sigma^-1 and the squared truncation radius); false when the clipped
// chord is empty.
static __device__ __forceinline__ bool hit_geom(const PrimF& P, const RayD& R, const double* __restrict__ A64j,
                                                HitGeom& H) {
    double A[6] = {A64j[0], A64j[1], A64j[2], A64j[3], A64j[4], A64j[5]};
    return hit_geom_a(P, R, A64j[6], A, true, H) == 1;
}

// Continuous LOD in binary64 (supplementary "LOD Selection"): primitive P
// stays on ray R unless its closest point lies ahead of the origin, at the
// distance d = tc |v|, with |f| d > lod_k (0: no cutoff).  The cutoff itself
// is held fixed by the adjoint.
static __device__ __forceinline__ bool lod_keep64(const PrimF& P, const RayD& R, const HitGeom& H, float lod_k) {
#pragma clang fp contract(off)
    if (!(lod_k > 0.0f) || !(H.tc > 0.0)) return true;
    double f2 = ((double)P.fx * P.fx + (double)P.fy * P.fy) + (double)P.fz * P.fz;
    double v2 = R.vx * R.vx + R.vy * R.vy + R.vz * R.vz;
    return f2 * (H.tc * H.tc * v2) <= (double)lod_k * (double)lod_k;
}

// Gauss-Legendre, 8 nodes on [-1, 1] (positive half; the rule is symmetric)
__constant__ static const float c_gl8x[4] = {0.18343464249564980f, 0.52553240991632899f, 0.79666647741362674f,
                                             0.96028985649753623f};
__constant__ static const float c_gl8w[4] = {0.36268378337836198f, 0.31370664587788729f, 0.22238103445337447f,
                                             0.10122853629037626f};

// int_{ua}^{ub} exp(-u^2/2) cos(psi(u)) du by composite 8-point Gauss-Legendre
// on `panels` equal panels
static __device__ float gl8_segment(float ua, float ub, double thc, double omc, int panels) {
    float w = (ub - ua) / panels;
    float acc = 0.0f;
    for (int p = 0; p < panels; ++p) {
        float c = ua + (p + 0.5f) * w, h = 0.5f * w;
        float part = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float d = h * c_gl8x[k];
            float u1 = c - d, u2 = c + d;
            float s1, c1, s2, c2;
            sincos_cycles(thc + (double)u1 * omc, &s1, &c1);
            sincos_cycles(thc + (double)u2 * omc, &s2, &c2);
            part += c_gl8w[k] * (__expf(-0.5f * u1 * u1) * c1 + __expf(-0.5f * u2 * u2) * c2);
        }
        acc += part * h;
    }
    return acc;
}

// e^{-u^2/2} Re{e^{i psi(u)} w((sgn(u) Omega + i|u|)/sqrt 2)}: the part of
// Re{e^{i theta} E(u)} that depends on the end point; *mag receives
// e^{-u^2/2} |w|, the size of the terms the real part is taken from (the
// real part cancels when the phase lines up with w).
static __device__ __forceinline__ float tail_term(float u, float Om, double thc, double omc,
                                                  const float* __restrict__ wa, float wL, float* mag) {
    const float is2 = 0.70710678118654752440f;
    float sg = u < 0.0f ? -1.0f : 1.0f;
    float2 w = wofz_weideman(sg * Om * is2, fabsf(u) * is2, wa, wL);
    float sp, cp;
    sincos_cycles(thc + (double)u * omc, &sp, &cp);
    float e = __expf(-0.5f * u * u);
    *mag = e * sqrtf(w.x * w.x + w.y * w.y);
    return e * (cp * w.x - sp * w.y);
}

// The closed form entirely in binary64 (for hits whose float32 closed form
// cancels by more than a factor 16).
static __device__ float hit_value64(const PrimF& P, const HitGeom& H, const double* __restrict__ wa, double wL) {
    const double is2 = 0.70710678118654752440;
    double Om = 2.0 * GF_PI * H.omc;
    double eO = exp(-0.5 * Om * Om);
    double sth, cth;
    sincospi(2.0 * (H.thc - rint(H.thc)), &sth, &cth);
    double us[2] = {H.uad, H.ubd};
    double f[2];
    for (int e = 0; e < 2; ++e) {
        double u = us[e];
        double sg = u < 0.0 ? -1.0 : 1.0;
        double wr, wi;
        wofz_weideman64(sg * Om * is2, fabs(u) * is2, wa, wL, &wr, &wi);
        double c = H.thc + u * H.omc;
        double sp, cp;
        sincospi(2.0 * (c - rint(c)), &sp, &cp);
        f[e] = sg * (eO * cth - exp(-0.5 * u * u) * (cp * wr - sp * wi));
    }
    double pre = (double)P.amp * H.inv_n * exp(-0.5 * H.h2d);
    return (float)(pre * (f[1] - f[0]));
}

// tau_i (including rho alpha) of one hit with a non-empty chord.
// Closed form: tau_i = pre Re{e^{i theta}[E(u_b) - E(u_a)]}, with
// Re{e^{i theta}E(u)} = sgn(u) [exp(-Omega^2/2) cos theta - tail_term(u)].
// Where that difference or a tail term's real part cancels (the segment
// integral is much smaller than the terms it is made of, as for a strongly
// oscillating kernel whose integral comes from its truncated ends, or the
// segment is short) float32 loses the digits:
// below 1e-4 whitened units the midpoint rule is used; short segments
// (len (1 + |Omega| + max|u|) < 4) use 8-point Gauss-Legendre; where the
// float32 closed form cancels by more than a factor 16 it is redone in
// binary64.
static __device__ __forceinline__ float hit_value(const PrimF& P, const HitGeom& H, const float* __restrict__ wa,
                                                  float wL, const double* __restrict__ wa64, double wL64) {
    const float sq2pi = 0.79788456080286535588f;  // sqrt(2/pi)
    float Om = (float)(2.0 * GF_PI * H.omc);
    float pre = P.amp * (float)H.inv_n * __expf(-0.5f * H.h2);
    float len = H.ub - H.ua;
    if (len < 1e-4f) {
        float um = 0.5f * (H.ua + H.ub);
        float sp, cp;
        sincos_cycles(H.thc + (double)um * H.omc, &sp, &cp);
        return pre * sq2pi * len * __expf(-0.5f * um * um) * cp;
    }
    float q = len * (1.0f + fabsf(Om) + fmaxf(fabsf(H.ua), fabsf(H.ub)));
    if (q < 4.0f) return pre * sq2pi * gl8_segment(H.ua, H.ub, H.thc, H.omc, 1);
    float sth, cth;
    sincos_cycles(H.thc, &sth, &cth);
    float eO = __expf(-0.5f * Om * Om);
    float val, mag;
    if (H.enda && H.endb) {
        // unclipped chord: E(h) - E(-h) = 2 Re E(h)
        float mt;
        float t = tail_term(H.half, Om, 0.0, H.omc, wa, wL, &mt);
        float reE = eO - t;
        val = 2.0f * cth * reE;
        mag = 2.0f * fabsf(cth) * (eO + mt);
    } else {
        float sa = H.ua < 0.0f ? -1.0f : 1.0f, sb = H.ub < 0.0f ? -1.0f : 1.0f;
        float mb, ma;
        float tb = tail_term(H.ub, Om, H.thc, H.omc, wa, wL, &mb), ta = tail_term(H.ua, Om, H.thc, H.omc, wa, wL, &ma);
        val = (sb - sa) * eO * cth - sb * tb + sa * ta;
        mag = fabsf((sb - sa) * eO * cth) + mb + ma;
    }
    if (mag > 16.0f * fabsf(val)) return hit_value64(P, H, wa64, wL64);
    return pre * val;
}

// Host: Weideman's coefficients (binary64 DFT) for N = 16 rounded to float32,
// and for N = 32 in binary64.
void gf_weideman_coeffs(float* a, float* L);
void gf_weideman_coeffs64(double* a, double* L);

#define PK_WAVES 4

// ray index of lane `lane` in global wave `gw`; -1 when outside.  With an
// image width W > 0 each wave takes an 8x8 pixel tile of the row-major image.
static __device__ __forceinline__ int packet_ray(int gw, int lane, int n, int tile_w) {
    if (tile_w <= 0) {
        int i = gw * 64 + lane;
        return i < n ? i : -1;
    }
    int tiles_x = tile_w >> 3;
    int height = n / tile_w;
    int px = (gw % tiles_x) * 8 + (lane & 7), py = (gw / tiles_x) * 8 + (lane >> 3);
    return py < height ? py * tile_w + px : -1;
}

static __device__ __forceinline__ RayD load_ray(const float* __restrict__ rays, int idx) {
    RayD R;
    const float* r = rays + (size_t)idx * 8;
    R.ox = r[0]; R.oy = r[1]; R.oz = r[2];
    R.vx = r[3]; R.vy = r[4]; R.vz = r[5];
    R.tmin = r[6]; R.tmax = r[7];
    return R;
}

// Wave-packet depth-first traversal of the LBVH: the node index, the stack
// (LDS, `stk`, GF_STACK entries) and the leaf index are wave-uniform; each
// lane tests its own ray against both child boxes and the wave descends where
// any lane hits.  leaf(j, active) is called wave-uniformly for every leaf
// whose box meets some lane's ray (active: this lane's ray meets it) and whose
// cell is in the mask.  node_hits counts this lane's box hits.
template <class LeafFn>
static __device__ __forceinline__ void packet_traverse(const SceneView& S, const MaskView& M, bool valid,
                                                       const RayD& R, int* __restrict__ stk, int& node_hits,
                                                       LeafFn&& leaf) {
    const float ix = 1.0f / (float)R.vx, iy = 1.0f / (float)R.vy, iz = 1.0f / (float)R.vz;
    const float ox = (float)R.ox, oy = (float)R.oy, oz = (float)R.oz;
    if (S.n == 1) {
        leaf(0, valid);
        node_hits += valid ? 1 : 0;
        return;
    }
    int sp = 0;
    int node = 0;
    node_hits += valid ? 1 : 0;  // root
    for (;;) {
        const TNode* nd = S.nodes + node;
        uint32_t cells = nd->cells;
        uint32_t cl = cells & 0xffffu & M.cells, cr = (cells >> 16) & M.cells;
        bool hl = valid && cl && slab_hit(nd->lbox, ox, oy, oz, ix, iy, iz, R.tmin, R.tmax);
        bool hr = valid && cr && slab_hit(nd->rbox, ox, oy, oz, ix, iy, iz, R.tmin, R.tmax);
        node_hits += (int)hl + (int)hr;
        uint64_t bl = __ballot(hl), br = __ballot(hr);
        int lc = nd->lchild, rc = nd->rchild;
        if (bl && lc < 0) {
            leaf(~lc, hl);
            bl = 0;
        }
        if (br && rc < 0) {
            leaf(~rc, hr);
            br = 0;
        }
        if (bl && br) {
            stk[sp] = rc;
            ++sp;
            node = lc;
        } else if (bl) {
            node = lc;
        } else if (br) {
            node = rc;
        } else {
            if (sp == 0) break;
            --sp;
            node = stk[sp];
        }
        node = uniform_int(node);
    }
}
