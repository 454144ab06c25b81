// Stochastic transport on the majorant grid: point density, ratio-tracking
// transmittance, weighted delta tracking, single / multiple scattering with
// fixed or per-segment stochastic masks (Sec. 3 radiative transfer; Sec. 4.5.1-
// 4.5.2 and Appendix B for the masks; local majorants after the voxel
// baseline's super-voxel grid).
//
// Per lane: one ray (all its samples, so per-ray sums are deterministic and
// independent of which rays share a wave).  A point-density query walks the
// LBVH with a per-lane stack in LDS, descending into children whose box
// contains the point and whose subtree holds a cell of non-zero weight.
#include <math.h>

#include "gf_hit.hpp"

#define TR_THREADS 64
#define TR_STACK 64

// Per-cell density weights w and majorant weights mw = min(w, MAJ_CAP).  The
// cap bounds the work of a path that drew a heavily weighted (rarely drawn)
// bin; ratio tracking and the signed-weight delta tracking stay unbiased when
// the majorant falls below |kappa| (only their variance grows).
#define MAJ_CAP 16.0f

struct CellW {
    float w[GF_NCELLS];
    float mw[GF_NCELLS];
    uint32_t cells;  // cells with non-zero weight
};

static __device__ __forceinline__ void fixed_weights(const MaskView& M, CellW& cw) {
#pragma unroll
    for (int c = 0; c < GF_NCELLS; ++c) cw.w[c] = cw.mw[c] = ((M.cells >> c) & 1u) ? 1.0f : 0.0f;
    cw.cells = M.cells;
}

// Uniform + control variate over levels, importance sampling over bins:
// level 0 keeps weight 1; one level l in 1..3 (probability 1/3) and one bin k
// (probability w_k / W, w_k = exp(-m_lk^2 a_k^2 / 2), a_k = |v_k| / |v|) get
// weight 3 W / w_k; every other cell weight 0.
static __device__ __forceinline__ void stochastic_weights(const SceneView& S, float vx, float vy, float vz, Rng& g,
                                                          CellW& cw) {
    float ul = g.u(), ub = g.u();
    int l = 1 + (int)(ul * 3.0f);
    l = l > 3 ? 3 : l;
    float vn2 = vx * vx + vy * vy + vz * vz;
    float a2[3] = {vx * vx / vn2, vy * vy / vn2, vz * vz / vn2};
    // log weights, normalised by their maximum so that W >= 1 never underflows
    float lw[3], mx = -INFINITY;
    for (int k = 0; k < 3; ++k) {
        float m = S.med[3 * l + k];
        lw[k] = -0.5f * m * m * a2[k];
        mx = fmaxf(mx, lw[k]);
    }
    float wk[3], W = 0.0f;
    for (int k = 0; k < 3; ++k) {
        wk[k] = __expf(lw[k] - mx);
        W += wk[k];
    }
    // inverse CDF over bins with non-zero weight
    int k = -1;
    float acc = 0.0f, target = ub * W;
    for (int j = 0; j < 3; ++j) {
        if (wk[j] <= 0.0f) continue;
        k = j;
        acc += wk[j];
        if (target < acc) break;
    }
#pragma unroll
    for (int c = 0; c < GF_NCELLS; ++c) cw.w[c] = cw.mw[c] = c < 3 ? 1.0f : 0.0f;
    int pick = 3 * l + k;
    cw.w[pick] = 3.0f * W / wk[k];
    cw.mw[pick] = fminf(cw.w[pick], MAJ_CAP);
    cw.cells = 0x7u | (1u << pick);
}

// Work counters of the counting variants (per lane, summed at the end):
// tentative collisions, internal nodes visited by point queries, primitive
// records read at leaves, voxels walked.
struct Work {
    unsigned long long tent, nodes, prims, voxels;
};

// kappa at x under per-cell weights (rho alpha c exp(-M/2) cos(psi) summed)
template <bool COUNT>
static __device__ float point_density(const SceneView& S, const MaskView& M, const CellW& cw, float x, float y,
                                      float z, int* __restrict__ stk, Work& wk) {
    float acc = 0.0f;
    auto leaf = [&](int j) {
        PrimF P = load_prim(S.prims, j);
        if (COUNT) ++wk.prims;
        float wgt = cw.w[P.cell];
        if (wgt == 0.0f) return;
        if (M.prim_bits && !((M.prim_bits[P.orig >> 5] >> (P.orig & 31)) & 1u)) return;
        float dx = x - P.mux, dy = y - P.muy, dz = z - P.muz;
        float m = dx * (P.a00 * dx + P.a01 * dy + P.a02 * dz) + dy * (P.a01 * dx + P.a11 * dy + P.a12 * dz) +
                  dz * (P.a02 * dx + P.a12 * dy + P.a22 * dz);
        if (!(m < S.r2)) return;
        float ph = P.fx * dx + P.fy * dy + P.fz * dz + P.phi * (float)GF_INV_2PI;
        float s, c;
        sincos2pi(ph - rintf(ph), &s, &c);
        acc += wgt * P.amp * 0.79788456080286535588f * __expf(-0.5f * m) * c;
    };
    if (S.n == 1) {
        leaf(0);
        return acc;
    }
    int sp = 0, node = 0;
    for (;;) {
        const TNode* nd = S.nodes + node;
        if (COUNT) ++wk.nodes;
        uint32_t cells = nd->cells;
        bool hl = (cells & 0xffffu & cw.cells) && box_contains(nd->lbox, x, y, z);
        bool hr = ((cells >> 16) & cw.cells) && box_contains(nd->rbox, x, y, z);
        int lc = nd->lchild, rc = nd->rchild;
        if (hl && lc < 0) {
            leaf(~lc);
            hl = false;
        }
        if (hr && rc < 0) {
            leaf(~rc);
            hr = false;
        }
        if (hl && hr) {
            stk[sp * TR_THREADS] = rc;
            ++sp;
            node = lc;
        } else if (hl) {
            node = lc;
        } else if (hr) {
            node = rc;
        } else {
            if (sp == 0) break;
            --sp;
            node = stk[sp * TR_THREADS];
        }
    }
    return acc;
}

// ---------------------------------------------------------------------------
// Local majorants along a ray (per-lane LBVH traversal restricted to a
// segment).  Pass A accumulates, for TB_BINS equal bins of the segment, the sum
// over every chord crossing the bin of rho w_c |alpha| c exp(-m/2) (m the
// minimum of the Mahalanobis form over the bin: h^2 + n^2 (clamp(tc) - tc)^2):
// a piecewise-constant majorant of |kappa| made only of primitives the ray
// actually crosses.  Tentative points are drawn from it in rounds of up to
// TB_PTS; pass B re-traverses the t-range of a round and adds every crossed
// primitive's density at every point of the round (no per-point queries).
// ---------------------------------------------------------------------------
#define TB_BINS 32
#define TB_PTS 8
// Hard bound on tentative points per segment: a segment that would need more
// (a majorant beyond any produced by the scenes here) is cut short there,
// which keeps every wave's work finite.
#define TB_MAX_TENT 65536

struct Lane {
    int* stk;     // TR_STACK entries, stride TR_THREADS
    float* bins;  // TB_BINS
    float* pt;    // TB_PTS tentative distances
    float* pm;    // majorant at each point
    float* pk;    // density at each point
};

// chord of primitive P with the ray in float32 (stochastic paths): returns
// false when M < r^2 misses [ta, tb]; otherwise the chord [ci, co], the
// closest-point parameter tc, n^2 = v.Av and h^2.
struct ChordF {
    float ci, co, tc, n2, h2;
};

static __device__ __forceinline__ bool chord_f32(const PrimF& P, float r2, float ox, float oy, float oz, float vx,
                                                 float vy, float vz, float ta, float tb, ChordF& C,
                                                 bool inclusive = false) {
    float dx = ox - P.mux, dy = oy - P.muy, dz = oz - P.muz;
    float avx = P.a00 * vx + P.a01 * vy + P.a02 * vz;
    float avy = P.a01 * vx + P.a11 * vy + P.a12 * vz;
    float avz = P.a02 * vx + P.a12 * vy + P.a22 * vz;
    float a = vx * avx + vy * avy + vz * avz;
    float tc = -(dx * avx + dy * avy + dz * avz) / a;
    float yx = dx + tc * vx, yy = dy + tc * vy, yz = dz + tc * vz;
    float h2 = yx * (P.a00 * yx + P.a01 * yy + P.a02 * yz) + yy * (P.a01 * yx + P.a11 * yy + P.a12 * yz) +
               yz * (P.a02 * yx + P.a12 * yy + P.a22 * yz);
    if (!(h2 < r2)) return false;
    float hw = sqrtf((r2 - h2) / a);
    C.ci = fmaxf(ta, tc - hw);
    C.co = fminf(tb, tc + hw);
    if (inclusive ? !(C.ci <= C.co) : !(C.ci < C.co)) return false;
    C.tc = tc;
    C.n2 = a;
    C.h2 = h2;
    return true;
}

// per-lane traversal of the nodes whose box meets [ta, tb] (and whose cells
// carry weight); leaf(j) for each such leaf
template <bool COUNT, class LeafFn>
static __device__ __forceinline__ void lane_traverse(const SceneView& S, uint32_t cells, float ox, float oy, float oz,
                                                     float vx, float vy, float vz, float ta, float tb,
                                                     int* __restrict__ stk, Work& wk, LeafFn&& leaf) {
    if (S.n == 1) {
        leaf(0);
        return;
    }
    const float ix = 1.0f / vx, iy = 1.0f / vy, iz = 1.0f / vz;
    int sp = 0, node = 0;
    for (;;) {
        const TNode* nd = S.nodes + node;
        if (COUNT) ++wk.nodes;
        uint32_t c = nd->cells;
        bool hl = (c & 0xffffu & cells) && slab_hit(nd->lbox, ox, oy, oz, ix, iy, iz, ta, tb);
        bool hr = ((c >> 16) & cells) && slab_hit(nd->rbox, ox, oy, oz, ix, iy, iz, ta, tb);
        int lc = nd->lchild, rc = nd->rchild;
        if (hl && lc < 0) {
            leaf(~lc);
            hl = false;
        }
        if (hr && rc < 0) {
            leaf(~rc);
            hr = false;
        }
        if (hl && hr) {
            stk[sp * TR_THREADS] = rc;
            ++sp;
            node = lc;
        } else if (hl) {
            node = lc;
        } else if (hr) {
            node = rc;
        } else {
            if (sp == 0) break;
            --sp;
            node = stk[sp * TR_THREADS];
        }
    }
}

// clip [t0, t1] to the scene box
static __device__ __forceinline__ bool clip_box(const SceneView& S, float ox, float oy, float oz, float vx, float vy,
                                                float vz, float& t0, float& t1) {
    float o[3] = {ox, oy, oz}, v[3] = {vx, vy, vz};
    for (int a = 0; a < 3; ++a) {
        if (v[a] == 0.0f) {
            if (o[a] < S.glo[a] || o[a] > S.ghi[a]) return false;
            continue;
        }
        float iv = 1.0f / v[a];
        float u0 = (S.glo[a] - o[a]) * iv, u1 = (S.ghi[a] - o[a]) * iv;
        t0 = fmaxf(t0, fminf(u0, u1));
        t1 = fminf(t1, fmaxf(u0, u1));
    }
    return t0 < t1;
}

template <bool COUNT>
static __device__ void pass_majorant(const SceneView& S, const MaskView& M, const CellW& cw, float ox, float oy,
                                     float oz, float vx, float vy, float vz, float ta, float tb, const Lane& L,
                                     Work& wk) {
    for (int k = 0; k < TB_BINS; ++k) L.bins[k * TR_THREADS] = 0.0f;
    const float inv_dt = TB_BINS / (tb - ta), dt = (tb - ta) / TB_BINS;
    lane_traverse<COUNT>(S, cw.cells, ox, oy, oz, vx, vy, vz, ta, tb, L.stk, wk, [&](int j) {
        PrimF P = load_prim(S.prims, j);
        if (COUNT) ++wk.prims;
        float wgt = cw.mw[P.cell];
        if (wgt == 0.0f) return;
        if (M.prim_bits && !((M.prim_bits[P.orig >> 5] >> (P.orig & 31)) & 1u)) return;
        ChordF C;
        if (!chord_f32(P, S.r2, ox, oy, oz, vx, vy, vz, ta, tb, C)) return;
        float peak = wgt * fabsf(P.amp) * 0.79788456080286535588f * 1.0001f;  // rho w |alpha| c
        int k0 = max(0, min(TB_BINS - 1, (int)floorf((C.ci - ta) * inv_dt)));
        int k1 = max(0, min(TB_BINS - 1, (int)floorf((C.co - ta) * inv_dt)));
        for (int k = k0; k <= k1; ++k) {
            float blo = ta + k * dt, bhi = blo + dt;
            float du = fminf(fmaxf(C.tc, blo), bhi) - C.tc;
            // shrink the minimum slightly so float32 rounding never raises it
            float m = (C.h2 + C.n2 * du * du) * 0.999f;
            L.bins[k * TR_THREADS] += peak * __expf(-0.5f * m);
        }
    });
}

// density at the np points (sorted, within [pa, pb]) into L.pk
template <bool COUNT>
static __device__ void pass_density(const SceneView& S, const MaskView& M, const CellW& cw, float ox, float oy,
                                    float oz, float vx, float vy, float vz, int np, const Lane& L, Work& wk) {
    float pa = L.pt[0], pb = L.pt[(np - 1) * TR_THREADS];
    for (int k = 0; k < np; ++k) L.pk[k * TR_THREADS] = 0.0f;
    lane_traverse<COUNT>(S, cw.cells, ox, oy, oz, vx, vy, vz, pa, pb, L.stk, wk, [&](int j) {
        PrimF P = load_prim(S.prims, j);
        if (COUNT) ++wk.prims;
        float wgt = cw.w[P.cell];
        if (wgt == 0.0f) return;
        if (M.prim_bits && !((M.prim_bits[P.orig >> 5] >> (P.orig & 31)) & 1u)) return;
        ChordF C;
        if (!chord_f32(P, S.r2, ox, oy, oz, vx, vy, vz, pa, pb, C, true)) return;
        float amp = wgt * P.amp * 0.79788456080286535588f;
        for (int k = 0; k < np; ++k) {
            float t = L.pt[k * TR_THREADS];
            if (t < C.ci || t > C.co) continue;
            float x = ox + t * vx, y = oy + t * vy, z = oz + t * vz;
            float dx = x - P.mux, dy = y - P.muy, dz = z - P.muz;
            float m = dx * (P.a00 * dx + P.a01 * dy + P.a02 * dz) + dy * (P.a01 * dx + P.a11 * dy + P.a12 * dz) +
                      dz * (P.a02 * dx + P.a12 * dy + P.a22 * dz);
            if (!(m < S.r2)) continue;
            float ph = P.fx * dx + P.fy * dy + P.fz * dz + P.phi * (float)GF_INV_2PI;
            float sn, cs;
            sincos2pi(ph - rintf(ph), &sn, &cs);
            L.pk[k * TR_THREADS] += amp * __expf(-0.5f * m) * cs;
        }
    });
}

// Draws the next round of tentative points from the binned majorant,
// continuing from (t, bin).  Returns the number of points (0 when the
// segment is exhausted).  The process restarts at each bin boundary
// (memoryless).
static __device__ __forceinline__ int draw_points(float ta, float tb, const Lane& L, float& t, int& bin, Rng& g) {
    const float dt = (tb - ta) / TB_BINS;
    int np = 0;
    while (bin < TB_BINS && np < TB_PTS) {
        float kb = L.bins[bin * TR_THREADS];
        float bend = bin == TB_BINS - 1 ? tb : ta + (bin + 1) * dt;
        if (!(kb > 0.0f)) {
            t = bend;
            ++bin;
            continue;
        }
        float tn = t - __logf(g.u()) / kb;
        if (tn >= bend) {
            t = bend;
            ++bin;
            continue;
        }
        t = fmaxf(tn, nextafterf(t, INFINITY));  // strict progress in float32
        L.pt[np * TR_THREADS] = t;
        L.pm[np * TR_THREADS] = kb;
        ++np;
    }
    return np;
}

// Ratio tracking over [t0, t1]: T = prod (1 - kappa / kbar).
template <bool COUNT>
static __device__ float ratio_track(const SceneView& S, const MaskView& M, const CellW& cw, float ox, float oy,
                                    float oz, float vx, float vy, float vz, float t0, float t1, Rng& g, const Lane& L,
                                    Work& wk) {
    float ta = t0, tb = t1;
    if (!clip_box(S, ox, oy, oz, vx, vy, vz, ta, tb)) return 1.0f;
    pass_majorant<COUNT>(S, M, cw, ox, oy, oz, vx, vy, vz, ta, tb, L, wk);
    float T = 1.0f, t = ta;
    int bin = 0;
    for (int drawn = 0; drawn < TB_MAX_TENT;) {
        int np = draw_points(ta, tb, L, t, bin, g);
        if (np == 0) break;
        drawn += np;
        if (COUNT) wk.tent += np;
        pass_density<COUNT>(S, M, cw, ox, oy, oz, vx, vy, vz, np, L, wk);
        for (int k = 0; k < np; ++k) T *= 1.0f - L.pk[k * TR_THREADS] / L.pm[k * TR_THREADS];
    }
    return T;
}

// Weighted delta tracking over [t0, t1] (null-collision form with signed
// collision weights; Woodcock tracking wherever 0 <= kappa <= kbar).
// Returns true on a real collision at *tc.
template <bool COUNT>
static __device__ bool delta_track(const SceneView& S, const MaskView& M, const CellW& cw, float ox, float oy,
                                   float oz, float vx, float vy, float vz, float t0, float t1, Rng& g, float* w,
                                   float* tc, const Lane& L, Work& wk) {
    float ta = t0, tb = t1;
    if (!clip_box(S, ox, oy, oz, vx, vy, vz, ta, tb)) return false;
    pass_majorant<COUNT>(S, M, cw, ox, oy, oz, vx, vy, vz, ta, tb, L, wk);
    float t = ta;
    int bin = 0;
    for (int drawn = 0; drawn < TB_MAX_TENT;) {
        int np = draw_points(ta, tb, L, t, bin, g);
        if (np == 0) return false;
        drawn += np;
        if (COUNT) wk.tent += np;
        pass_density<COUNT>(S, M, cw, ox, oy, oz, vx, vy, vz, np, L, wk);
        for (int k = 0; k < np; ++k) {
            float kap = L.pk[k * TR_THREADS], kb = L.pm[k * TR_THREADS];
            float xi = g.u();
            if (kap >= 0.0f && kap <= kb) {
                if (xi * kb < kap) {
                    *tc = L.pt[k * TR_THREADS];
                    return true;
                }
            } else {
                float kn = kb - kap;
                float Dn = fabsf(kap) + fabsf(kn);
                if (xi * Dn < fabsf(kap)) {
                    *w *= copysignf(Dn / kb, kap);
                    *tc = L.pt[k * TR_THREADS];
                    return true;
                }
                *w *= copysignf(Dn / kb, kn);
            }
        }
    }
    return false;
}

// per-lane LDS of a TR_THREADS-wide block
#define LANE_LDS                                                               \
    __shared__ int stk_all[TR_STACK * TR_THREADS];                             \
    __shared__ float fl_all[(TB_BINS + 3 * TB_PTS) * TR_THREADS];              \
    Lane L;                                                                    \
    L.stk = stk_all + threadIdx.x;                                             \
    L.bins = fl_all + threadIdx.x;                                             \
    L.pt = fl_all + TB_BINS * TR_THREADS + threadIdx.x;                        \
    L.pm = fl_all + (TB_BINS + TB_PTS) * TR_THREADS + threadIdx.x;             \
    L.pk = fl_all + (TB_BINS + 2 * TB_PTS) * TR_THREADS + threadIdx.x;

static __device__ __forceinline__ void sample_sphere(Rng& g, float* d) {
    float u1 = g.u(), u2 = g.u();
    float z = 1.0f - 2.0f * u1, sr = sqrtf(fmaxf(0.0f, 1.0f - z * z));
    float s, c;
    sincos2pi(u2 - 0.5f, &s, &c);  // phase 2 pi u2 shifted by pi: uniform either way
    d[0] = -sr * c;
    d[1] = -sr * s;
    d[2] = z;
}

// Henyey-Greenstein: cos(theta) by inverting its CDF; theta from the
// propagation direction, azimuth uniform.
static __device__ __forceinline__ void sample_hg(Rng& g, float gg, const float* wi, float* wo) {
    float u = g.u();
    float ct;
    if (fabsf(gg) < 1e-6f) {
        ct = 1.0f - 2.0f * u;
    } else {
        float sq = (1.0f - gg * gg) / (1.0f - gg + 2.0f * gg * u);
        ct = (1.0f + gg * gg - sq * sq) / (2.0f * gg);
        ct = fminf(1.0f, fmaxf(-1.0f, ct));
    }
    float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
    float sp, cp;
    sincos2pi(g.u() - 0.5f, &sp, &cp);
    float t[3];
    if (fabsf(wi[0]) > 0.5f) {
        t[0] = -wi[1]; t[1] = wi[0]; t[2] = 0.0f;
    } else {
        t[0] = 0.0f; t[1] = -wi[2]; t[2] = wi[1];
    }
    float tn = rsqrtf(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    t[0] *= tn; t[1] *= tn; t[2] *= tn;
    float b[3] = {wi[1] * t[2] - wi[2] * t[1], wi[2] * t[0] - wi[0] * t[2], wi[0] * t[1] - wi[1] * t[0]};
    for (int a = 0; a < 3; ++a) wo[a] = ct * wi[a] + st * (cp * t[a] + sp * b[a]);
}

static __device__ __forceinline__ int ray_of_tr(int gid, int n, int tile_w) {
    if (tile_w <= 0) return gid < n ? gid : -1;
    int lane = gid & 63, gw = gid >> 6;
    int tiles_x = tile_w >> 3, height = n / tile_w;
    int px = (gw % tiles_x) * 8 + (lane & 7), py = (gw / tiles_x) * 8 + (lane >> 3);
    return py < height ? py * tile_w + px : -1;
}

static __device__ __forceinline__ int64_t tr_threads(int n, int tile_w) {
    if (tile_w <= 0) return n;
    return (int64_t)(tile_w / 8) * ((n / tile_w + 7) / 8) * 64;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(TR_THREADS) void k_density(SceneView S, MaskView M, const float* __restrict__ pts, int n,
                                                        float* __restrict__ kappa, float* __restrict__ kbar) {
    __shared__ int stk[TR_STACK * TR_THREADS];
    int i = blockIdx.x * TR_THREADS + threadIdx.x;
    if (i >= n) return;
    CellW cw;
    fixed_weights(M, cw);
    float x = pts[3 * (size_t)i], y = pts[3 * (size_t)i + 1], z = pts[3 * (size_t)i + 2];
    Work wk{};
    kappa[i] = point_density<false>(S, M, cw, x, y, z, stk + threadIdx.x, wk);
    if (kbar) {
        float kb = 0.0f;
        if (x >= S.glo[0] && x <= S.ghi[0] && y >= S.glo[1] && y <= S.ghi[1] && z >= S.glo[2] && z <= S.ghi[2]) {
            int ix = min(S.G - 1, max(0, (int)floorf((x - S.glo[0]) * S.ginv[0])));
            int iy = min(S.G - 1, max(0, (int)floorf((y - S.glo[1]) * S.ginv[1])));
            int iz = min(S.G - 1, max(0, (int)floorf((z - S.glo[2]) * S.ginv[2])));
            kb = voxel_majorant(S, (iz * S.G + iy) * S.G + ix, cw.mw);
        }
        kbar[i] = kb;
    }
}

__global__ __launch_bounds__(TR_THREADS) void k_ratio(SceneView S, MaskView M, const float* __restrict__ rays, int n,
                                                      int tile_w, int spp, uint64_t seed, float* __restrict__ Tm,
                                                      float* __restrict__ Tv) {
    LANE_LDS
    int gid = blockIdx.x * TR_THREADS + threadIdx.x;
    int idx = ray_of_tr(gid, n, tile_w);
    if (idx < 0) return;
    const float* r = rays + (size_t)idx * 8;
    CellW cw;
    fixed_weights(M, cw);
    float s1 = 0.0f, s2 = 0.0f;
    Work wk{};
    for (int s = 0; s < spp; ++s) {
        Rng g;
        g.init(seed, (uint32_t)idx, (uint32_t)s, 1u);
        float T = ratio_track<false>(S, M, cw, r[0], r[1], r[2], r[3], r[4], r[5], r[6], r[7], g, L, wk);
        s1 += T;
        s2 += T * T;
    }
    Tm[idx] = s1 / spp;
    if (Tv) Tv[idx] = spp > 1 ? fmaxf(0.0f, (s2 - s1 * s1 / spp) / (spp - 1)) : 0.0f;
}

struct RenderArgs {
    int spp, multiple, max_scatter, stochastic;
    float albedo, hg, env;
    uint64_t seed;
};

// All samples of one ray; random streams keyed by (seed, key, sample).
template <bool COUNT>
static __device__ void render_ray(const SceneView& S, const MaskView& M, const RenderArgs& A, const float* r,
                                  uint32_t key, const Lane& ln, float* Lmean, float* Lvar, float* Tmean, float* Tvar,
                                  Work& wk) {
    CellW fixed;
    fixed_weights(M, fixed);
    float s1 = 0.0f, s2 = 0.0f, q1 = 0.0f, q2 = 0.0f;
    for (int s = 0; s < A.spp; ++s) {
        Rng g, gT;
        g.init(A.seed, key, (uint32_t)s, 0u);
        gT.init(A.seed, key, (uint32_t)s, 1u);
        float ox = r[0], oy = r[1], oz = r[2], vx = r[3], vy = r[4], vz = r[5], t0 = r[6], t1 = r[7];
        float w = 1.0f, L = 0.0f, Tp = 1.0f;
        int nsc = 0;
        for (int seg = 0;; ++seg) {
            CellW cw = fixed;
            if (A.stochastic) stochastic_weights(S, vx, vy, vz, g, cw);
            if (seg == 0) Tp = ratio_track<COUNT>(S, M, cw, ox, oy, oz, vx, vy, vz, t0, t1, gT, ln, wk);
            float tc;
            if (!delta_track<COUNT>(S, M, cw, ox, oy, oz, vx, vy, vz, t0, t1, g, &w, &tc, ln, wk)) {
                L += w * A.env;
                break;
            }
            float x = ox + tc * vx, y = oy + tc * vy, z = oz + tc * vz;
            if (!A.multiple) {
                float d[3];
                sample_sphere(g, d);
                L += w * A.albedo *
                     ratio_track<COUNT>(S, M, cw, x, y, z, d[0], d[1], d[2], 0.0f, INFINITY, g, ln, wk) * A.env;
                break;
            }
            if (nsc >= A.max_scatter) break;
            ++nsc;
            w *= A.albedo;
            float vn = rsqrtf(vx * vx + vy * vy + vz * vz);
            float wi[3] = {vx * vn, vy * vn, vz * vn}, wo[3];
            sample_hg(g, A.hg, wi, wo);
            ox = x; oy = y; oz = z;
            vx = wo[0]; vy = wo[1]; vz = wo[2];
            t0 = 0.0f;
            t1 = INFINITY;
        }
        s1 += L;
        s2 += L * L;
        q1 += Tp;
        q2 += Tp * Tp;
    }
    float inv = 1.0f / A.spp;
    *Lmean = s1 * inv;
    *Lvar = A.spp > 1 ? fmaxf(0.0f, (s2 - s1 * s1 * inv) / (A.spp - 1)) : 0.0f;
    *Tmean = q1 * inv;
    *Tvar = A.spp > 1 ? fmaxf(0.0f, (q2 - q1 * q1 * inv) / (A.spp - 1)) : 0.0f;
}

template <bool COUNT>
__global__ __launch_bounds__(TR_THREADS) void k_render(SceneView S, MaskView M, const float* __restrict__ rays, int n,
                                                       int tile_w, RenderArgs A, float* __restrict__ Lm,
                                                       float* __restrict__ Lv, float* __restrict__ Tm,
                                                       float* __restrict__ Tv,
                                                       unsigned long long* __restrict__ counters) {
    LANE_LDS
    int gid = blockIdx.x * TR_THREADS + threadIdx.x;
    int idx = ray_of_tr(gid, n, tile_w);
    if (idx < 0) return;
    float a, b, c, d;
    Work wk{};
    render_ray<COUNT>(S, M, A, rays + (size_t)idx * 8, (uint32_t)idx, L, &a, &b, &c, &d, wk);
    if (COUNT) {
        atomicAdd(counters + 0, wk.tent);
        atomicAdd(counters + 1, wk.nodes);
        atomicAdd(counters + 2, wk.prims);
        atomicAdd(counters + 3, wk.voxels);
        return;
    }
    Lm[idx] = a;
    if (Lv) Lv[idx] = b;
    if (Tm) Tm[idx] = c;
    if (Tv) Tv[idx] = d;
}

// Serving: one launch renders tiles of many requests (each tile a contiguous
// range of one request's rays).  A request's random streams are keyed by its
// own seed and pixel index, so its image does not depend on the batch.
struct ServeReq {
    SceneView S;
    MaskView M;
    RenderArgs A;
    const float* rays;
    float* out;
    int n;
};

struct ServeTile {
    int req, first, count, pad;
};

__global__ __launch_bounds__(TR_THREADS) void k_render_tiles(const ServeReq* __restrict__ reqs,
                                                             const ServeTile* __restrict__ tiles, int blocks_per_tile) {
    LANE_LDS
    const ServeTile tl = tiles[blockIdx.x / blocks_per_tile];
    int local = (blockIdx.x % blocks_per_tile) * TR_THREADS + threadIdx.x;
    if (local >= tl.count) return;
    const ServeReq& R = reqs[tl.req];
    int idx = tl.first + local;
    float a, b, c, d;
    Work wk{};
    render_ray<false>(R.S, R.M, R.A, R.rays + (size_t)idx * 8, (uint32_t)idx, L, &a, &b, &c, &d, wk);
    R.out[idx] = a;
}

gf_status gf_serve_fill_req(const gf_request* q, const float* rays, void* out_desc) {
    ServeReq* d = (ServeReq*)out_desc;
    d->S = gf_scene_view(q->scene);
    d->M = gf_mask_view(q->render.mask);
    d->A.spp = q->render.spp;
    d->A.multiple = q->render.multiple;
    d->A.max_scatter = q->render.max_scatter;
    d->A.stochastic = q->render.stochastic;
    d->A.albedo = q->render.albedo;
    d->A.hg = q->render.hg_g;
    d->A.env = q->render.env;
    d->A.seed = q->render.seed;
    d->rays = rays;
    d->out = q->out;
    d->n = q->camera.width * q->camera.height;
    return GF_OK;
}

size_t gf_serve_req_size() { return sizeof(ServeReq); }
size_t gf_serve_tile_size() { return sizeof(ServeTile); }
int gf_serve_tile_threads() { return TR_THREADS; }

gf_status gf_serve_launch(const void* dreqs, const void* dtiles, int ntiles, int tile_rays, hipStream_t sm) {
    int bpt = (tile_rays + TR_THREADS - 1) / TR_THREADS;
    k_render_tiles<<<(unsigned)(ntiles * bpt), TR_THREADS, 0, sm>>>((const ServeReq*)dreqs, (const ServeTile*)dtiles,
                                                                    bpt);
    GF_HIP(hipGetLastError());
    return GF_OK;
}

__global__ __launch_bounds__(256) void k_camera(gf_camera cam, float fx, float fy, float fz, float rx, float ry,
                                                float rz, float ux, float uy, float uz, float th,
                                                float* __restrict__ rays) {
    int i = blockIdx.x * 256 + threadIdx.x;
    int W = cam.width, H = cam.height;
    if (i >= W * H) return;
    int px = i % W, py = i / W;
    float* o = rays + (size_t)i * 8;
    if (cam.kind == 0) {
        o[0] = (px + 0.5f) / W;
        o[1] = (py + 0.5f) / H;
        o[2] = cam.eye[2];
        o[3] = 0.0f;
        o[4] = 0.0f;
        o[5] = 1.0f;
    } else {
        float aspect = (float)W / H;
        float sx = (2.0f * (px + 0.5f) / W - 1.0f) * th * aspect;
        float sy = (1.0f - 2.0f * (py + 0.5f) / H) * th;
        float dx = fx + sx * rx + sy * ux, dy = fy + sx * ry + sy * uy, dz = fz + sx * rz + sy * uz;
        float inv = rsqrtf(dx * dx + dy * dy + dz * dz);
        o[0] = cam.eye[0];
        o[1] = cam.eye[1];
        o[2] = cam.eye[2];
        o[3] = dx * inv;
        o[4] = dy * inv;
        o[5] = dz * inv;
    }
    o[6] = 0.0f;
    o[7] = INFINITY;
}

// ---------------------------------------------------------------------------
// host entry points
// ---------------------------------------------------------------------------
static gf_status check_depth(const gf_scene_s* s, const char* who) {
    if (s->depth > TR_STACK) return gf_fail(GF_EINVAL, "%s: LBVH depth %d exceeds the point-query stack", who, s->depth);
    return GF_OK;
}

static unsigned tr_blocks(int64_t n, int tile_w) {
    int64_t t = tile_w <= 0 ? n : (int64_t)(tile_w / 8) * ((n / tile_w + 7) / 8) * 64;
    return (unsigned)((t + TR_THREADS - 1) / TR_THREADS);
}

static gf_status check_rays_tr(int64_t n, int tile_w, const char* who) {
    if (n < 0 || n > (int64_t)INT32_MAX / 8) return gf_fail(GF_EINVAL, "%s: ray count out of range", who);
    if (tile_w < 0 || (tile_w > 0 && (tile_w % 8 != 0 || n % tile_w != 0)))
        return gf_fail(GF_EINVAL, "%s: image_width must be a multiple of 8 dividing n", who);
    return GF_OK;
}

extern "C" gf_status gf_density(gf_scene s, const float* pts, int64_t n, gf_mask mask, float* kappa, float* kbar,
                                void* stream) {
    if (!s || (n && (!pts || !kappa))) return gf_fail(GF_EINVAL, "gf_density: NULL argument");
    if (n < 0 || n > INT32_MAX / 3) return gf_fail(GF_EINVAL, "gf_density: n out of range");
    gf_status st = check_depth(s, "gf_density");
    if (st != GF_OK || n == 0) return st;
    k_density<<<(unsigned)((n + TR_THREADS - 1) / TR_THREADS), TR_THREADS, 0, (hipStream_t)stream>>>(
        gf_scene_view(s), gf_mask_view(mask), pts, (int)n, kappa, kbar);
    GF_HIP(hipGetLastError());
    return GF_OK;
}

extern "C" gf_status gf_transmittance_ratio(gf_scene s, const float* rays, int64_t n, int image_width, gf_mask mask,
                                            int spp, uint64_t seed, float* T_mean, float* T_var, void* stream) {
    if (!s || (n && (!rays || !T_mean))) return gf_fail(GF_EINVAL, "gf_transmittance_ratio: NULL argument");
    if (spp < 1) return gf_fail(GF_EINVAL, "gf_transmittance_ratio: spp must be >= 1");
    gf_status st = check_rays_tr(n, image_width, "gf_transmittance_ratio");
    if (st == GF_OK) st = check_depth(s, "gf_transmittance_ratio");
    if (st != GF_OK || n == 0) return st;
    k_ratio<<<tr_blocks(n, image_width), TR_THREADS, 0, (hipStream_t)stream>>>(
        gf_scene_view(s), gf_mask_view(mask), rays, (int)n, image_width, spp, seed, T_mean, T_var);
    GF_HIP(hipGetLastError());
    return GF_OK;
}

gf_status gf_render_launch(gf_scene s, const float* rays, int64_t n, int image_width, const gf_render_desc* d,
                           float* L_mean, float* L_var, float* T_mean, float* T_var, hipStream_t sm,
                           unsigned long long* counters) {
    RenderArgs A;
    A.spp = d->spp;
    A.multiple = d->multiple;
    A.max_scatter = d->max_scatter;
    A.stochastic = d->stochastic;
    A.albedo = d->albedo;
    A.hg = d->hg_g;
    A.env = d->env;
    A.seed = d->seed;
    if (counters)
        k_render<true><<<tr_blocks(n, image_width), TR_THREADS, 0, sm>>>(
            gf_scene_view(s), gf_mask_view(d->mask), rays, (int)n, image_width, A, nullptr, nullptr, nullptr, nullptr,
            counters);
    else
        k_render<false><<<tr_blocks(n, image_width), TR_THREADS, 0, sm>>>(
            gf_scene_view(s), gf_mask_view(d->mask), rays, (int)n, image_width, A, L_mean, L_var, T_mean, T_var,
            nullptr);
    GF_HIP(hipGetLastError());
    return GF_OK;
}

gf_status gf_check_render_desc(const gf_render_desc* d, const char* who) {
    if (!d) return gf_fail(GF_EINVAL, "%s: NULL desc", who);
    if (d->spp < 1 || d->max_scatter < 0) return gf_fail(GF_EINVAL, "%s: spp >= 1 and max_scatter >= 0 required", who);
    if (!isfinite(d->albedo) || !isfinite(d->hg_g) || !(fabsf(d->hg_g) < 1.0f) || !isfinite(d->env))
        return gf_fail(GF_EINVAL, "%s: albedo / hg_g / env invalid", who);
    return GF_OK;
}

extern "C" gf_status gf_render(gf_scene s, const float* rays, int64_t n, int image_width, const gf_render_desc* d,
                               float* L_mean, float* L_var, float* T_mean, float* T_var, void* stream) {
    if (!s || (n && (!rays || !L_mean))) return gf_fail(GF_EINVAL, "gf_render: NULL argument");
    gf_status st = gf_check_render_desc(d, "gf_render");
    if (st == GF_OK) st = check_rays_tr(n, image_width, "gf_render");
    if (st == GF_OK) st = check_depth(s, "gf_render");
    if (st != GF_OK || n == 0) return st;
    return gf_render_launch(s, rays, n, image_width, d, L_mean, L_var, T_mean, T_var, (hipStream_t)stream, nullptr);
}

extern "C" gf_status gf_render_counts(gf_scene s, const float* rays, int64_t n, int image_width,
                                      const gf_render_desc* d, uint64_t* counts, void* stream) {
    if (!s || !counts || (n && !rays)) return gf_fail(GF_EINVAL, "gf_render_counts: NULL argument");
    gf_status st = gf_check_render_desc(d, "gf_render_counts");
    if (st == GF_OK) st = check_rays_tr(n, image_width, "gf_render_counts");
    if (st == GF_OK) st = check_depth(s, "gf_render_counts");
    if (st != GF_OK) return st;
    hipStream_t sm = (hipStream_t)stream;
    GF_HIP(hipMemsetAsync(counts, 0, 4 * sizeof(uint64_t), sm));
    if (n == 0) return GF_OK;
    return gf_render_launch(s, rays, n, image_width, d, nullptr, nullptr, nullptr, nullptr, sm,
                            (unsigned long long*)counts);
}

gf_status gf_camera_launch(const gf_camera* cam, float* rays, hipStream_t sm) {
    double f[3] = {0, 0, 1}, rt[3] = {1, 0, 0}, up[3] = {0, 1, 0};
    if (cam->kind == 1) {
        for (int a = 0; a < 3; ++a) f[a] = (double)cam->target[a] - cam->eye[a];
        double fn = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        for (int a = 0; a < 3; ++a) f[a] /= fn;
        double u[3] = {cam->up[0], cam->up[1], cam->up[2]};
        rt[0] = u[1] * f[2] - u[2] * f[1];
        rt[1] = u[2] * f[0] - u[0] * f[2];
        rt[2] = u[0] * f[1] - u[1] * f[0];
        double rn = sqrt(rt[0] * rt[0] + rt[1] * rt[1] + rt[2] * rt[2]);
        for (int a = 0; a < 3; ++a) rt[a] /= rn;
        up[0] = f[1] * rt[2] - f[2] * rt[1];
        up[1] = f[2] * rt[0] - f[0] * rt[2];
        up[2] = f[0] * rt[1] - f[1] * rt[0];
    }
    float th = (float)tan(cam->fov_y_deg * GF_PI / 360.0);
    int64_t n = (int64_t)cam->width * cam->height;
    k_camera<<<(unsigned)((n + 255) / 256), 256, 0, sm>>>(*cam, (float)f[0], (float)f[1], (float)f[2], (float)rt[0],
                                                         (float)rt[1], (float)rt[2], (float)up[0], (float)up[1],
                                                         (float)up[2], th, rays);
    GF_HIP(hipGetLastError());
    return GF_OK;
}

gf_status gf_check_camera(const gf_camera* cam, const char* who) {
    if (!cam) return gf_fail(GF_EINVAL, "%s: NULL camera", who);
    if (cam->width < 1 || cam->height < 1 || (int64_t)cam->width * cam->height > (int64_t)INT32_MAX / 8)
        return gf_fail(GF_EINVAL, "%s: bad camera size", who);
    if (cam->kind != 0 && cam->kind != 1) return gf_fail(GF_EINVAL, "%s: camera kind must be 0 or 1", who);
    if (cam->kind == 1) {
        double f[3];
        for (int a = 0; a < 3; ++a) f[a] = (double)cam->target[a] - cam->eye[a];
        if (!(f[0] * f[0] + f[1] * f[1] + f[2] * f[2] > 0.0) || !(cam->fov_y_deg > 0.0f && cam->fov_y_deg < 179.0f))
            return gf_fail(GF_EINVAL, "%s: degenerate pinhole camera", who);
    }
    return GF_OK;
}

extern "C" gf_status gf_camera_rays(const gf_camera* cam, float* rays, void* stream) {
    gf_status st = gf_check_camera(cam, "gf_camera_rays");
    if (st != GF_OK) return st;
    if (!rays) return gf_fail(GF_EINVAL, "gf_camera_rays: NULL rays");
    return gf_camera_launch(cam, rays, (hipStream_t)stream);
}
